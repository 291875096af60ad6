"""Edge cases of the library against the oracle (needs an MI355X): the
smallest and largest chain counts per fold, the largest number of shuffle
blocks, a fold that trains on a single row, zero-transition steps and the
error paths before enough draws exist."""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import diagnostics, sampler
from paper_2310_07002_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _with_L(w, L, seed):
    """w with L chains per fold, starting at the truth plus seeded noise of
    the inverse-mass scale (input generation only)."""
    rng = np.random.default_rng(seed)
    init = w.truth[None, :] + np.sqrt(w.inv_mass)[None, :] * rng.standard_normal((w.K * L, w.d))
    return dataclasses.replace(w, L=L, init_pos=init)


def _replay(w, n_iter, prec=None):
    s = binding.PCV.from_workload(w, precision=prec)
    s.step(n_iter)
    th, _, sv = s.get_state()
    acc = s.get_accumulators(w.n_blocks)
    run = sampler.run_all(w, n_iter=n_iter)
    return s, th, sv, acc, run


@pytest.mark.parametrize("name,folds_,L", [("c1", (0, 6), 2), ("c1", (0, 6), 64),
                                           ("c3", (0, 3), 2), ("c3", (0, 3), 64)])
def test_chains_per_fold_extremes_replay_the_oracle(dev, name, folds_, L):
    """L = 2 (the fewest chains R-hat allows) and L = 64 (the most) on the
    fused (c1) and row-split (c3) fp64 paths: 60 transitions replay the
    oracle accept for accept, with equal accumulators and diagnostics."""
    w = W.fold_subset(W.make(name), *folds_)
    w = dataclasses.replace(_with_L(w, L, seed=L), n_warmup=10, n_samples=50, batch_size=10, n_blocks=5)
    _say(f"[edge L] {name} K={w.K} L={L} C={w.C}")
    s, th, sv, acc, run = _replay(w, 60)
    np.testing.assert_allclose(th, run.state.q, rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(sv, run.state.s, rtol=1e-10, atol=1e-11)
    np.testing.assert_array_equal(acc["n_accept"], run.acc.n_accept)
    for key in ("U", "U2", "V", "V2"):
        np.testing.assert_allclose(acc[key], getattr(run.acc, key), rtol=1e-10, atol=1e-12)
    d = s.diagnostics()
    o = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    np.testing.assert_allclose(d["rhat_fold"], o["rhat_fold"], rtol=1e-9)
    assert d["elpd"] == pytest.approx(o["elpd"], rel=1e-10)
    s.close()


def test_sixty_four_shuffle_blocks(dev):
    """D = 64 shuffle blocks of one draw each (b = G = 1), the largest block
    count: per-block Welford states and the block-shuffle replicates equal
    the oracle's."""
    w = W.fold_subset(W.make("c1"), 0, 10)
    w = dataclasses.replace(w, n_warmup=5, n_samples=64, batch_size=1, n_blocks=64)
    assert w.batches_per_block == 1
    s, th, sv, acc, run = _replay(w, 5 + 64)
    np.testing.assert_array_equal(acc["n_accept"], run.acc.n_accept)
    np.testing.assert_allclose(acc["blk_mean"], run.acc.blk_mean, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(acc["blk_m2"], run.acc.blk_m2, rtol=1e-9, atol=1e-12)
    rep_g = s.shuffle_benchmark(20, seed=9)
    _, rep_o = diagnostics.shuffle_benchmark(run.acc, w.K, w.L, w.n_blocks, 20, seed=9)
    np.testing.assert_allclose(rep_g, rep_o, rtol=1e-9)
    s.close()


def test_fold_training_on_a_single_row(dev):
    """LOO on two rows: each fold's posterior rests on one training row (the
    smallest training set), yet chains, accumulators and elpd replay the
    oracle."""
    base = W.make("c1")
    keep = 2
    w = dataclasses.replace(base, X=base.X[:keep].copy(), y=base.y[:keep].copy(), K=keep,
                            fold_index=np.arange(keep, dtype=np.int32),
                            init_pos=base.init_pos[:keep * base.L].copy(),
                            n_warmup=20, n_samples=100, batch_size=20)
    s, th, sv, acc, run = _replay(w, 120)
    np.testing.assert_allclose(th, run.state.q, rtol=1e-10, atol=1e-11)
    np.testing.assert_array_equal(acc["n_accept"], run.acc.n_accept)
    o = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    assert s.elpd()["elpd"] == pytest.approx(o["elpd"], rel=1e-10)
    s.close()


def test_zero_transitions_and_early_results(dev):
    """pcv_step(0) changes nothing; diagnostics, elpd and the shuffle
    benchmark refuse (PCV_ERR_STATE) until their draws exist; a negative
    transition count is an invalid argument."""
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 5), n_warmup=3)
    s = binding.PCV.from_workload(w)
    before = s.get_state()
    s.step(0)
    for x, y in zip(before, s.get_state()):
        np.testing.assert_array_equal(x, y)

    def status(fn):
        with pytest.raises(binding.PcvError) as e:
            fn()
        return e.value.status

    assert status(s.diagnostics) == 4
    assert status(s.elpd) == 4
    assert status(lambda: s.shuffle_benchmark(4, seed=1)) == 4
    assert status(lambda: s.step(-1)) == 1
    s.step(4)                      # warm-up done, one post-warm-up draw
    assert status(s.diagnostics) == 4
    e = s.elpd()
    assert np.isfinite(e["elpd"])
    s.step(1)                      # two draws: R-hat defined, batch-means MCSE not yet
    d = s.diagnostics()
    assert np.isfinite(d["rhat_max"]) and math.isnan(d["ess"])
    s.close()
