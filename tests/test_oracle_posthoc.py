"""Pins of the post-hoc diagnostics on stored draws (CPU only)."""
import numpy as np

from oracle import diagnostics, posthoc, sampler
from paper_2310_07002_amd import workloads as W


def test_rank_rhat_is_invariant_to_monotone_maps():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(4, 301)) + np.array([[0.0], [0.1], [0.0], [0.3]])
    r = posthoc.rank_rhat(x)
    assert r == posthoc.rank_rhat(2.0 * x + 3.0) == posthoc.rank_rhat(np.exp(x))
    # ties: a constant shift of all draws keeps every rank
    assert posthoc.rank_rhat(np.round(x, 1)) == posthoc.rank_rhat(np.round(x, 1) + 7.0)


def test_split_rhat_detects_a_drifting_chain():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4, 1000))
    assert abs(posthoc.split_rhat(x) - 1.0) < 0.01
    assert abs(posthoc.rhat_chains(x) - 1.0) < 0.01
    drift = x.copy()
    drift[2] += np.linspace(-1.5, 1.5, 1000)          # same chain mean, trending within
    assert posthoc.rhat_chains(drift) < 1.02 < posthoc.split_rhat(drift)
    assert posthoc.rank_rhat(drift) > 1.02


def test_stored_draws_reproduce_the_online_estimates():
    w = W.fold_subset(W.make_c1(), 0, 20)
    run = sampler.run_all(w, n_iter=w.n_warmup + 400, store_draws=True)
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    ph = posthoc.fold_rhats(run.draws, w.K, w.L)
    np.testing.assert_allclose(ph["rhat_fold"], on["rhat_fold"], rtol=1e-10)
    assert ph["split_rhat_max"] < 1.1 and ph["rank_rhat_max"] < 1.1
