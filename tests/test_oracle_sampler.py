"""Pins of the oracle's online accumulators and diagnostics (CPU only)."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

from oracle import closed_form, diagnostics, folds, sampler
from paper_2310_07002_amd import workloads as W


@pytest.fixture(scope="module")
def c1_run():
    w = W.make_c1()
    run = sampler.run_all(w, store_draws=True)
    return w, run


def test_online_accumulators_equal_two_pass(c1_run):
    w, run = c1_run
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    tp = diagnostics.two_pass(run.draws, w.K, w.L, w.batch_size)
    for key in ("elpd_fold", "rhat_fold", "mcse_fold", "ess_fold", "sigma2_rel_fold", "s2_rel_fold"):
        np.testing.assert_allclose(on[key], tp[key], rtol=1e-10, err_msg=key)
    assert abs(on["elpd"] - tp["elpd"]) < 1e-10 * abs(tp["elpd"])


def test_partial_batch_is_in_elpd_but_not_batch_means():
    w = dataclasses.replace(W.make_c1(), n_warmup=5)
    w = W.fold_subset(w, 0, 6)
    run = sampler.run_all(w, n_iter=5 + 73, store_draws=True)    # 73 = one batch + 23
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    tp = diagnostics.two_pass(run.draws, w.K, w.L, w.batch_size)
    np.testing.assert_allclose(on["elpd_fold"], tp["elpd_fold"], rtol=1e-12)
    np.testing.assert_allclose(on["rhat_fold"], tp["rhat_fold"], rtol=1e-10)
    assert run.acc.n_draws == 73


def test_elpd_within_mcse_of_closed_form(c1_run):
    w, run = c1_run
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    roles = folds.roles_of(w)
    exact = np.array([closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale,
                                             roles[k] == 1, roles[k] == 2)["elpd"]
                      for k in range(w.K)])
    assert abs(on["elpd"] - exact.sum()) < 4 * on["mcse"]
    z = (on["elpd_fold"] - exact) / on["mcse_fold"]
    assert abs(z.mean()) < 4 / math.sqrt(w.K)
    assert 0.7 < z.std() < 1.4


def test_log_pred_mean_matches_closed_form(c1_run):
    w, run = c1_run
    n, mean, m2 = diagnostics.merge_blocks(run.acc.blk_n, run.acc.blk_mean, run.acc.blk_m2)
    roles = folds.roles_of(w)
    zs = []
    for k in range(0, w.K, 5):
        ex = closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1, roles[k] == 2)
        fold_mean = mean[k * w.L:(k + 1) * w.L].mean()
        se = math.sqrt(ex["Vars"] / (w.L * run.acc.n_draws)) * 3.0   # generous autocorrelation allowance
        zs.append((fold_mean - ex["Es"]) / se)
    assert np.max(np.abs(zs)) < 4.0


def test_rhat_on_iid_draws_follows_f_distribution():
    """For iid normal draws B/W ~ F(L-1, L(N-1)), so Rhat^2 = (N-1)/N + F/N."""
    K, L, N, b, D = 400, 4, 200, 20, 5
    rng = np.random.default_rng(9)
    draws = rng.normal(size=(K * L, N)) * 0.3 - 2.0
    acc = sampler.Accumulators.empty(K * L, D)
    for i in range(N):
        sampler.accumulate(acc, draws[:, i], i, b, N // (b * D), D)
    out = diagnostics.from_accumulators(acc, K, L, b)
    F = (out["rhat_fold"] ** 2 - (N - 1) / N) * N
    assert stats.kstest(F, stats.f(L - 1, L * (N - 1)).cdf).pvalue > 1e-3


def test_rhat_max_flags_stuck_and_shifted_chains():
    """Section 4.2 / Fig. 5: a stuck or shifted chain pushes Rhat_max above the
    block-shuffle benchmark."""
    K, L, N, b, D = 20, 4, 1000, 50, 5
    G = N // (b * D)
    rng = np.random.default_rng(10)
    phi = 0.5
    e = rng.normal(size=(K * L, N))
    draws = np.empty_like(e)
    draws[:, 0] = e[:, 0]
    for i in range(1, N):
        draws[:, i] = phi * draws[:, i - 1] + math.sqrt(1 - phi ** 2) * e[:, i]

    def rhat_and_bench(x):
        acc = sampler.Accumulators.empty(K * L, D)
        for i in range(N):
            sampler.accumulate(acc, x[:, i], i, b, G, D)
        out = diagnostics.from_accumulators(acc, K, L, b)
        _, rep = diagnostics.shuffle_benchmark(acc, K, L, D, 100, seed=1)
        return out["rhat_max"], rep

    ok, rep = rhat_and_bench(draws)
    assert ok <= np.quantile(rep, 0.999) + 0.05
    stuck = draws.copy()
    stuck[5] = 1.5            # the chain never leaves its first draw, 1.5 sd from the mean
    r_stuck, rep_stuck = rhat_and_bench(stuck)
    assert r_stuck > rep_stuck.max()
    shifted = draws.copy()
    shifted[9] += 5.0
    r_shift, rep_shift = rhat_and_bench(shifted)
    assert r_shift > rep_shift.max()


def test_fold_subset_replays_the_same_chains():
    w = dataclasses.replace(W.make_c1(), n_warmup=3)
    full = sampler.run_all(w, n_iter=8, store_draws=True)
    sub = sampler.run_all(W.fold_subset(w, 10, 14), n_iter=8, store_draws=True)
    np.testing.assert_array_equal(sub.state.q, full.state.q[10 * w.L:14 * w.L])
    np.testing.assert_array_equal(sub.draws, full.draws[10 * w.L:14 * w.L])


def test_shifted_sums_mode_matches_welford_and_two_pass():
    """Algorithm A2's shifted sums: C_k is the mean of the fold's L*N_wu
    warm-up draws, each block keeps sum (s - C_k) and sum (s - C_k)^2, and
    Rhat and its block-shuffle benchmark equal the Welford and two-pass
    values on the same draws (the shift cancels)."""
    w = W.fold_subset(dataclasses.replace(W.make_c1(), n_warmup=40, rhat_mode=1), 0, 10)
    b, G, D = w.batch_size, w.batches_per_block, w.n_blocks
    run = sampler.start(w)
    wu = []
    for _ in range(w.n_warmup):
        sampler.advance(w, run, 1)
        wu.append(run.state.s.copy())
    wu = np.stack(wu, axis=1).reshape(w.K, w.L * w.n_warmup)
    np.testing.assert_allclose(run.acc.center, np.repeat(wu.mean(axis=1), w.L), rtol=1e-13)
    N = 237                                        # blocks of G*b = 200 draws: one full, one partial
    sampler.advance(w, run, N, store_draws=True)
    y = run.draws - run.acc.center[:, None]
    for dd in range(D):
        seg = y[:, dd * G * b:(dd + 1) * G * b] if dd < D - 1 else y[:, dd * G * b:]
        np.testing.assert_allclose(run.acc.blk_mean[:, dd], seg.sum(axis=1), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(run.acc.blk_m2[:, dd], (seg * seg).sum(axis=1), rtol=1e-11, atol=1e-11)
    wf = sampler.run_all(dataclasses.replace(w, rhat_mode=0), n_iter=w.n_warmup + N)
    np.testing.assert_array_equal(wf.state.s, run.state.s)
    on_s = diagnostics.from_accumulators(run.acc, w.K, w.L, b)
    on_w = diagnostics.from_accumulators(wf.acc, w.K, w.L, b)
    tp = diagnostics.two_pass(run.draws, w.K, w.L, b)
    np.testing.assert_allclose(on_s["rhat_fold"], on_w["rhat_fold"], rtol=1e-10)
    np.testing.assert_allclose(on_s["rhat_fold"], tp["rhat_fold"], rtol=1e-10)
    _, rep_s = diagnostics.shuffle_benchmark(run.acc, w.K, w.L, D, 20, seed=3)
    _, rep_w = diagnostics.shuffle_benchmark(wf.acc, w.K, w.L, D, 20, seed=3)
    np.testing.assert_allclose(rep_s, rep_w, rtol=1e-9)


def test_hvblock_elpd_within_mcse_of_closed_form():
    """hv-block folds (v = 5 test rows, h = 10 excluded on each side) of the
    conjugate AR(4) regression: the oracle's run on 6 folds (100 warm-up and
    600 sampling transitions) lies within Monte Carlo error of the exact joint
    predictive density of each fold's test block (Section 2, hv-block CV;
    Gaussian closed form)."""
    w = dataclasses.replace(W.fold_subset(W.make_c3(), 100, 106), n_warmup=100, n_samples=600)
    run = sampler.run_all(w)
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    roles = folds.roles_of(w)
    assert np.all((roles == folds.ROLE_TEST).sum(axis=1) == 5)
    assert np.all((roles == folds.ROLE_EXCLUDED).sum(axis=1) == 20)
    exact = np.array([closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale,
                                             roles[k] == 1, roles[k] == 2)["elpd"]
                      for k in range(w.K)])
    assert abs(on["elpd"] - exact.sum()) < 4 * on["mcse"]
    z = (on["elpd_fold"] - exact) / on["mcse_fold"]
    assert np.max(np.abs(z)) < 4.5
