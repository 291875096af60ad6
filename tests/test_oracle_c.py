"""Pins of the plain C oracle (oracle/c/pcv_oracle.c), CPU only.

The C oracle is pinned on its own (published Philox vectors, central finite
differences of its log density, the conjugate Gaussian's exact gradient and
exact elpd) and held to the numpy oracle: the same masked log density, the
same HMC trajectories accept for accept, the same accumulators and the same
diagnostics.  Two independent restatements of the method agreeing to
rounding is the check that neither carries a transcription slip."""
import dataclasses
import os

import numpy as np
import pytest

from oracle import c_oracle, closed_form, diagnostics, folds, model, sampler
from paper_2310_07002_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


@pytest.fixture(scope="module", autouse=True)
def built():
    c_oracle.build()
    c_oracle._lib = None


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            words = [int(t, 16) for t in line.split()]
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    seed = key[0] | (key[1] << 32)
    assert [int(v) for v in c_oracle.philox(seed, *ctr)] == expect


def _small(family, groups=0, n=40, p=3, K=4, L=2, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, p))
    if family in (model.GAUSSIAN, model.HIER_GAUSSIAN):
        y = rng.normal(size=n)
    elif family == model.POISSON:
        y = rng.poisson(1.5, size=n).astype(float)
    else:
        y = (rng.random(n) < 0.5).astype(float)
    fold_index = (np.arange(n) % K).astype(np.int32)
    group_of = None
    if groups:
        group_of = np.sort(rng.integers(0, groups, size=n)).astype(np.int32)
        fold_index = group_of.copy()
        K = groups
    w = W.Workload(name="small", family=family, precision=0, X=X, y=y, K=K, L=L, fold_kind=W.FOLDS_INDEX,
                   fold_index=fold_index, group_of=group_of, n_groups=groups, sigma=0.8)
    w.prior_scale = rng.uniform(0.5, 2.0, size=w.d)
    w.inv_mass = np.ones(w.d)
    return w


@pytest.mark.parametrize("family,groups", [(model.GAUSSIAN, 0), (model.LOGISTIC, 0), (model.POISSON, 0),
                                           (model.HIER_LOGISTIC, 5), (model.HIER_GAUSSIAN, 5)])
def test_gradient_matches_central_differences(family, groups):
    w = _small(family, groups)
    theta = 0.3 * np.random.default_rng(1).normal(size=(w.C, w.d))
    _, g, _ = c_oracle.log_density_grad(w, theta)
    h = 1e-6
    fd = np.zeros_like(theta)
    for j in range(w.d):
        e = np.zeros(w.d)
        e[j] = h
        fd[:, j] = (c_oracle.log_density_grad(w, theta + e)[0] - c_oracle.log_density_grad(w, theta - e)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6)


def test_conjugate_gradient_value_and_prediction_match_closed_form():
    w = W.make_c1()
    roles = folds.roles_of(w)
    rng = np.random.default_rng(2)
    theta = rng.normal(size=(w.C, w.p))
    lp, g, s = c_oracle.log_density_grad(w, theta)
    for c in (0, 69, 399):
        k = c // w.L
        gc = closed_form.grad_log_posterior(theta[c], w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
        np.testing.assert_allclose(g[c], gc, rtol=1e-10, atol=1e-9)
        vc = closed_form.log_posterior_density(theta[c], w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
        assert abs(lp[c] - vc) < 1e-8 * abs(vc)
        # the test row's Gaussian log density, written out
        row = int(np.flatnonzero(roles[k] == 2)[0])
        eta = float(w.X[row] @ theta[c])
        assert s[c] == pytest.approx(-0.5 * np.log(2 * np.pi * w.sigma ** 2) - (w.y[row] - eta) ** 2 / (2 * w.sigma ** 2),
                                     rel=1e-12)


@pytest.mark.parametrize("name,folds_", [("c1", (0, 10)), ("c2", (0, 4)), ("c3", (0, 6)), ("c4", (0, 3)),
                                         ("c5", (0, 2)), ("ex1", (0, 5))])
def test_log_density_equals_numpy_oracle(name, folds_):
    w = W.fold_subset(W.make(name), *folds_)
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    theta = w.init_pos + 0.1 * np.random.default_rng(3).standard_normal(w.init_pos.shape)
    lp, g, s = c_oracle.log_density_grad(w, theta)
    np.testing.assert_allclose(lp, model.log_density(w, theta, roles, foc), rtol=1e-12)
    go = model.grad_log_density(w, theta, roles, foc)
    assert np.max(np.abs(g - go)) <= 1e-12 * np.max(np.abs(go))
    np.testing.assert_allclose(s, model.log_pred(w, theta, roles, foc), rtol=1e-12)


def _runs(name, folds_, n_iter, **over):
    w = W.fold_subset(W.make(name), *folds_)
    w = dataclasses.replace(w, n_warmup=min(w.n_warmup, 50), batch_size=10, n_blocks=5, **over)
    return w, c_oracle.run_all(w, n_iter), sampler.run_all(w, n_iter=n_iter)


@pytest.mark.parametrize("name,folds_,n_iter,over", [("c1", (0, 20), 300, {}),
                                                     ("c1", (0, 20), 300, {"rhat_mode": 1}),
                                                     ("c3", (0, 4), 120, {}),
                                                     ("c2", (0, 2), 80, {}),
                                                     ("ex1", (0, 4), 100, {})])
def test_runs_replay_numpy_oracle(name, folds_, n_iter, over):
    """Same Philox streams, same arithmetic: every accept decision, state,
    accumulator and diagnostic agrees to rounding."""
    w, rc, ro = _runs(name, folds_, n_iter, **over)
    np.testing.assert_array_equal(rc.arr["n_accept"], ro.acc.n_accept)
    np.testing.assert_array_equal(rc.arr["n_divergent"], ro.acc.n_divergent)
    np.testing.assert_allclose(rc.q, ro.state.q, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(rc.s, ro.state.s, rtol=1e-11, atol=1e-12)
    for key in ("U", "U2", "V", "V2", "Z"):
        a, b = rc.arr[key], getattr(ro.acc, key)
        np.testing.assert_array_equal(np.isfinite(a), np.isfinite(b))
        f = np.isfinite(b)
        np.testing.assert_allclose(a[f], b[f], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(rc.arr["blk_n"], ro.acc.blk_n)
    np.testing.assert_allclose(rc.arr["blk_mean"], ro.acc.blk_mean, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(rc.arr["blk_m2"], ro.acc.blk_m2, rtol=1e-10, atol=1e-10)
    dc = rc.diagnostics()
    do = diagnostics.from_accumulators(ro.acc, w.K, w.L, w.batch_size)
    for key in ("elpd_fold", "mcse_fold", "rhat_fold", "ess_fold"):
        np.testing.assert_allclose(dc[key], do[key], rtol=1e-9)
    for key in ("elpd", "mcse", "rhat_max", "ess", "accept_rate"):
        assert dc[key] == pytest.approx(do[key], rel=1e-9)
    assert dc["n_divergent"] == do["n_divergent"] and dc["n_draws"] == ro.acc.n_draws


def test_fold_encodings_agree():
    """The same folds given as an index, as intervals and as a dense role
    matrix: identical log densities, gradients and log predictives."""
    w = W.fold_subset(W.make("c3"), 0, 6)                    # hv-block intervals
    theta = w.init_pos + 0.1 * np.random.default_rng(5).standard_normal(w.init_pos.shape)
    a = c_oracle.log_density_grad(w, theta)
    b = c_oracle.log_density_grad(W.with_dense_roles(w), theta)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    w1 = W.fold_subset(W.make("c1"), 0, 10)                   # LOO index
    theta1 = w1.init_pos + 0.1 * np.random.default_rng(6).standard_normal(w1.init_pos.shape)
    a = c_oracle.log_density_grad(w1, theta1)
    b = c_oracle.log_density_grad(W.with_dense_roles(w1), theta1)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_divergent_transitions_are_counted_alike():
    """A step size far past the leapfrog's stability limit: every energy
    error exceeds the divergence threshold, none is accepted, and both
    oracles count the same divergences."""
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 10), n_warmup=0, batch_size=5, n_blocks=2, step_size=2.0)
    rc, ro = c_oracle.run_all(w, 20), sampler.run_all(w, n_iter=20)
    assert ro.acc.n_divergent.sum() == w.C * 20 and ro.acc.n_accept.sum() == 0
    np.testing.assert_array_equal(rc.arr["n_divergent"], ro.acc.n_divergent)
    np.testing.assert_array_equal(rc.arr["n_accept"], ro.acc.n_accept)


def test_threads_do_not_change_results():
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 16), n_warmup=20, batch_size=10, n_blocks=4)
    a = c_oracle.run_all(w, 80, threads=1)
    b = c_oracle.run_all(w, 80, threads=4)
    np.testing.assert_array_equal(a.q, b.q)
    np.testing.assert_array_equal(a.arr["U"], b.arr["U"])
    assert a.diagnostics()["elpd"] == b.diagnostics()["elpd"]


def test_elpd_within_mcse_of_closed_form():
    """LOO of the conjugate Gaussian: the C oracle's whole run estimates the
    exact elpd within 4 Monte Carlo standard errors."""
    w = W.make_c1()
    r = c_oracle.run_all(w, threads=4)
    d = r.diagnostics()
    roles = folds.roles_of(w)
    exact = sum(closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1, roles[k] == 2)["elpd"]
                for k in range(w.K))
    assert abs(d["elpd"] - exact) < 4 * d["mcse"]
    assert d["rhat_max"] < 1.1
