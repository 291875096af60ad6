"""Pins of the oracle's fold roles, log densities, gradients and closed forms (CPU only)."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

from oracle import closed_form, folds, model
from paper_2310_07002_amd import workloads as W


# --------------------------------------------------------------------------- roles

def test_roles_from_index_by_enumeration():
    fi = np.array([2, 0, 1, 1, -1, 0], dtype=np.int32)
    r = folds.roles_from_index(fi, 3)
    for k in range(3):
        for i in range(6):
            assert r[k, i] == (folds.ROLE_TEST if fi[i] == k else folds.ROLE_TRAIN)


def test_roles_from_intervals_by_enumeration():
    n = 23
    iv = np.array([[0, 5, 0, 8], [5, 10, 2, 13], [20, 23, 17, 23]])
    r = folds.roles_from_intervals(iv, n)
    for k, (lo, hi, elo, ehi) in enumerate(iv):
        for i in range(n):
            want = folds.ROLE_TEST if lo <= i < hi else (
                folds.ROLE_EXCLUDED if elo <= i < ehi else folds.ROLE_TRAIN)
            assert r[k, i] == want


def test_hvblock_workload_fold_shapes():
    w = W.make_c3()
    assert w.n == 4996 and w.K == 1000
    r = folds.roles_of(w)
    test_sizes = (r == folds.ROLE_TEST).sum(axis=1)
    train_sizes = (r == folds.ROLE_TRAIN).sum(axis=1)
    assert test_sizes[:-1].min() == 5 and test_sizes[-1] == 1
    assert train_sizes.min() == 4971 and train_sizes.max() == 4985
    # every row is tested exactly once
    assert np.all((r == folds.ROLE_TEST).sum(axis=0) == 1)


# --------------------------------------------------------------------------- likelihoods

def test_loglik_rows_match_library_densities():
    rng = np.random.default_rng(0)
    eta = rng.normal(size=50)
    yg = rng.normal(size=50)
    np.testing.assert_allclose(model.loglik_rows(model.GAUSSIAN, yg, eta, 0.7),
                               stats.norm.logpdf(yg, loc=eta, scale=0.7), rtol=1e-13)
    yb = (rng.random(50) < 0.4).astype(float)
    np.testing.assert_allclose(model.loglik_rows(model.LOGISTIC, yb, eta, 1.0),
                               stats.bernoulli.logpmf(yb, 1 / (1 + np.exp(-eta))), rtol=1e-12)
    yp = rng.poisson(2.0, size=50).astype(float)
    np.testing.assert_allclose(model.loglik_rows(model.POISSON, yp, eta, 1.0),
                               stats.poisson.logpmf(yp, np.exp(eta)), rtol=1e-12)


def _small(family, n=40, p=3, K=4, L=2, seed=0, hier_groups=0):
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
    if hier_groups:
        group_of = np.sort(rng.integers(0, hier_groups, size=n)).astype(np.int32)
        fold_index = group_of.copy()
        K = hier_groups
    w = W.Workload(name="small", family=family, precision=0, X=X, y=y, K=K, L=L,
                   fold_kind=W.FOLDS_INDEX, fold_index=fold_index, group_of=group_of,
                   n_groups=hier_groups, sigma=0.8)
    w.prior_scale = rng.uniform(0.5, 2.0, size=w.d)
    w.inv_mass = np.ones(w.d)
    return w


@pytest.mark.parametrize("family,groups", [(model.GAUSSIAN, 0), (model.LOGISTIC, 0),
                                           (model.POISSON, 0), (model.HIER_LOGISTIC, 5),
                                           (model.HIER_GAUSSIAN, 5)])
def test_gradient_matches_central_differences(family, groups):
    w = _small(family, hier_groups=groups)
    rng = np.random.default_rng(1)
    theta = 0.3 * rng.normal(size=(w.C, w.d))
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    g = model.grad_log_density(w, theta, roles, foc)
    h = 1e-6
    fd = np.zeros_like(theta)
    for j in range(w.d):
        e = np.zeros(w.d)
        e[j] = h
        fd[:, j] = (model.log_density(w, theta + e, roles, foc)
                    - model.log_density(w, theta - e, roles, foc)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6)


def test_planted_gradient_sign_error_is_caught():
    """The finite-difference pin fails when a term's sign is flipped in the oracle."""
    w = _small(model.POISSON)
    theta = 0.2 * np.ones((w.C, w.d))
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    wrong = -model.grad_log_prior(w, theta) + (model.grad_log_density(w, theta, roles, foc)
                                               - model.grad_log_prior(w, theta))
    h = 1e-6
    e = np.zeros(w.d)
    e[0] = h
    fd0 = (model.log_density(w, theta + e, roles, foc) - model.log_density(w, theta - e, roles, foc)) / (2 * h)
    assert not np.allclose(wrong[:, 0], fd0, rtol=1e-6, atol=1e-6)


def test_hier_linear_predictor_by_loops():
    w = _small(model.HIER_LOGISTIC, n=12, hier_groups=3)
    rng = np.random.default_rng(3)
    theta = rng.normal(size=(w.C, w.d))
    eta = model.linear_predictor(w, theta)
    for c in range(w.C):
        beta, mu, u, z = theta[c, :w.p], theta[c, w.p], theta[c, w.p + 1], theta[c, w.p + 2:]
        for i in range(w.n):
            want = sum(w.X[i, j] * beta[j] for j in range(w.p)) + mu + math.exp(u) * z[w.group_of[i]]
            assert abs(eta[i, c] - want) < 1e-12


def test_hier_prior_is_halfnormal_with_jacobian():
    """exp of the u-part of the prior integrates to one over u (change of variables)."""
    w = _small(model.HIER_LOGISTIC, hier_groups=2)
    u = np.linspace(-30, 4, 40001)
    theta = np.zeros((u.size, w.d))
    theta[:, w.p + 1] = u
    lp = model.log_prior(w, theta) - (w.d - 1) * (-0.5 * math.log(2 * math.pi))
    assert abs(np.trapezoid(np.exp(lp), u) - 1.0) < 1e-6


def _hier_gauss_by_loops(w, theta, rows):
    """log prior + sum over `rows` of the row log densities, for one chain,
    by explicit loops and library densities (Example 1's model as written:
    alpha_j = mu + sigma_a z_j, y ~ N(alpha_j + x'beta, sigma_y^2), half-normal
    scale priors with variance 10 in their log-scale parameters)."""
    p = w.p
    beta, mu, ua, uy, z = theta[:p], theta[p], theta[p + 1], theta[p + 2], theta[p + 3:]
    sa, sy = math.exp(ua), math.exp(uy)
    total = 0.0
    for i in rows:
        eta = sum(w.X[i, j] * beta[j] for j in range(p)) + mu + sa * z[w.group_of[i]]
        total += stats.norm.logpdf(w.y[i], loc=eta, scale=sy)
    prior = (stats.norm.logpdf(beta).sum() + stats.norm.logpdf(mu) + stats.norm.logpdf(z).sum()
             + stats.halfnorm.logpdf(sa, scale=math.sqrt(10.0)) + ua
             + stats.halfnorm.logpdf(sy, scale=math.sqrt(10.0)) + uy)
    return prior, total


def test_hier_gaussian_value_and_predictive_by_loops():
    """Example 1's family: log density and LOGO log predictive against the
    model written out with scipy's normal and half-normal densities."""
    w = _small(model.HIER_GAUSSIAN, n=30, hier_groups=4)
    rng = np.random.default_rng(5)
    theta = 0.5 * rng.normal(size=(w.C, w.d))
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    lp = model.log_density(w, theta, roles, foc)
    s = model.log_pred(w, theta, roles, foc)
    for c in range(w.C):
        k = foc[c]
        prior, lik = _hier_gauss_by_loops(w, theta[c], np.flatnonzero(roles[k] == folds.ROLE_TRAIN))
        _, pred = _hier_gauss_by_loops(w, theta[c], np.flatnonzero(roles[k] == folds.ROLE_TEST))
        assert abs(lp[c] - (prior + lik)) < 1e-10 * abs(prior + lik)
        assert abs(s[c] - pred) < 1e-10 * abs(pred)


def test_hier_gaussian_gradient_matches_conditional_conjugate_posterior():
    """At fixed log scales the (beta, mu, z) block of Example 1's model is a
    linear Gaussian regression y = A (beta, mu, z) + noise, A = [X, 1, sigma_a
    G] (G the group indicators of the training rows), with an N(0, I) prior:
    its conditional posterior is N(m, P^-1), P = I + A'A / sigma_y^2,
    m = P^-1 A'y / sigma_y^2, so the gradient of the log density in that
    block is -P (theta_lin - m) exactly."""
    w = _small(model.HIER_GAUSSIAN, n=36, p=3, hier_groups=6)
    rng = np.random.default_rng(9)
    roles = folds.roles_of(w)
    for k in (0, 3):
        theta = rng.normal(size=(1, w.d))
        tr = roles[k] == folds.ROLE_TRAIN
        sa, sy = math.exp(theta[0, w.p + 1]), math.exp(theta[0, w.p + 2])
        Gm = np.zeros((w.n, w.n_groups))
        Gm[np.arange(w.n), w.group_of] = 1.0
        A = np.concatenate([w.X, np.ones((w.n, 1)), sa * Gm], axis=1)[tr]
        P = np.eye(A.shape[1]) + A.T @ A / sy ** 2
        m = np.linalg.solve(P, A.T @ w.y[tr] / sy ** 2)
        lin = np.concatenate([np.arange(w.p + 1), np.arange(w.p + 3, w.d)])
        g = model.grad_log_density(w, theta, roles, np.array([k]))[0]
        np.testing.assert_allclose(g[lin], -P @ (theta[0, lin] - m), rtol=1e-10, atol=1e-10)


def test_hier_gaussian_scale_priors_are_halfnormal_with_jacobian():
    """exp of each log-scale's prior part integrates to one over u (the
    half-normal with variance 10 under sigma = e^u)."""
    w = _small(model.HIER_GAUSSIAN, hier_groups=2)
    u = np.linspace(-30, 5, 40001)
    for j in (w.p + 1, w.p + 2):
        theta = np.zeros((u.size, w.d))
        theta[:, w.p + 1] = -40.0
        theta[:, w.p + 2] = -40.0
        theta[:, j] = u
        lp = model.log_prior(w, theta)
        # subtract the standard-normal block and the other scale's term
        lp = lp - (w.d - 2) * (-0.5 * math.log(2 * math.pi))
        lp = lp - (stats.halfnorm.logpdf(math.exp(-40.0), scale=math.sqrt(10.0)) - 40.0)
        assert abs(np.trapezoid(np.exp(lp), u) - 1.0) < 1e-6, j


# --------------------------------------------------------------------------- conjugate case

def _c1_small():
    w = W.make_c1()
    return w, folds.roles_of(w)


def test_conjugate_gradient_and_value_match_closed_form():
    w, roles = _c1_small()
    rng = np.random.default_rng(2)
    for k in (0, 17, 99):
        theta = rng.normal(size=(1, w.p))
        foc = np.array([k])
        g = model.grad_log_density(w, theta, roles, foc)[0]
        gc = closed_form.grad_log_posterior(theta[0], w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
        np.testing.assert_allclose(g, gc, rtol=1e-10, atol=1e-9)
        v = model.log_density(w, theta, roles, foc)[0]
        vc = closed_form.log_posterior_density(theta[0], w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
        assert abs(v - vc) < 1e-8 * abs(vc)


def test_closed_form_elpd_two_routes():
    w, roles = _c1_small()
    for k in (0, 5, 50):
        tr, te = roles[k] == 1, roles[k] == 2
        ex = closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, tr, te)
        both = tr | te
        ratio = closed_form.log_marginal(w.X[both], w.y[both], w.sigma, w.prior_scale) - \
            closed_form.log_marginal(w.X[tr], w.y[tr], w.sigma, w.prior_scale)
        assert abs(ex["elpd"] - ratio) < 1e-9
        m2, V2 = closed_form.loo_by_downdate(w.X, w.y, w.sigma, w.prior_scale, k)
        np.testing.assert_allclose(ex["m"], m2, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(ex["V"], V2, rtol=1e-8, atol=1e-14)


def test_closed_form_predictive_moments_by_iid_monte_carlo():
    w, roles = _c1_small()
    k = 3
    tr, te = roles[k] == 1, roles[k] == 2
    ex = closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, tr, te)
    rng = np.random.default_rng(7)
    th = rng.multivariate_normal(ex["m"], ex["V"], size=400000)
    s = model.log_pred(w, th, roles, np.full(th.shape[0], k))
    f = np.exp(s)
    n = f.size
    assert abs(f.mean() - math.exp(ex["log_Ef"])) < 5 * f.std() / math.sqrt(n)
    assert abs((f ** 2).mean() - math.exp(ex["log_Ef2"])) < 5 * (f ** 2).std() / math.sqrt(n)
    assert abs(s.mean() - ex["Es"]) < 5 * s.std() / math.sqrt(n)
    assert abs(s.var() - ex["Vars"]) < 0.02 * ex["Vars"]


def test_multirow_test_set_is_joint_density():
    """With hv-blocks, s is the joint log density of the whole test block."""
    w = W.make_c3()
    roles = folds.roles_of(w)
    k = 10
    theta = w.truth[None, :]
    s = model.log_pred(w, theta, roles, np.array([k]))[0]
    rows = np.where(roles[k] == 2)[0]
    assert rows.size == 5
    want = sum(stats.norm.logpdf(w.y[i], loc=w.X[i] @ w.truth, scale=w.sigma) for i in rows)
    assert abs(s - want) < 1e-10
