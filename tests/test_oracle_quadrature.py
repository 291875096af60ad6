"""The sampler's elpd on non-conjugate models, pinned by brute force (CPU only).

Logistic and Poisson GLMs with two coefficients have no closed-form
posterior, but with two coefficients the exact K-fold predictive density,
log of the integral of p(y_test | beta) p(beta | y_train), is a quadrature on a
fine grid.  The likelihoods and the prior are written out here from their
textbook definitions, independently of the oracle's model code.  The oracle's
HMC run (fixed trajectories, streaming log-sum-exp of the fold's test log
density over draws, Section 2.4 and Algorithm A2) must land within 4 Monte
Carlo standard errors of the exact value, fold by fold and in total, and its
R-hat must be near 1.  A dropped term, a wrong sign in the likelihood or a
misplaced fold mask moves the estimate by many standard errors."""
import math

import numpy as np
import pytest

from oracle import c_oracle, diagnostics, model, sampler
from paper_2310_07002_amd import workloads as W


def _workload(family, seed):
    rng = np.random.default_rng(seed)
    n, p, K, L = 48, 2, 4, 4
    X = rng.normal(size=(n, p))
    beta = np.array([0.8, -0.5])
    eta = X @ beta
    if family == model.LOGISTIC:
        y = (rng.random(n) < 1.0 / (1.0 + np.exp(-eta))).astype(float)
        info = 0.25 * (X ** 2).sum(axis=0)
    else:
        y = rng.poisson(np.exp(eta)).astype(float)
        info = (np.exp(eta)[:, None] * X ** 2).sum(axis=0)
    prior_scale = np.array([1.5, 1.0])
    inv_mass = 1.0 / (info * (K - 1) / K + 1.0 / prior_scale ** 2)
    fold_index = (np.arange(n) % K).astype(np.int32)
    init = beta[None, :] + 0.3 * rng.standard_normal((K * L, p)) * np.sqrt(inv_mass)[None, :]
    return W.Workload(name="quad", family=family, precision=0, X=X, y=y, K=K, L=L, fold_kind=W.FOLDS_INDEX,
                      fold_index=fold_index, prior_scale=prior_scale, step_size=0.35, n_leapfrog=8,
                      inv_mass=inv_mass, init_pos=init, n_warmup=200, n_samples=4000, batch_size=100,
                      n_blocks=5, seed=11 + seed)


def _loglik(family, y, eta):
    """Pointwise log p(y | eta): Bernoulli with a logit link, or Poisson with a log link."""
    if family == model.LOGISTIC:
        return y * eta - np.logaddexp(0.0, eta)
    lgam = np.array([math.lgamma(v + 1.0) for v in np.ravel(y)]).reshape(np.shape(y))
    return y * eta - np.exp(eta) - lgam


def _fold_grid_terms(w, k, lo, hi, m):
    """Log posterior (unnormalised) and the fold's test log density on an
    m x m grid over the box [lo, hi]."""
    B0, B1 = np.meshgrid(np.linspace(lo[0], hi[0], m), np.linspace(lo[1], hi[1], m), indexing="ij")
    grid = np.stack([B0.ravel(), B1.ravel()], axis=1)                 # [m^2, 2]
    log_prior = -0.5 * ((grid / w.prior_scale) ** 2).sum(axis=1)
    test = w.fold_index == k
    ll = _loglik(w.family, w.y[None, :], grid @ w.X.T)                  # [m^2, n]
    return grid, log_prior + ll[:, ~test].sum(axis=1), ll[:, test].sum(axis=1)


def _exact_fold_elpd(w, k, m=401, width=10.0):
    """log p(y_test | y_train) for fold k by quadrature: a coarse grid locates
    the posterior (mean and sd per coefficient), a fine m x m grid over
    mean +- width sd integrates it.  Returns the value and the largest
    posterior mass of one cell."""
    grid, lp, _ = _fold_grid_terms(w, k, (-4.0, -4.0), (4.0, 4.0), 201)
    wts = np.exp(lp - np.logaddexp.reduce(lp))
    mean = wts @ grid
    sd = np.sqrt(wts @ (grid - mean) ** 2)
    _, lp, s = _fold_grid_terms(w, k, mean - width * sd, mean + width * sd, m)
    lz = np.logaddexp.reduce(lp)
    return float(np.logaddexp.reduce(lp + s) - lz), float(np.exp(lp - lz).max())


@pytest.mark.parametrize("family,seed", [(model.LOGISTIC, 0), (model.POISSON, 1)])
def test_sampler_elpd_matches_quadrature(family, seed):
    w = _workload(family, seed)
    exact = []
    for k in range(w.K):
        e, peak = _exact_fold_elpd(w, k)
        assert peak < 1e-3            # the grid resolves the posterior (no single cell dominates)
        exact.append(e)
    exact = np.array(exact)
    # the grid is wide and fine enough: halving the spacing moves nothing
    e2, _ = _exact_fold_elpd(w, 0, m=801)
    assert abs(e2 - exact[0]) < 1e-6
    run = sampler.run_all(w, n_iter=w.n_iter)
    d = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    z = np.abs(d["elpd_fold"] - exact) / d["mcse_fold"]
    assert np.all(z < 4), (d["elpd_fold"], exact, d["mcse_fold"])
    assert abs(d["elpd"] - exact.sum()) < 4 * d["mcse"]
    assert d["rhat_max"] < 1.05
    assert 0.5 < d["accept_rate"] <= 1.0


def test_c_oracle_elpd_matches_quadrature():
    """The plain C oracle on the same logistic workload, against the same
    quadrature."""
    w = _workload(model.LOGISTIC, 0)
    exact = np.array([_exact_fold_elpd(w, k)[0] for k in range(w.K)])
    c_oracle.build(force=False)
    d = c_oracle.run_all(w, threads=4).diagnostics()
    z = np.abs(d["elpd_fold"] - exact) / d["mcse_fold"]
    assert np.all(z < 4), (d["elpd_fold"], exact, d["mcse_fold"])
    assert abs(d["elpd"] - exact.sum()) < 4 * d["mcse"]
