"""Hyvaerinen (HS) and Dawid-Sebastiani (DSS) cross-validation scores by online estimators.

TEST INFRASTRUCTURE ONLY (see the package header).

Appendix, sections on HS and DSS, the table of online estimator functions,
and the online HS and DSS samplers.  Both scores are positively oriented.
Per fold k with test rows V_k and, for every chain, the post-warm-up draws:

HS (continuous responses: the Gaussian family here).  With
  d1_i = d/dy_i log p(y_i | theta) = -(y_i - eta_i) / sigma^2,   d2_i = -1 / sigma^2,
every chain accumulates H1 = sum_draws sum_i (d2_i + d1_i^2) and, per test row,
H2_i = sum_draws d1_i; then, with mu1_i and mu2_i the averages over the LN
draws of the fold,
  HS_k = sum_i ( -2 mu1_i + mu2_i^2 ).
Reading: the printed online algorithm squares the fold average of the
first derivatives summed over the test rows, while the per-observation
formula it comes from squares each observation's average; they agree for a
single test row, and the per-observation form is taken.

DSS.  One predictive draw ytil_i ~ p(y_i | theta) per chain, draw and test
row, from its own Philox stream (counter (chain, t, TAG_PREDICT, i-slot)):
  Gaussian  eta + sigma z, z by Box-Muller from the block's four words;
  Bernoulli 1 if u < 1/(1+e^-eta) else 0;
  Poisson   the smallest k with u <= sum_{j<=k} e^-lam lam^j / j!, lam = e^eta
            (the terms built by the recurrence p_j = p_{j-1} lam / j);
with u from the block's first two words.  Every chain accumulates, per test
row and pair of rows, Dx_i = sum_draws (ytil_i - y_i) and
Dxx_ab = sum_draws (ytil_a - y_a)(ytil_b - y_b); then
  m = sum_l Dx / (LN) = mu_hat - y,
  Sigma_hat = [sum_l Dxx - (sum_l Dx)(sum_l Dx)' / (LN)] / (LN - 1),
  DSS_k = -log|Sigma_hat| - m' Sigma_hat^-1 m.
Reading: the draws are centred on the observed test values instead of a
warm-up mean; the estimator is algebraically the same and no warm-up pass
is needed.

Pins: the conjugate Gaussian's exact targets (conjugate_targets below,
checked against the sampled estimates in tests/test_oracle_scores.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

SCORE_HS, SCORE_DSS = 1, 2
POISSON_MAX_K = 100000


def test_rows_of_folds(roles: np.ndarray):
    """List of the test-row index arrays of each fold (roles K x n)."""
    return [np.flatnonzero(roles[k] == 2) for k in range(roles.shape[0])]


def predictive_draw(family: int, eta: np.ndarray, sigma: float, words) -> np.ndarray:
    w0, w1, w2, w3 = words
    u = philox.uniform_from_words(w0, w1)
    if family == 0:                                   # Gaussian
        u2 = philox.uniform_from_words(w2, w3)
        return eta + sigma * np.sqrt(-2.0 * np.log(u)) * np.cos(2.0 * np.pi * u2)
    if family in (1, 3):                              # Bernoulli (logistic, hierarchical logistic)
        return (u < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    lam = np.exp(eta)                                 # Poisson, inverse cdf
    k = np.zeros_like(eta)
    p = np.exp(-lam)
    F = p.copy()
    active = u > F
    j = 0
    while active.any() and j < POISSON_MAX_K:
        j += 1
        p = np.where(active, p * lam / j, p)
        F = np.where(active, F + p, F)
        k = np.where(active, k + 1.0, k)
        active = active & (u > F)
    return k


def test_eta(w, theta: np.ndarray, rows_of_chain: np.ndarray) -> np.ndarray:
    """eta at each chain's test rows: rows_of_chain [C, vmax] (-1 = none) ->
    [C, vmax] (NaN where there is no row)."""
    r = np.maximum(rows_of_chain, 0)
    Xr = w.X[r]                                              # [C, vmax, p]
    if w.family == 3:
        p = w.p
        beta, mu, tau, z = theta[:, :p], theta[:, p], np.exp(theta[:, p + 1]), theta[:, p + 2:]
        g = w.group_of[r]
        eta = np.einsum("cvp,cp->cv", Xr, beta) + mu[:, None] + tau[:, None] * np.take_along_axis(z, g, axis=1)
    else:
        eta = np.einsum("cvp,cp->cv", Xr, theta)
    return np.where(rows_of_chain >= 0, eta, np.nan)


def rows_of_chains(roles: np.ndarray, L: int) -> np.ndarray:
    """[C, vmax] test rows of each chain's fold, padded with -1."""
    tests = test_rows_of_folds(roles)
    vmax = max(len(t) for t in tests)
    out = -np.ones((len(tests) * L, vmax), dtype=np.int64)
    for k, t in enumerate(tests):
        out[k * L:(k + 1) * L, :len(t)] = t
    return out


class ScoreAccumulators:
    """Per-chain HS and DSS sums (padded to the largest test set)."""

    def __init__(self, C: int, vmax: int, flags: int):
        self.flags = flags
        self.H1 = np.zeros(C)
        self.H2 = np.zeros((C, vmax))
        self.Dx = np.zeros((C, vmax))
        self.Dxx = np.zeros((C, vmax, vmax))


def accumulate(w, acc: ScoreAccumulators, eta_test, y_test, t: int) -> None:
    """Fold one post-warm-up draw into the sums.  eta_test, y_test: [C, vmax]
    with NaN where a chain's fold has fewer test rows."""
    valid = ~np.isnan(y_test)
    e = np.where(valid, eta_test, 0.0)
    yv = np.where(valid, y_test, 0.0)
    if acc.flags & SCORE_HS:
        d1 = -(yv - e) / w.sigma ** 2
        d2 = -1.0 / w.sigma ** 2
        acc.H1 += np.sum(np.where(valid, d2 + d1 * d1, 0.0), axis=1)
        acc.H2 += np.where(valid, d1, 0.0)
    if acc.flags & SCORE_DSS:
        chains = w.chain_offset + np.arange(w.C)
        words = philox.predictive_words(w.seed, chains, t, y_test.shape[1])
        yt = predictive_draw(w.family, e, w.sigma, words)
        r = np.where(valid, yt - yv, 0.0)
        acc.Dx += r
        acc.Dxx += r[:, :, None] * r[:, None, :]


def fold_scores(acc: ScoreAccumulators, K: int, L: int, N: int, sizes) -> dict:
    """HS_k and DSS_k (arrays of K) from the sums of N draws per chain."""
    LN = L * N
    out = {}
    if acc.flags & SCORE_HS:
        hs = np.empty(K)
        for k in range(K):
            v = sizes[k]
            sl = slice(k * L, (k + 1) * L)
            mu1_sum = acc.H1[sl].sum() / LN
            mu2 = acc.H2[sl, :v].sum(axis=0) / LN
            hs[k] = -2.0 * mu1_sum + np.sum(mu2 * mu2)
        out["hs_fold"] = hs
        out["hs"] = float(hs.sum())
    if acc.flags & SCORE_DSS:
        dss = np.empty(K)
        for k in range(K):
            v = sizes[k]
            sl = slice(k * L, (k + 1) * L)
            sx = acc.Dx[sl, :v].sum(axis=0)
            sxx = acc.Dxx[sl, :v, :v].sum(axis=0)
            m = sx / LN
            S = (sxx - np.outer(sx, sx) / LN) / (LN - 1)
            sign, logdet = np.linalg.slogdet(S)
            dss[k] = -logdet - m @ np.linalg.solve(S, m) if sign > 0 else np.nan
        out["dss_fold"] = dss
        out["dss"] = float(dss.sum())
    return out


def conjugate_targets(X, y, sigma, prior_scale, roles) -> dict:
    """What the two estimators converge to for the conjugate Gaussian, fold by
    fold, from the exact fold posterior N(m_k, V_k) (closed_form)."""
    from . import closed_form
    K = roles.shape[0]
    hs = np.empty(K)
    dss = np.empty(K)
    s2 = sigma * sigma
    for k in range(K):
        tr, te = roles[k] == 1, roles[k] == 2
        m, V, _ = closed_form.fold_posterior(X, y, sigma, prior_scale, tr)
        XV = X[te]
        mu = XV @ m
        Q = XV @ V @ XV.T
        r = y[te] - mu
        vi = np.diag(Q)
        # HS: mu1_i = -1/s2 + (r_i^2 + v_i)/s2^2, mu2_i = -r_i/s2
        hs[k] = np.sum(-2.0 * (-1.0 / s2 + (r * r + vi) / s2 ** 2) + (r / s2) ** 2)
        S = s2 * np.eye(XV.shape[0]) + Q
        sign, logdet = np.linalg.slogdet(S)
        dss[k] = -logdet - r @ np.linalg.solve(S, r)
    return {"hs_fold": hs, "dss_fold": dss}
