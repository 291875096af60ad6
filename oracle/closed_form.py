"""Exact fold posteriors and predictives of the conjugate Gaussian regression.

TEST INFRASTRUCTURE ONLY (see the package header).

For y | theta ~ N(X theta, sigma^2 I) with known sigma and prior
theta ~ N(0, S0), S0 = diag(prior_scale^2), fold k's posterior given its
training rows T is Gaussian:

  V_k = (S0^-1 + X_T' X_T / sigma^2)^-1,   m_k = V_k X_T' y_T / sigma^2

and, for its v test rows with design X_V, the exact quantities a PCV run
estimates by Monte Carlo (f = p(y_V | theta), s = log f):

  elpd_k = log p(y_V | y_T) = log N(y_V | X_V m_k, sigma^2 I + X_V V_k X_V')
  E[f]   = exp(elpd_k)
  E[f^2] = (2 sigma sqrt(pi))^-v N(y_V | X_V m_k, sigma^2/2 I + X_V V_k X_V')
  E[s]   = -v/2 log(2 pi sigma^2) - (|y_V - X_V m_k|^2 + tr(X_V V_k X_V')) / (2 sigma^2)
  Var[s] = (2 tr(Q^2) + 4 r' Q r) / (4 sigma^4),   Q = X_V V_k X_V',  r = y_V - X_V m_k
  grad log pi_k(theta) = -V_k^-1 (theta - m_k)
  log pi_k(theta) = log N(theta | m_k, V_k) + log N(y_T | 0, sigma^2 I + X_T S0 X_T')

These pin the oracle's model, HMC and diagnostics (the first and third configs
of the test suite are conjugate).  A second, independent route to elpd_k is
the ratio of marginal likelihoods p(y_T u y_V) / p(y_T); for leave-one-out a
Sherman-Morrison downdate of the full-data posterior gives V_k and m_k a
second way.  Both are checked against the formulas above in the tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.stats import multivariate_normal


def fold_posterior(X, y, sigma, prior_scale, train_mask):
    Xt, yt = X[train_mask], y[train_mask]
    prec = np.diag(1.0 / np.asarray(prior_scale) ** 2) + Xt.T @ Xt / sigma ** 2
    V = np.linalg.inv(prec)
    V = 0.5 * (V + V.T)
    m = V @ (Xt.T @ yt) / sigma ** 2
    return m, V, prec


def _logpdf(x, mean, cov):
    return float(multivariate_normal(mean=mean, cov=cov, allow_singular=False).logpdf(x))


def fold_exact(X, y, sigma, prior_scale, train_mask, test_mask) -> dict:
    m, V, prec = fold_posterior(X, y, sigma, prior_scale, train_mask)
    Xv, yv = X[test_mask], y[test_mask]
    v = Xv.shape[0]
    Q = Xv @ V @ Xv.T
    r = yv - Xv @ m
    elpd = _logpdf(yv, Xv @ m, sigma ** 2 * np.eye(v) + Q)
    log_ef2 = -v * math.log(2.0 * sigma * math.sqrt(math.pi)) + \
        _logpdf(yv, Xv @ m, 0.5 * sigma ** 2 * np.eye(v) + Q)
    es = -0.5 * v * math.log(2 * math.pi * sigma ** 2) - (r @ r + np.trace(Q)) / (2 * sigma ** 2)
    vs = (2.0 * np.trace(Q @ Q) + 4.0 * r @ Q @ r) / (4.0 * sigma ** 4)
    return {"m": m, "V": V, "prec": prec, "elpd": elpd, "log_Ef": elpd,
            "log_Ef2": log_ef2, "Es": es, "Vars": vs}


def log_marginal(X, y, sigma, prior_scale) -> float:
    S0 = np.diag(np.asarray(prior_scale) ** 2)
    cov = sigma ** 2 * np.eye(X.shape[0]) + X @ S0 @ X.T
    return _logpdf(y, np.zeros(X.shape[0]), cov)


def log_posterior_density(theta, X, y, sigma, prior_scale, train_mask) -> float:
    """Unnormalised fold log posterior (log prior + log likelihood) in closed form."""
    m, V, _ = fold_posterior(X, y, sigma, prior_scale, train_mask)
    return _logpdf(theta, m, V) + log_marginal(X[train_mask], y[train_mask], sigma, prior_scale)


def grad_log_posterior(theta, X, y, sigma, prior_scale, train_mask):
    m, _, prec = fold_posterior(X, y, sigma, prior_scale, train_mask)
    return -(prec @ (np.asarray(theta) - m))


def loo_by_downdate(X, y, sigma, prior_scale, i):
    """Leave-one-out posterior of row i from the full-data posterior (Sherman-Morrison)."""
    S0inv = np.diag(1.0 / np.asarray(prior_scale) ** 2)
    Vf = np.linalg.inv(S0inv + X.T @ X / sigma ** 2)
    bf = X.T @ y / sigma ** 2
    x = X[i]
    Vx = Vf @ x
    Vk = Vf + np.outer(Vx, Vx) / (sigma ** 2 - x @ Vx)
    mk = Vk @ (bf - x * y[i] / sigma ** 2)
    return mk, Vk
