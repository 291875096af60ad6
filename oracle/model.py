"""Masked fold log density, its gradient, and the fold log predictive.

TEST INFRASTRUCTURE ONLY (see the package header).

Appendix B ("Masking for parallel evaluation") writes each fold's log
likelihood and log predictive density as sums over *all* n rows, weighted by a
0/1 row indicator, so that every fold runs the same program.  The likelihood
takes the fold's training rows and the predictive its test rows (the
appendix's listing marks training rows by a fold index that differs from the
fold id; its displayed equation reuses the test indicator for both sums, which
is read as a typo).  For chain c of fold k:

  log pi_c(theta) = log prior(theta) + sum_n [role_k(n) = train] * l(y_n, eta_n)
  s_c(theta)      =                    sum_n [role_k(n) = test ] * l(y_n, eta_n)

s is the joint log density of the fold's whole test set, the quantity whose
posterior mean the fold's LogS estimate takes the log of (Sections 2.1, 2.2,
Algorithm A2).  All normalising constants are kept, so absolute elpd values
compare with closed forms.

Families (l is the per-row log likelihood, eta the linear predictor):
  Gaussian, known sigma:  l = -log(2 pi sigma^2)/2 - (y - eta)^2 / (2 sigma^2)
  Bernoulli, logit link:  l = y eta - log(1 + e^eta)
  Poisson, log link:      l = y eta - e^eta - log(y!)
  hierarchical logistic:  Bernoulli-logit with eta = x'beta + mu + tau z_g(n),
                          theta = (beta, mu, u = log tau, z), tau = e^u,
                          priors beta, mu, z ~ N(0, 1), tau ~ HalfNormal(1)
                          (the log-Jacobian u of tau = e^u is added)
  hierarchical Gaussian:  the grouped regression of Section 2, Example 1:
                          y ~ N(alpha_g(n) + x'beta, sigma_y^2) with
                          alpha_g = mu + sigma_a z_g (non-centred form of
                          alpha_g ~ N(mu, sigma_a^2)),
                          theta = (beta, mu, u_a = log sigma_a, u_y = log sigma_y, z),
                          priors beta, mu, z ~ N(0, 1) and sigma_a, sigma_y
                          half-normal with variance 10 (log-Jacobians u_a, u_y
                          added); l = -log(2 pi)/2 - u_y - (y - eta)^2 / (2 sigma_y^2)
GLM priors: theta_j ~ N(0, prior_scale_j^2).

The gradient is written out by hand (chain rule on the sums above); it is
pinned against central finite differences of log_density and, for the
conjugate Gaussian, against the exact posterior gradient
(tests/test_oracle_model.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import expit, gammaln

from .folds import ROLE_TEST, ROLE_TRAIN

GAUSSIAN, LOGISTIC, POISSON, HIER_LOGISTIC, HIER_GAUSSIAN = 0, 1, 2, 3, 4
HIER_FAMILIES = (HIER_LOGISTIC, HIER_GAUSSIAN)
HIER_SCALE_VAR = 10.0     # variance of the half-normal priors of sigma_a and sigma_y (Example 1)

_LOG_2PI = math.log(2.0 * math.pi)


def loglik_rows(family: int, y: np.ndarray, eta: np.ndarray, sigma: float) -> np.ndarray:
    """Per-row log likelihood l(y_n, eta_n); y broadcasts against eta [n, C]."""
    if family == GAUSSIAN:
        return -0.5 * math.log(2.0 * math.pi * sigma ** 2) - (y - eta) ** 2 / (2.0 * sigma ** 2)
    if family in (LOGISTIC, HIER_LOGISTIC):
        return y * eta - np.logaddexp(0.0, eta)
    if family == POISSON:
        return y * eta - np.exp(eta) - gammaln(y + 1.0)
    raise ValueError(family)


def dloglik_deta(family: int, y: np.ndarray, eta: np.ndarray, sigma: float) -> np.ndarray:
    """Derivative of l(y, eta) with respect to eta."""
    if family == GAUSSIAN:
        return (y - eta) / sigma ** 2
    if family in (LOGISTIC, HIER_LOGISTIC):
        return y - expit(eta)
    if family == POISSON:
        return y - np.exp(eta)
    raise ValueError(family)


def _split_hier(w, theta):
    """(beta, mu, log group scale, z) of the hierarchical families."""
    p = w.p
    z0 = p + 3 if w.family == HIER_GAUSSIAN else p + 2
    return theta[:, :p], theta[:, p], theta[:, p + 1], theta[:, z0:]


def _sigma_y(w, theta):
    """Noise sd per chain [C] (hierarchical Gaussian: e^{u_y}), else the known sigma."""
    if w.family == HIER_GAUSSIAN:
        return np.exp(theta[:, w.p + 2])
    return w.sigma


def linear_predictor(w, theta: np.ndarray) -> np.ndarray:
    """eta[n, C] for chain parameters theta[C, d]."""
    if w.family in HIER_FAMILIES:
        beta, mu, u, z = _split_hier(w, theta)
        tau = np.exp(u)
        return w.X @ beta.T + mu[None, :] + tau[None, :] * z[:, w.group_of].T
    return w.X @ theta.T


def _loglik(w, theta, eta):
    """Per-row log likelihood [n, C] at eta for the chains theta."""
    if w.family == HIER_GAUSSIAN:
        sy = _sigma_y(w, theta)[None, :]
        return -0.5 * _LOG_2PI - np.log(sy) - (w.y[:, None] - eta) ** 2 / (2.0 * sy ** 2)
    return loglik_rows(w.family, w.y[:, None], eta, w.sigma)


def _log_halfnormal(x, var):
    """log density of the half-normal with variance parameter var at x > 0."""
    return math.log(2.0) - 0.5 * math.log(2.0 * math.pi * var) - x ** 2 / (2.0 * var)


def log_prior(w, theta: np.ndarray) -> np.ndarray:
    if w.family == HIER_GAUSSIAN:
        beta, mu, ua, z = _split_hier(w, theta)
        uy = theta[:, w.p + 2]
        std = np.concatenate([beta, mu[:, None], z], axis=1)
        lp = np.sum(-0.5 * _LOG_2PI - 0.5 * std ** 2, axis=1)
        # sigma_a, sigma_y half-normal (variance 10), each with the log-Jacobian of sigma = e^u
        lp += _log_halfnormal(np.exp(ua), HIER_SCALE_VAR) + ua
        lp += _log_halfnormal(np.exp(uy), HIER_SCALE_VAR) + uy
        return lp
    if w.family == HIER_LOGISTIC:
        beta, mu, u, z = _split_hier(w, theta)
        std = np.concatenate([beta, mu[:, None], z], axis=1)
        lp = np.sum(-0.5 * _LOG_2PI - 0.5 * std ** 2, axis=1)
        # tau ~ HalfNormal(1): log 2 + log N(tau | 0, 1); plus log|d tau / d u| = u
        tau = np.exp(u)
        lp += math.log(2.0) - 0.5 * _LOG_2PI - 0.5 * tau ** 2 + u
        return lp
    s = np.asarray(w.prior_scale, dtype=np.float64)[None, :]
    return np.sum(-0.5 * _LOG_2PI - np.log(s) - 0.5 * (theta / s) ** 2, axis=1)


def grad_log_prior(w, theta: np.ndarray) -> np.ndarray:
    if w.family == HIER_GAUSSIAN:
        g = -theta.copy()
        for j in (w.p + 1, w.p + 2):
            g[:, j] = -np.exp(2.0 * theta[:, j]) / HIER_SCALE_VAR + 1.0
        return g
    if w.family == HIER_LOGISTIC:
        g = -theta.copy()
        u = theta[:, w.p + 1]
        g[:, w.p + 1] = -np.exp(2.0 * u) + 1.0
        return g
    s = np.asarray(w.prior_scale, dtype=np.float64)[None, :]
    return -theta / s ** 2


def role_masks(roles: np.ndarray, fold_of_chain: np.ndarray):
    """Train and test indicators [n, C] for the chains' folds."""
    r = roles[fold_of_chain].T
    return (r == ROLE_TRAIN).astype(np.float64), (r == ROLE_TEST).astype(np.float64)


def log_density(w, theta: np.ndarray, roles: np.ndarray, fold_of_chain: np.ndarray) -> np.ndarray:
    train, _ = role_masks(roles, fold_of_chain)
    eta = linear_predictor(w, theta)
    return log_prior(w, theta) + np.sum(train * _loglik(w, theta, eta), axis=0)


def grad_log_density(w, theta: np.ndarray, roles: np.ndarray,
                     fold_of_chain: np.ndarray) -> np.ndarray:
    train, _ = role_masks(roles, fold_of_chain)
    eta = linear_predictor(w, theta)
    if w.family == HIER_GAUSSIAN:
        sy = _sigma_y(w, theta)[None, :]
        r = train * (w.y[:, None] - eta) / sy ** 2                     # dl/deta, [n, C]
    else:
        r = train * dloglik_deta(w.family, w.y[:, None], eta, w.sigma)   # [n, C]
    if w.family in HIER_FAMILIES:
        beta, mu, u, z = _split_hier(w, theta)
        z0 = theta.shape[1] - w.n_groups
        tau = np.exp(u)
        g = np.zeros_like(theta)
        g[:, :w.p] = r.T @ w.X
        g[:, w.p] = r.sum(axis=0)
        onehot = np.zeros((w.n, w.n_groups))
        onehot[np.arange(w.n), w.group_of] = 1.0
        per_group = r.T @ onehot                                         # [C, G]
        g[:, z0:] = tau[:, None] * per_group
        g[:, w.p + 1] = tau * np.sum(per_group * z, axis=1)
        if w.family == HIER_GAUSSIAN:
            # d/du_y of sum_train (-u_y - (y - eta)^2 e^{-2 u_y} / 2)
            g[:, w.p + 2] = np.sum(train * ((w.y[:, None] - eta) ** 2 / sy ** 2 - 1.0), axis=0)
        return g + grad_log_prior(w, theta)
    return r.T @ w.X + grad_log_prior(w, theta)


def log_pred(w, theta: np.ndarray, roles: np.ndarray, fold_of_chain: np.ndarray) -> np.ndarray:
    """s_c = joint log density of fold k's test rows given theta_c."""
    _, test = role_masks(roles, fold_of_chain)
    eta = linear_predictor(w, theta)
    return np.sum(test * _loglik(w, theta, eta), axis=0)
