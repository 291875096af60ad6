"""PCV estimates and diagnostics from the online accumulators and from stored draws.

TEST INFRASTRUCTURE ONLY (see the package header).

Per fold k with L chains of N post-warm-up draws, f = e^s, a = floor(N/b)
complete batches of b draws:

  elpd_k   = log( (1/LN) sum_l sum_n e^{s} )                  (eqs est-e, cv-score)
  elpd     = sum_k elpd_k
  sigma2_k = b/(La - 1) sum_l sum_h (fbar_lh - fbar)^2        (eq bmvar, batch means;
             fbar = mean of the La batch means)
  Var(fhat_k) = sigma2_k / (LN)                                (eq clt)
  MCSE(elpd_k) = sqrt(Var(fhat_k)) / fhat_k;  MCSE(elpd) = sqrt(sum_k Var/fhat^2)  (eq mc-var)
  s2_k     = pooled sample variance of the LN draws of f
  ESS_k    = LN s2_k / sigma2_k;  ESS = LN (sum_k s2_k/fhat_k^2) / (sum_k sigma2_k/fhat_k^2)
                                                               (Section 4.1)
  Rhat_k   = sqrt((N-1)/N + B/(N W)),  W = mean_l var_l(s),
             B = N/(L-1) sum_l (sbar_l - sbar)^2               (eq rhat; Section 4.2)
  Rhat_max = max_k Rhat_k                                      (eq rhat-max)

Readings (the closing formulas printed in Appendix A.2 are garbled):
the batch-means variance uses the mean of batch means and the factor b/(La-1)
of eq bmvar; s2 pools all LN draws (the printed version centres each chain
separately); the delta-method MCSE is sqrt(sum_k sigma2_k/fhat_k^2 / LN),
i.e. the printed 1/(NL) prefactor is not applied twice.  Every e^x is taken
relative to the fold's largest log term so nothing under- or overflows.

from_accumulators() evaluates these from the online state; two_pass() from the
full array of stored draws with textbook formulas.  Their agreement, and the
closed-form checks in tests/, pin this module.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import logsumexp

from . import philox


def _chan_merge(n_a, mean_a, m2_a, n_b, mean_b, m2_b):
    n = n_a + n_b
    with np.errstate(invalid="ignore", divide="ignore"):
        delta = mean_b - mean_a
        mean = np.where(n > 0, mean_a + delta * (n_b / np.maximum(n, 1)), 0.0)
        m2 = m2_a + m2_b + np.where(n > 0, delta * delta * n_a * n_b / np.maximum(n, 1), 0.0)
    return n, mean, m2


def merge_blocks(blk_n, blk_mean, blk_m2):
    """Combine per-block Welford states [..., D] into per-chain (n, mean, M2)."""
    n = np.zeros(blk_n.shape[:-1])
    mean = np.zeros(blk_n.shape[:-1])
    m2 = np.zeros(blk_n.shape[:-1])
    for dd in range(blk_n.shape[-1]):
        n, mean, m2 = _chan_merge(n, mean, m2, blk_n[..., dd].astype(np.float64),
                                  blk_mean[..., dd], blk_m2[..., dd])
    return n, mean, m2


def chain_moments(acc):
    """Per-chain (n, mean, M2) of s over all blocks, from either block mode.
    Shifted sums give the mean relative to C_k, which Rhat does not see."""
    if getattr(acc, "mode", 0) == 1:
        n = acc.blk_n.sum(axis=-1).astype(np.float64)
        y = acc.blk_mean.sum(axis=-1)
        y2 = acc.blk_m2.sum(axis=-1)
        with np.errstate(invalid="ignore", divide="ignore"):
            mean = np.where(n > 0, y / np.maximum(n, 1), 0.0)
            m2 = y2 - np.where(n > 0, y * y / np.maximum(n, 1), 0.0)
        return n, mean, m2
    return merge_blocks(acc.blk_n, acc.blk_mean, acc.blk_m2)


def rhat_from_moments(N, chain_mean, chain_m2):
    """Rhat of one fold from per-chain means [L] and M2 [L] (N draws each)."""
    L = chain_mean.shape[-1]
    W = np.mean(chain_m2 / (N - 1.0), axis=-1)
    grand = np.mean(chain_mean, axis=-1, keepdims=True)
    B = N / (L - 1.0) * np.sum((chain_mean - grand) ** 2, axis=-1)
    return np.sqrt((N - 1.0) / N + B / (N * W))


def _fold_terms(logf_sum, log2_sum, n_terms, K, L):
    """log of (sum e^x) and the pooled-variance bracket, per fold, stably."""
    a = logf_sum.reshape(K, L)
    a2 = log2_sum.reshape(K, L)
    m = np.max(a, axis=1)
    s1 = np.sum(np.exp(a - m[:, None]), axis=1)
    s2 = np.sum(np.exp(a2 - 2.0 * m[:, None]), axis=1)
    bracket = s2 - s1 * s1 / n_terms          # = e^{-2m} * (sum x^2 - (sum x)^2 / n)
    return m, s1, bracket


def from_accumulators(acc, K: int, L: int, b: int) -> dict:
    N = acc.n_draws
    out = {"n_draws": N}
    C = K * L
    U_all = np.logaddexp(acc.U, acc.Z)
    # elpd
    log_total = logsumexp(U_all.reshape(K, L), axis=1)
    elpd_k = log_total - math.log(L * N) if N > 0 else np.full(K, np.nan)
    out["elpd_fold"] = elpd_k
    out["elpd"] = float(np.sum(elpd_k))
    # Rhat
    n, mean, m2 = chain_moments(acc)
    if N >= 2:
        rk = rhat_from_moments(float(N), mean.reshape(K, L), m2.reshape(K, L))
    else:
        rk = np.full(K, np.nan)
    out["rhat_fold"] = rk
    out["rhat_max"] = float(np.max(rk))
    # pooled variance of f = e^s, relative to fhat^2
    mU, t1, brU = _fold_terms(U_all, acc.U2, L * N, K, L)
    # log fhat = mU + log(t1) - log(LN)
    log_fhat = mU + np.log(t1) - math.log(L * N)
    with np.errstate(divide="ignore", invalid="ignore"):
        s2_rel = np.exp(2.0 * mU + np.log(np.maximum(brU, 0.0)) - math.log(L * N - 1.0)
                        - 2.0 * log_fhat)
    # batch-means variance relative to fhat^2
    a = N // b
    if a >= 1 and L * a > 1:
        mV, v1, brV = _fold_terms(acc.V, acc.V2, L * a, K, L)
        with np.errstate(divide="ignore", invalid="ignore"):
            sig2_rel = np.exp(math.log(b) - math.log(L * a - 1.0) + 2.0 * mV
                              + np.log(np.maximum(brV, 0.0)) - 2.0 * log_fhat)
    else:
        sig2_rel = np.full(K, np.nan)
    var_rel = sig2_rel / (L * N)
    out["sigma2_rel_fold"] = sig2_rel
    out["s2_rel_fold"] = s2_rel
    out["mcse_fold"] = np.sqrt(var_rel)
    out["mcse"] = float(np.sqrt(np.sum(var_rel)))
    with np.errstate(divide="ignore", invalid="ignore"):
        out["ess_fold"] = L * N * s2_rel / sig2_rel
        out["ess"] = float(L * N * np.sum(s2_rel) / np.sum(sig2_rel))
    out["accept_rate"] = float(np.sum(acc.n_accept) / max(1, C * N))
    out["n_divergent"] = int(np.sum(acc.n_divergent))
    return out


def two_pass(draws: np.ndarray, K: int, L: int, b: int) -> dict:
    """The same quantities from stored draws s[C, N] with textbook formulas."""
    C, N = draws.shape
    s = draws.reshape(K, L, N)
    out = {"n_draws": N}
    elpd_k = logsumexp(s.reshape(K, L * N), axis=1) - math.log(L * N)
    out["elpd_fold"] = elpd_k
    out["elpd"] = float(np.sum(elpd_k))
    chain_mean = s.mean(axis=2)
    chain_var = s.var(axis=2, ddof=1)
    W = chain_var.mean(axis=1)
    B = N * chain_mean.var(axis=1, ddof=1)
    rk = np.sqrt((N - 1.0) / N + B / (N * W))
    out["rhat_fold"] = rk
    out["rhat_max"] = float(rk.max())
    # f relative to the fold's max draw
    mx = s.reshape(K, -1).max(axis=1)
    f = np.exp(s - mx[:, None, None])
    fhat = f.reshape(K, -1).mean(axis=1)
    s2 = f.reshape(K, -1).var(axis=1, ddof=1)
    a = N // b
    bm = f[:, :, :a * b].reshape(K, L, a, b).mean(axis=3)          # batch means
    gbar = bm.reshape(K, -1).mean(axis=1)
    sig2 = b / (L * a - 1.0) * np.sum((bm - gbar[:, None, None]) ** 2, axis=(1, 2))
    out["sigma2_rel_fold"] = sig2 / fhat ** 2
    out["s2_rel_fold"] = s2 / fhat ** 2
    var_rel = sig2 / (L * N) / fhat ** 2
    out["mcse_fold"] = np.sqrt(var_rel)
    out["mcse"] = float(np.sqrt(var_rel.sum()))
    out["ess_fold"] = L * N * s2 / sig2
    out["ess"] = float(L * N * np.sum(s2 / fhat ** 2) / np.sum(sig2 / fhat ** 2))
    return out


def shuffle_benchmark(acc, K: int, L: int, D: int, R: int, seed: int, fold_offset: int = 0):
    """Rhat_max under block shuffling (Section 4.2, Fig. 4; Algorithm A2, last loop).

    For replicate r every chain slot l is rebuilt from D blocks, block d taken
    from a chain drawn uniformly with replacement among the fold's L chains;
    Rhat is recomputed on the rebuilt chains.  Returns rhat_rep[K, R] and the
    replicate maxima over folds [R].
    """
    N = float(acc.n_draws)
    bn = acc.blk_n.reshape(K, L, D)
    bm = acc.blk_mean.reshape(K, L, D)
    b2 = acc.blk_m2.reshape(K, L, D)
    out = np.empty((K, R))
    for k in range(K):
        for r in range(R):
            idx = philox.shuffle_indices(seed, fold_offset + k, r, L, D)   # [L, D]
            n = np.zeros(L)
            mean = np.zeros(L)
            m2 = np.zeros(L)
            if getattr(acc, "mode", 0) == 1:
                # shifted sums: a rebuilt chain's Y and Y2 are sums of its blocks'
                y = np.zeros(L)
                y2 = np.zeros(L)
                for dd in range(D):
                    src = idx[:, dd]
                    n = n + bn[k, src, dd]
                    y = y + bm[k, src, dd]
                    y2 = y2 + b2[k, src, dd]
                mean = y / n
                m2 = y2 - y * y / n
            else:
                for dd in range(D):
                    src = idx[:, dd]
                    n, mean, m2 = _chan_merge(n, mean, m2, bn[k, src, dd].astype(np.float64),
                                              bm[k, src, dd], b2[k, src, dd])
            out[k, r] = rhat_from_moments(N, mean, m2)
    return out, out.max(axis=0)


def compare(elpd_fold_a, mcse_fold_a, elpd_fold_b, mcse_fold_b) -> dict:
    """Pairwise comparison of models A and B evaluated on the same folds.

      Delta_k  = S_A,k - S_B,k,   Delta = sum_k Delta_k                       (eq sel-cv)
      sigma2   = 1/(K-1) sum_k (Delta_k - Delta/K)^2
      Pr(A > B) ~ Phi(Delta / sqrt(K sigma2))                                  (eq norm-approx)
      MCSE(Delta)^2 = sum over both models and all folds of MCSE(S_M,k)^2      (eq mc-var)

    Reading: with Delta = 0 and sigma2 = 0 the ratio is undefined; it is taken
    as Pr = 1/2 (no evidence either way), and sigma2 = 0 with Delta != 0 gives
    Pr = 1 or 0 by the sign of Delta.
    """
    dk = np.asarray(elpd_fold_a, dtype=np.float64) - np.asarray(elpd_fold_b, dtype=np.float64)
    K = dk.size
    delta = float(np.sum(dk))
    sigma2 = float(np.sum((dk - delta / K) ** 2) / (K - 1)) if K > 1 else float("nan")
    if sigma2 > 0:
        prob = 0.5 * math.erfc(-delta / math.sqrt(2.0 * K * sigma2))
    else:
        prob = 0.5 if delta == 0 else (1.0 if delta > 0 else 0.0)
    mcse = math.sqrt(float(np.sum(np.square(mcse_fold_a)) + np.sum(np.square(mcse_fold_b))))
    return {"delta": delta, "delta_fold": dk, "sigma2": sigma2, "prob_a_better": prob, "mcse": mcse}
