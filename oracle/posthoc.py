"""Post-hoc diagnostics from stored log predictive draws (Algorithm 1's output).

TEST INFRASTRUCTURE ONLY (see the package header).

Algorithm 1 keeps every post-warm-up draw s[k, l, i], so the conventional
workflow of diagnostics after inference applies (Section 3, the discussion
of online versus stored draws).  Besides the estimates and the paper's R-hat
(two_pass in diagnostics.py) this module gives two standard cross-checks of
convergence for the draws of one fold (L chains x N draws):

  split R-hat: every chain cut into its first and second half (the middle
    draw dropped when N is odd), then the R-hat of eq rhat over the 2L
    half-chains;
  rank-normalised split R-hat (Vehtari, Gelman, Simpson, Carpenter and
    Buerkner, 2021): the fold's LN draws replaced by normal scores
    Phi^-1((r - 3/8) / (LN + 1/4)) of their ranks r (ties get the average
    rank), then split R-hat; the same for the folded draws |s - median(s)|;
    the larger of the two.
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def rhat_chains(x: np.ndarray) -> float:
    """R-hat of eq rhat for chains x[m, n] (m chains of n draws)."""
    m, n = x.shape
    W = np.mean(np.var(x, axis=1, ddof=1))
    B = n * np.var(np.mean(x, axis=1), ddof=1)
    return float(np.sqrt((n - 1.0) / n + B / (n * W)))


def split_chains(x: np.ndarray) -> np.ndarray:
    n = x.shape[1]
    h = n // 2
    return np.concatenate([x[:, :h], x[:, n - h:]], axis=0)


def split_rhat(x: np.ndarray) -> float:
    return rhat_chains(split_chains(x))


def normal_scores(x: np.ndarray) -> np.ndarray:
    r = stats.rankdata(x, method="average").reshape(x.shape)
    return stats.norm.ppf((r - 0.375) / (x.size + 0.25))


def rank_rhat(x: np.ndarray) -> float:
    bulk = split_rhat(normal_scores(x))
    folded = split_rhat(normal_scores(np.abs(x - np.median(x))))
    return max(bulk, folded)


def fold_rhats(draws: np.ndarray, K: int, L: int) -> dict:
    """Per fold: the paper's R-hat, split R-hat and rank-normalised R-hat."""
    C, N = draws.shape
    s = draws.reshape(K, L, N)
    out = {"rhat_fold": np.array([rhat_chains(s[k]) for k in range(K)]),
           "split_rhat_fold": np.array([split_rhat(s[k]) for k in range(K)]),
           "rank_rhat_fold": np.array([rank_rhat(s[k]) for k in range(K)])}
    for key in list(out):
        out[key.replace("_fold", "_max")] = float(np.max(out[key]))
    return out
