"""Per-fold row roles for cross-validation schemes.

TEST INFRASTRUCTURE ONLY (see the package header).

A CV scheme splits the rows into a test set and a training set per fold
(Section 2.2).  Appendix B selects each fold's rows with indicator masks so
that every fold is evaluated by the same branch-free program; its listing
marks training rows by "fold index differs from the fold id" and test rows by
"fold index equals the fold id".  hv-block CV (Racine 2000, cited in the
introduction) also drops h rows on each side of the test block from the
training set, so a row can be in neither set: roles are tri-state here.

  ROLE_EXCLUDED = 0, ROLE_TRAIN = 1, ROLE_TEST = 2

Encodings accepted:
  index      fold_index[n]: test in fold fold_index[n], train in every other
             fold (a value of -1 means train in every fold)
  intervals  per fold (test_lo, test_hi, excl_lo, excl_hi): rows in
             [test_lo, test_hi) are test, rows in [excl_lo, excl_hi) that are
             not test are excluded, all others are train
  dense      a K x n matrix of roles

Parity: pinned by direct enumeration on small cases (tests/test_oracle_model.py).
"""
from __future__ import annotations

import numpy as np

ROLE_EXCLUDED = 0
ROLE_TRAIN = 1
ROLE_TEST = 2


def roles_from_index(fold_index, K: int) -> np.ndarray:
    fi = np.asarray(fold_index)
    is_test = fi[None, :] == np.arange(K)[:, None]
    return np.where(is_test, ROLE_TEST, ROLE_TRAIN).astype(np.int8)


def roles_from_intervals(intervals, n: int) -> np.ndarray:
    iv = np.asarray(intervals)
    K = iv.shape[0]
    roles = np.full((K, n), ROLE_TRAIN, dtype=np.int8)
    for k in range(K):
        lo, hi, elo, ehi = (int(v) for v in iv[k])
        roles[k, elo:ehi] = ROLE_EXCLUDED
        roles[k, lo:hi] = ROLE_TEST
    return roles


def roles_of(w) -> np.ndarray:
    """K x n role matrix of a workload-like object (fold_kind 0/1/2)."""
    if w.fold_kind == 0:
        return roles_from_index(w.fold_index, w.K)
    if w.fold_kind == 1:
        return roles_from_intervals(w.intervals, w.n)
    return np.asarray(w.roles, dtype=np.int8).copy()
