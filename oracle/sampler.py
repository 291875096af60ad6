"""Online single-model LogS sampler: all folds and chains at once.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows Algorithm A2 (Appendix A.2): after N_wu discarded warm-up
transitions, draws are grouped into D shuffle blocks of G batches of b draws.
For every chain, with s the log predictive of the fold's test set at the
current draw:

  per draw:        Z  <- logaddexp(Z, s)            (log sum of e^s in this batch)
                   U2 <- logaddexp(U2, 2 s)         (log sum of e^{2s})
                   Welford update of (count, mean, M2) of s for the current block
  at a batch end:  U  <- logaddexp(U, Z)            (log sum of e^s)
                   V  <- logaddexp(V, Z - log b)    (log sum of batch means of e^s)
                   V2 <- logaddexp(V2, 2Z - 2 log b)
                   Z  <- -inf

Reading: the paper accumulates shifted sums of s and s^2 per block around a
warm-up centring constant (Appendix A.1); Welford's running mean and M2 per
block give the same within/between-chain variances without the centring
constant and without cancellation.  Draws past D*G*b go to the last block.  A
partial batch is part of U (through Z), U2 and the block statistics, and is
left out of V, V2.  Accept and divergence counts cover post-warm-up
transitions.

Pins: accumulators against two-pass statistics of the stored draws, elpd of
the conjugate Gaussian against its closed form (tests/test_oracle_sampler.py).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import folds, hmc


@dataclasses.dataclass
class Accumulators:
    Z: np.ndarray
    U: np.ndarray
    U2: np.ndarray
    V: np.ndarray
    V2: np.ndarray
    blk_n: np.ndarray      # [C, D] int64
    blk_mean: np.ndarray   # [C, D]
    blk_m2: np.ndarray     # [C, D]
    n_draws: int = 0
    n_accept: Optional[np.ndarray] = None
    n_divergent: Optional[np.ndarray] = None

    @staticmethod
    def empty(C: int, D: int) -> "Accumulators":
        ninf = lambda: np.full(C, -np.inf)
        return Accumulators(Z=ninf(), U=ninf(), U2=ninf(), V=ninf(), V2=ninf(),
                            blk_n=np.zeros((C, D), dtype=np.int64),
                            blk_mean=np.zeros((C, D)), blk_m2=np.zeros((C, D)),
                            n_draws=0, n_accept=np.zeros(C, dtype=np.int64),
                            n_divergent=np.zeros(C, dtype=np.int64))


def accumulate(acc: Accumulators, s: np.ndarray, i: int, b: int, G: int, D: int) -> None:
    """Fold post-warm-up draw number i (0-based) into the accumulators."""
    acc.Z = np.logaddexp(acc.Z, s)
    acc.U2 = np.logaddexp(acc.U2, 2.0 * s)
    blk = min(i // (G * b), D - 1)
    acc.blk_n[:, blk] += 1
    n = acc.blk_n[:, blk].astype(np.float64)
    delta = s - acc.blk_mean[:, blk]
    acc.blk_mean[:, blk] += delta / n
    acc.blk_m2[:, blk] += delta * (s - acc.blk_mean[:, blk])
    if (i + 1) % b == 0:
        acc.U = np.logaddexp(acc.U, acc.Z)
        acc.V = np.logaddexp(acc.V, acc.Z - math.log(b))
        acc.V2 = np.logaddexp(acc.V2, 2.0 * acc.Z - 2.0 * math.log(b))
        acc.Z = np.full_like(acc.Z, -np.inf)
    acc.n_draws = i + 1


@dataclasses.dataclass
class Run:
    state: hmc.ChainState
    acc: Accumulators
    t: int                              # next global iteration
    draws: Optional[np.ndarray] = None  # [C, N] stored s (when requested)
    accepted: Optional[np.ndarray] = None   # [C, iters] accept decisions (when requested)


def start(w) -> Run:
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    st = hmc.initial_state(w, roles, foc)
    return Run(state=st, acc=Accumulators.empty(w.C, w.n_blocks), t=0)


def advance(w, run: Run, n_iter: int, store_draws: bool = False,
            store_accepts: bool = False) -> Run:
    """Advance every chain n_iter transitions (Algorithm A2's loops, flattened)."""
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    chain_ids = w.chain_offset + np.arange(w.C)
    b, G, D = w.batch_size, w.batches_per_block, w.n_blocks
    draws = [] if store_draws else None
    accs = [] if store_accepts else None
    for _ in range(n_iter):
        t = run.t
        run.state, accepted, divergent = hmc.transition(w, run.state, t, roles, foc, chain_ids)
        if store_accepts:
            accs.append(accepted.copy())
        if t >= w.n_warmup:
            accumulate(run.acc, run.state.s, t - w.n_warmup, b, G, D)
            run.acc.n_accept += accepted
            run.acc.n_divergent += divergent
            if store_draws:
                draws.append(run.state.s.copy())
        run.t = t + 1
    if store_draws:
        new = np.stack(draws, axis=1) if draws else np.zeros((w.C, 0))
        run.draws = new if run.draws is None else np.concatenate([run.draws, new], axis=1)
    if store_accepts:
        new = np.stack(accs, axis=1)
        run.accepted = new if run.accepted is None else np.concatenate([run.accepted, new], axis=1)
    return run


def run_all(w, n_iter: Optional[int] = None, store_draws: bool = False,
            store_accepts: bool = False) -> Run:
    run = start(w)
    return advance(w, run, w.n_iter if n_iter is None else n_iter, store_draws, store_accepts)
