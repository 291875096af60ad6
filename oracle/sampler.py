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

Block statistics for Rhat come in two modes (rhat_mode of the workload):
  0  Welford: running (count, mean, M2) of s per block, Chan-merged later;
  1  shifted sums, as Algorithm A2 writes them: during warm-up every draw of
     every chain of fold k adds to the fold's centring constant
     C_k = mean of the fold's L*N_wu warm-up log predictive draws; afterwards
     each block keeps Y = sum (s - C_k) and Y2 = sum (s - C_k)^2.
Both give the same within/between-chain variances (the shift cancels); the
Welford form avoids the cancellation in Y2 - Y^2/N.  Draws past D*G*b go to
the last block.  A
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

from . import folds, hmc, scores


RHAT_WELFORD, RHAT_SHIFTED_SUMS = 0, 1


@dataclasses.dataclass
class Accumulators:
    Z: np.ndarray
    U: np.ndarray
    U2: np.ndarray
    V: np.ndarray
    V2: np.ndarray
    blk_n: np.ndarray      # [C, D] int64
    blk_mean: np.ndarray   # [C, D] Welford mean of s         | shifted: Y  = sum (s - C_k)
    blk_m2: np.ndarray     # [C, D] Welford M2 of s           | shifted: Y2 = sum (s - C_k)^2
    n_draws: int = 0
    n_accept: Optional[np.ndarray] = None
    n_divergent: Optional[np.ndarray] = None
    mode: int = RHAT_WELFORD
    wsum: Optional[np.ndarray] = None      # [C] sum of warm-up draws of s (shifted mode)
    n_wu: int = 0                          # warm-up draws summed so far
    center: Optional[np.ndarray] = None    # [C] C_k of each chain's fold (shifted mode)

    @staticmethod
    def empty(C: int, D: int, mode: int = RHAT_WELFORD) -> "Accumulators":
        ninf = lambda: np.full(C, -np.inf)
        return Accumulators(Z=ninf(), U=ninf(), U2=ninf(), V=ninf(), V2=ninf(),
                            blk_n=np.zeros((C, D), dtype=np.int64),
                            blk_mean=np.zeros((C, D)), blk_m2=np.zeros((C, D)),
                            n_draws=0, n_accept=np.zeros(C, dtype=np.int64),
                            n_divergent=np.zeros(C, dtype=np.int64), mode=mode,
                            wsum=np.zeros(C), n_wu=0, center=np.zeros(C))


def warmup_draw(acc: Accumulators, s: np.ndarray) -> None:
    """Shifted mode: a warm-up draw adds to its fold's centring constant."""
    if acc.mode == RHAT_SHIFTED_SUMS:
        acc.wsum += s
        acc.n_wu += 1


def fix_center(acc: Accumulators, L: int) -> None:
    """Shifted mode, end of warm-up: C_k = mean of the fold's L * N_wu warm-up
    draws (0 when there was no warm-up), copied to each of its chains."""
    if acc.mode == RHAT_SHIFTED_SUMS:
        K = acc.wsum.size // L
        ck = acc.wsum.reshape(K, L).sum(axis=1) / (L * acc.n_wu) if acc.n_wu > 0 else np.zeros(K)
        acc.center = np.repeat(ck, L)


def accumulate(acc: Accumulators, s: np.ndarray, i: int, b: int, G: int, D: int) -> None:
    """Fold post-warm-up draw number i (0-based) into the accumulators."""
    acc.Z = np.logaddexp(acc.Z, s)
    acc.U2 = np.logaddexp(acc.U2, 2.0 * s)
    blk = min(i // (G * b), D - 1)
    acc.blk_n[:, blk] += 1
    if acc.mode == RHAT_SHIFTED_SUMS:
        dv = s - acc.center
        acc.blk_mean[:, blk] += dv
        acc.blk_m2[:, blk] += dv * dv
    else:
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
    score_acc: Optional[scores.ScoreAccumulators] = None   # HS / DSS sums (workload flag `scores`)
    score_rows: Optional[np.ndarray] = None                # [C, vmax] test rows per chain
    draws: Optional[np.ndarray] = None  # [C, N] stored s (when requested)
    accepted: Optional[np.ndarray] = None   # [C, iters] accept decisions (when requested)


def start(w) -> Run:
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    st = hmc.initial_state(w, roles, foc)
    acc = Accumulators.empty(w.C, w.n_blocks, getattr(w, "rhat_mode", RHAT_WELFORD))
    if w.n_warmup == 0:
        fix_center(acc, w.L)
    run = Run(state=st, acc=acc, t=0)
    flags = getattr(w, "scores", 0)
    if flags:
        run.score_rows = scores.rows_of_chains(roles, w.L)
        run.score_acc = scores.ScoreAccumulators(w.C, run.score_rows.shape[1], flags)
    return run


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
        if t < w.n_warmup:
            warmup_draw(run.acc, run.state.s)
            if t + 1 == w.n_warmup:
                fix_center(run.acc, w.L)
        else:
            accumulate(run.acc, run.state.s, t - w.n_warmup, b, G, D)
            if run.score_acc is not None:
                r = run.score_rows
                yt = np.where(r >= 0, w.y[np.maximum(r, 0)], np.nan)
                scores.accumulate(w, run.score_acc, scores.test_eta(w, run.state.q, r), yt, t)
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
