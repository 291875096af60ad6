"""Full-data tuning by window adaptation, and chain starts from full-data draws.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3.1 (efficient warm-up) and the workflow's Steps 1-2: every fold's
kernel reuses the step size and inverse mass matrix of the full-data
inference, and each fold's chains start at random draws of the full-data
posterior.  The paper names Stan's window adaptation as its example and
gives no constants, so the constants of Stan's published algorithm are used.

Full data: one "fold" whose rows are all training rows (fold id -1).

Schedule of n adaptation transitions (counts of transitions):
  an initial fast buffer of 75, a final fast buffer of 50 and a first slow
  window of 25; when 75 + 25 + 50 > n, the buffers are 15% and 10% of n and
  the single slow window the rest.  Slow windows double in length; a window
  is stretched to end where the final buffer starts when the next (doubled)
  window would not fit before it.  For n = 1000: slow windows end after
  transitions 100, 150, 250, 450 and 950.

Step size, every transition: dual averaging (Hoffman and Gelman, 2014) of
the chains' mean acceptance statistic a = mean_c min(1, e^(H0 - H1)) (0 for
a non-finite energy) toward the target delta, with gamma = 0.05, t0 = 10,
kappa = 0.75:
    m <- m + 1
    Hbar <- (1 - 1/(m + t0)) Hbar + (delta - a) / (m + t0)
    log eps <- mu - sqrt(m) / gamma * Hbar
    log epsbar <- m^-kappa log eps + (1 - m^-kappa) log epsbar
starting from mu = log(10 eps), Hbar = 0, log epsbar = 0, m = 0, and
restarted that way after every inverse-mass update.  After the last
transition eps = exp(log epsbar).

Inverse mass, diagonal: during a slow window, the positions of all chains
after every transition feed a per-coordinate variance (n samples = chains x
transitions of the window); at its end
    Minv_j = n / (n + 5) * var_j + 1e-3 * 5 / (n + 5).

Pins (tests/test_oracle_adapt.py): the schedule for n = 1000 against the
published default windows (tests/golden/stan_windows.txt); dual averaging
against the analytic step size of a closed-form acceptance curve; the
adapted inverse mass of the conjugate Gaussian against its exact posterior
variances; the post-adaptation acceptance rate near the target.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import folds, hmc, philox

DA_GAMMA, DA_T0, DA_KAPPA = 0.05, 10.0, 0.75
INIT_BUFFER, TERM_BUFFER, BASE_WINDOW = 75, 50, 25


def buffers(n: int):
    """(initial fast buffer, final fast buffer, first slow window) for n transitions."""
    init, term, win = INIT_BUFFER, TERM_BUFFER, BASE_WINDOW
    if init + win + term > n:
        init = int(0.15 * n)
        term = int(0.1 * n)
        win = n - init - term
    return init, term, win


def slow_window_ends(n: int):
    """Transition counts after which a slow window ends (the inverse mass is updated)."""
    init, term, win = buffers(n)
    if win <= 0:
        return []
    last = n - term                      # slow windows end by here
    ends = []
    start, size = init, win
    while start < last:
        end = start + size
        if end + 2 * size > last:        # the next, doubled window would not fit
            end = last
        ends.append(end)
        start, size = end, 2 * size
    return ends


@dataclasses.dataclass
class DualAveraging:
    mu: float
    log_eps: float
    hbar: float = 0.0
    log_epsbar: float = 0.0
    m: int = 0

    @staticmethod
    def start(eps: float) -> "DualAveraging":
        return DualAveraging(mu=math.log(10.0 * eps), log_eps=math.log(eps))

    def update(self, accept_stat: float, delta: float) -> None:
        self.m += 1
        w = 1.0 / (self.m + DA_T0)
        self.hbar = (1.0 - w) * self.hbar + w * (delta - accept_stat)
        self.log_eps = self.mu - math.sqrt(self.m) / DA_GAMMA * self.hbar
        eta = self.m ** (-DA_KAPPA)
        self.log_epsbar = eta * self.log_eps + (1.0 - eta) * self.log_epsbar


def regularised_variance(samples: np.ndarray) -> np.ndarray:
    """Minv from samples [n, d] of one slow window."""
    n = samples.shape[0]
    var = np.var(samples, axis=0, ddof=1)
    return n / (n + 5.0) * var + 1e-3 * 5.0 / (n + 5.0)


def adapt(w, n_adapt: int, delta: float = 0.8, state: hmc.ChainState = None):
    """Window adaptation of workload w's step size and inverse mass over its
    chains (all folds of w share them).  Returns (w with the adapted
    step_size and inv_mass, final chain state, per-transition step sizes,
    per-transition mean acceptance statistics)."""
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    chain_ids = w.chain_offset + np.arange(w.C)
    st = hmc.initial_state(w, roles, foc) if state is None else state
    ends = slow_window_ends(n_adapt)
    slow_lo = buffers(n_adapt)[0]
    slow_hi = ends[-1] if ends else 0     # transitions [slow_lo, slow_hi) feed the variance
    da = DualAveraging.start(w.step_size)
    window = []
    eps_trace, acc_trace = [], []
    for t in range(n_adapt):
        w = dataclasses.replace(w, step_size=math.exp(da.log_eps))
        eps_trace.append(w.step_size)
        st, _, _ = hmc.transition(w, st, t, roles, foc, chain_ids)
        a = float(np.mean(st.alpha))
        acc_trace.append(a)
        da.update(a, delta)
        if slow_lo <= t < slow_hi:
            window.append(st.q.copy())
        if t + 1 in ends:
            minv = regularised_variance(np.concatenate(window, axis=0))
            w = dataclasses.replace(w, inv_mass=minv)
            da = DualAveraging.start(math.exp(da.log_eps))
            window = []
    w = dataclasses.replace(w, step_size=math.exp(da.log_epsbar))
    return w, st, np.array(eps_trace), np.array(acc_trace)


def init_positions(draws: np.ndarray, C: int, seed: int, chain_offset: int = 0) -> np.ndarray:
    """Starting positions [C, d] of the CV chains: chain c takes full-data draw
    init_draw_indices(seed, chain_offset + c) of draws [n_draws, d] (Step 2)."""
    idx = philox.init_draw_indices(seed, chain_offset + np.arange(C), draws.shape[0])
    return draws[idx].copy()
