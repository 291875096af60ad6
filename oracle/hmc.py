"""One Hamiltonian Monte Carlo transition per chain, fixed trajectory length.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3.3 runs every fold's chains in lock-step with HMC (Neal 2011): a
fixed number S of leapfrog steps of size eps, with a shared diagonal inverse
mass matrix, reused from the full-data fit (Section 3.1).  One transition:

  1. draw momentum p ~ N(0, M), M = diag(1 / inv_mass)   (p = z / sqrt(inv_mass))
  2. H0 = -log pi(q) + K(p),  K(p) = 1/2 sum_j inv_mass_j p_j^2
  3. leapfrog: p += eps/2 grad(q); then S times { q += eps inv_mass p;
     p += eps grad(q) }, the last momentum update being eps/2
  4. H1 = -log pi(q') + K(p');  accept with probability min(1, exp(H0 - H1)):
     accept iff H0 - H1 is finite and log u < H0 - H1 (u ~ U(0,1))
  5. a transition is divergent if H0 - H1 is not finite or H1 - H0 > 1000

The gradient at the current state is carried between transitions, so one
transition costs S gradient evaluations.  Random numbers come from the Philox
streams in philox.py, keyed by global chain id and iteration.

Pins: leapfrog reversibility, second-order energy error, exact linear map for
a Gaussian target, stationarity against the conjugate posterior
(tests/test_oracle_hmc.py).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import model, philox

DIVERGENCE_THRESHOLD = 1000.0


@dataclasses.dataclass
class ChainState:
    q: np.ndarray        # [C, d]
    logp: np.ndarray     # [C]
    grad: np.ndarray     # [C, d]
    s: np.ndarray        # [C]  log predictive at q
    alpha: Optional[np.ndarray] = None   # [C] acceptance statistic of the last transition


def initial_state(w, roles, fold_of_chain, q0=None) -> ChainState:
    q = np.array(w.init_pos if q0 is None else q0, dtype=np.float64)
    return ChainState(q=q,
                      logp=model.log_density(w, q, roles, fold_of_chain),
                      grad=model.grad_log_density(w, q, roles, fold_of_chain),
                      s=model.log_pred(w, q, roles, fold_of_chain))


def leapfrog(w, q, p, grad, n_steps, eps, roles, fold_of_chain):
    """S leapfrog steps from (q, p) with grad = grad log pi(q).

    Returns (q', p', grad(q'), log pi(q')).
    """
    inv_mass = np.asarray(w.inv_mass, dtype=np.float64)[None, :]
    q = q.copy()
    p = p + 0.5 * eps * grad
    g = grad
    for step in range(n_steps):
        q = q + eps * inv_mass * p
        g = model.grad_log_density(w, q, roles, fold_of_chain)
        p = p + (eps if step < n_steps - 1 else 0.5 * eps) * g
    logp = model.log_density(w, q, roles, fold_of_chain)
    return q, p, g, logp


def kinetic(w, p):
    return 0.5 * np.sum(np.asarray(w.inv_mass)[None, :] * p * p, axis=1)


def transition(w, st: ChainState, t: int, roles, fold_of_chain, chain_ids):
    """One HMC transition of every chain at global iteration t.

    Returns (new state, accepted[C] bool, divergent[C] bool).
    """
    z = philox.momentum_normals(w.seed, chain_ids, t, st.q.shape[1])
    p0 = z / np.sqrt(np.asarray(w.inv_mass))[None, :]
    h0 = -st.logp + kinetic(w, p0)
    q1, p1, g1, logp1 = leapfrog(w, st.q, p0, st.grad, w.n_leapfrog, w.step_size,
                                 roles, fold_of_chain)
    with np.errstate(invalid="ignore", over="ignore"):
        h1 = -logp1 + kinetic(w, p1)
        log_ratio = h0 - h1
        u = philox.accept_uniforms(w.seed, chain_ids, t)
        finite = np.isfinite(log_ratio)
        accepted = finite & (np.log(u) < np.where(finite, log_ratio, -np.inf))
        divergent = (~finite) | (np.where(finite, -log_ratio, 0.0) > DIVERGENCE_THRESHOLD)
    a = accepted[:, None]
    q = np.where(a, q1, st.q)
    # acceptance statistic min(1, e^(H0 - H1)); 0 for a non-finite energy
    with np.errstate(over="ignore"):
        alpha = np.where(finite, np.minimum(1.0, np.exp(np.where(finite, log_ratio, 0.0))), 0.0)
    new = ChainState(q=q,
                     logp=np.where(accepted, logp1, st.logp),
                     grad=np.where(a, g1, st.grad),
                     s=st.s.copy(), alpha=alpha)
    if np.any(accepted):
        s_new = model.log_pred(w, q, roles, fold_of_chain)
        new.s = np.where(accepted, s_new, st.s)
    return new, accepted, divergent
