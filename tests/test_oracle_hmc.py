"""Pins of the oracle's HMC transition (CPU only)."""
import numpy as np
import pytest

from oracle import closed_form, folds, hmc, model, philox
from paper_2310_07002_amd import workloads as W


@pytest.fixture(scope="module")
def c1():
    w = W.make_c1()
    return w, folds.roles_of(w)


def test_leapfrog_is_reversible(c1):
    w, roles = c1
    foc = np.arange(w.C) // w.L
    rng = np.random.default_rng(0)
    q0 = w.init_pos
    p0 = rng.normal(size=q0.shape) / np.sqrt(w.inv_mass)
    g0 = model.grad_log_density(w, q0, roles, foc)
    q1, p1, g1, _ = hmc.leapfrog(w, q0, p0, g0, 8, 0.1, roles, foc)
    q2, p2, _, _ = hmc.leapfrog(w, q1, -p1, g1, 8, 0.1, roles, foc)
    np.testing.assert_allclose(q2, q0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(-p2, p0, rtol=0, atol=1e-12)


def test_energy_error_is_second_order(c1):
    w, roles = c1
    foc = np.arange(w.C) // w.L
    rng = np.random.default_rng(1)
    q0 = w.init_pos
    p0 = rng.normal(size=q0.shape) / np.sqrt(w.inv_mass)
    lp0 = model.log_density(w, q0, roles, foc)
    g0 = model.grad_log_density(w, q0, roles, foc)
    errs = []
    for eps in (0.08, 0.04, 0.02):
        n = int(round(0.64 / eps))                 # fixed trajectory length
        q1, p1, _, lp1 = hmc.leapfrog(w, q0, p0, g0, n, eps, roles, foc)
        dh = (-lp1 + hmc.kinetic(w, p1)) - (-lp0 + hmc.kinetic(w, p0))
        errs.append(np.median(np.abs(dh)))
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


def test_leapfrog_equals_exact_linear_map(c1):
    """For a Gaussian target the leapfrog map is linear: check it against the
    matrix built from the closed-form posterior precision."""
    w, roles = c1
    k = 7
    m, V, A = closed_form.fold_posterior(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
    eps, S = 0.1, 8
    Minv = np.diag(w.inv_mass)
    d = w.p
    half = np.block([[np.eye(d), np.zeros((d, d))], [-0.5 * eps * A, np.eye(d)]])
    drift = np.block([[np.eye(d), eps * Minv], [np.zeros((d, d)), np.eye(d)]])
    T = np.eye(2 * d)
    for _ in range(S):
        T = half @ drift @ half @ T
    rng = np.random.default_rng(4)
    q0 = m + rng.normal(size=d) * 0.1
    p0 = rng.normal(size=d)
    g0 = model.grad_log_density(w, q0[None], roles, np.array([k]))
    q1, p1, _, _ = hmc.leapfrog(w, q0[None], p0[None], g0, S, eps, roles, np.array([k]))
    want = T @ np.concatenate([q0 - m, p0])
    np.testing.assert_allclose(q1[0] - m, want[:d], atol=1e-11)
    np.testing.assert_allclose(p1[0], want[d:], atol=1e-9)


def test_momentum_covariance_is_mass_matrix():
    inv_mass = np.array([0.5, 2.0, 0.01])
    z = philox.momentum_normals(11, np.arange(100000), 0, 3)
    p = z / np.sqrt(inv_mass)
    np.testing.assert_allclose(p.var(axis=0), 1.0 / inv_mass, rtol=0.02)


def test_hmc_leaves_conjugate_posterior_invariant(c1):
    """Chains started at exact posterior draws stay distributed as the posterior."""
    w, roles = c1
    k = 11
    m, V, _ = closed_form.fold_posterior(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1)
    C = 4000
    rng = np.random.default_rng(5)
    q0 = rng.multivariate_normal(m, V, size=C)
    foc = np.full(C, k)
    st = hmc.initial_state(w, roles, foc, q0=q0)
    ids = np.arange(C)
    for t in range(5):
        st, acc, div = hmc.transition(w, st, t, roles, foc, ids)
    z = np.linalg.solve(np.linalg.cholesky(V), (st.q - m).T).T
    assert np.all(np.abs(z.mean(axis=0)) < 4.5 / np.sqrt(C))
    np.testing.assert_allclose(np.cov(z.T), np.eye(w.p), atol=0.1)


def test_divergence_is_flagged_and_rejected(c1):
    w, roles = c1
    import dataclasses
    wb = dataclasses.replace(w, step_size=10.0)
    foc = np.arange(w.C) // w.L
    st = hmc.initial_state(wb, roles, foc)
    st2, acc, div = hmc.transition(wb, st, 0, roles, foc, np.arange(w.C))
    assert div.mean() > 0.9
    assert not np.any(acc & div)
    np.testing.assert_array_equal(st2.q[div], st.q[div])
