"""Pins of the oracle's full-data window adaptation and chain starts (CPU only)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import adapt, closed_form, folds, hmc
from paper_2310_07002_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stan_windows.txt")


def test_windows_match_the_published_default_schedule():
    rows = [list(map(int, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for n, *ends in rows:
        assert adapt.slow_window_ends(n) == ends


@pytest.mark.parametrize("n", [20, 60, 100, 149, 150, 151, 200, 333, 500, 999, 2000, 5000])
def test_windows_tile_the_slow_phase_and_double(n):
    init, term, win = adapt.buffers(n)
    ends = adapt.slow_window_ends(n)
    assert ends[-1] == n - term
    sizes = np.diff([init] + ends)
    assert (sizes > 0).all()
    assert sizes[0] == win or len(sizes) == 1      # only a lone first window is stretched
    for a, b in zip(sizes[:-2], sizes[1:-1]):
        assert b == 2 * a
    if len(sizes) > 1:
        assert sizes[-1] >= 2 * sizes[-2]          # the stretched last window


def test_dual_averaging_reaches_the_analytic_step_size():
    """Acceptance curve a(eps) = exp(-eps^2 / 2): the target delta is met at
    eps* = sqrt(-2 log delta)."""
    for delta in (0.6, 0.8, 0.95):
        da = adapt.DualAveraging.start(1.0)
        for _ in range(20000):
            da.update(math.exp(-0.5 * math.exp(da.log_eps) ** 2), delta)
        target = math.sqrt(-2.0 * math.log(delta))
        assert abs(math.exp(da.log_epsbar) / target - 1.0) < 0.02


def test_regularised_variance_by_hand():
    s = np.array([[0.0, 1.0], [2.0, 1.0], [4.0, 4.0]])
    # column variances (n - 1 denominator): 4 and 3; n = 3
    expect = np.array([3 / 8 * 4 + 1e-3 * 5 / 8, 3 / 8 * 3 + 1e-3 * 5 / 8])
    np.testing.assert_allclose(adapt.regularised_variance(s), expect, rtol=1e-15)


@pytest.fixture(scope="module")
def adapted_c1():
    w = W.make("c1")
    f = W.full_data(w, L=8, n_warmup=2000)
    return w, f, adapt.adapt(f, 1000, 0.8)


def test_adapted_inverse_mass_is_the_posterior_variance(adapted_c1):
    """Conjugate Gaussian on the full data: the adapted diagonal inverse mass
    estimates the exact posterior variances (8 chains x 500 draws of the last
    slow window; 30% covers the Monte Carlo error of a correlated sample)."""
    w, f, (fa, st, eps, acc) = adapted_c1
    _, V, _ = closed_form.fold_posterior(w.X, w.y, w.sigma, w.prior_scale, np.ones(w.n, dtype=bool))
    ratio = fa.inv_mass / np.diag(V)
    assert (np.abs(ratio - 1.0) < 0.3).all(), ratio
    assert fa.step_size > 0 and np.isfinite(eps).all()


def test_adapted_step_size_hits_the_target_acceptance(adapted_c1):
    w, f, (fa, st, eps, acc) = adapted_c1
    roles = folds.roles_of(fa)
    foc = np.zeros(fa.C, dtype=np.int64)
    ids = np.arange(fa.C)
    a = []
    for t in range(1000, 1400):
        st, _, _ = hmc.transition(fa, st, t, roles, foc, ids)
        a.append(st.alpha.mean())
    assert abs(np.mean(a) - 0.8) < 0.1


def test_init_positions_pick_draws_uniformly():
    draws = np.arange(30, dtype=np.float64).reshape(10, 3)
    pos = adapt.init_positions(draws, 20000, seed=7)
    idx = (pos[:, 0] / 3).astype(int)
    np.testing.assert_array_equal(pos, draws[idx])
    np.testing.assert_array_equal(pos, adapt.init_positions(draws, 20000, seed=7))
    counts = np.bincount(idx, minlength=10)
    assert stats.chisquare(counts).pvalue > 1e-3
    # chain ids, not positions in the call, decide the draw
    np.testing.assert_array_equal(adapt.init_positions(draws, 10, seed=7, chain_offset=5), pos[5:15])
