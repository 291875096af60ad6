"""Pins of the oracle's pairwise model comparison (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import closed_form, diagnostics, folds, sampler
from paper_2310_07002_amd import workloads as W


def _exact_elpd_fold(w):
    roles = folds.roles_of(w)
    out = np.empty(w.K)
    for k in range(w.K):
        ex = closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, roles[k] == folds.ROLE_TRAIN,
                                    roles[k] == folds.ROLE_TEST)
        out[k] = ex["elpd"]
    return out


@pytest.fixture(scope="module")
def pair():
    a = W.make_c1()
    drop = int(np.argmax(np.abs(a.truth)))       # model B misses the strongest covariate
    b = W.drop_covariates(a, [drop])
    return a, b


def test_normal_approximation_against_library_cdf(pair):
    """With the exact fold contributions, Pr(A > B) is the standard normal cdf
    of Delta / sqrt(K sigma2) (scipy's, an independent routine)."""
    a, b = pair
    ea, eb = _exact_elpd_fold(a), _exact_elpd_fold(b)
    c = diagnostics.compare(ea, np.zeros(a.K), eb, np.zeros(b.K))
    dk = ea - eb
    assert c["delta"] == pytest.approx(dk.sum(), rel=1e-14)
    assert c["sigma2"] == pytest.approx(np.var(dk, ddof=1), rel=1e-12)
    z = dk.sum() / math.sqrt(a.K * np.var(dk, ddof=1))
    assert c["prob_a_better"] == pytest.approx(stats.norm.cdf(z), rel=1e-12)
    assert c["delta"] > 0 and c["mcse"] == 0.0          # the true model predicts better


def test_swap_and_self_comparison():
    rng = np.random.default_rng(3)
    ea, eb = rng.normal(size=20), rng.normal(size=20)
    ma, mb = rng.uniform(0.01, 0.1, 20), rng.uniform(0.01, 0.1, 20)
    ab, ba = diagnostics.compare(ea, ma, eb, mb), diagnostics.compare(eb, mb, ea, ma)
    assert ab["delta"] == pytest.approx(-ba["delta"], rel=1e-14)
    assert ab["prob_a_better"] == pytest.approx(1.0 - ba["prob_a_better"], rel=1e-12)
    assert ab["mcse"] == pytest.approx(math.sqrt(np.sum(ma ** 2) + np.sum(mb ** 2)), rel=1e-14)
    same = diagnostics.compare(ea, ma, ea, ma)
    assert same["delta"] == 0.0 and same["prob_a_better"] == 0.5


def test_sampled_difference_within_mcse_of_exact(pair):
    """Both models sampled by the oracle (LOO, 100 folds x 4 chains): the
    estimated Delta lies within 4 MCSE of the closed-form Delta."""
    a, b = pair
    ra, rb = sampler.run_all(a), sampler.run_all(b)
    da = diagnostics.from_accumulators(ra.acc, a.K, a.L, a.batch_size)
    db = diagnostics.from_accumulators(rb.acc, b.K, b.L, b.batch_size)
    c = diagnostics.compare(da["elpd_fold"], da["mcse_fold"], db["elpd_fold"], db["mcse_fold"])
    exact = float(np.sum(_exact_elpd_fold(a) - _exact_elpd_fold(b)))
    assert abs(c["delta"] - exact) < 4.0 * c["mcse"], (c["delta"], exact, c["mcse"])
    assert c["prob_a_better"] > 0.99
