"""Pins of the oracle's HS and DSS online estimators (CPU only)."""
import dataclasses

import numpy as np
import pytest

from oracle import folds, scores, sampler
from paper_2310_07002_amd import workloads as W


@pytest.fixture(scope="module")
def gauss_runs():
    """Conjugate Gaussian, LOO (one test row) and blocked folds of 4 rows."""
    w1 = dataclasses.replace(W.make_c1(), scores=3, n_warmup=100, n_samples=1500)
    fi = (np.arange(w1.n) // 4).astype(np.int32)
    w4 = dataclasses.replace(w1, K=25, fold_index=fi, init_pos=w1.init_pos[:25 * w1.L])
    out = []
    for w in (w1, w4):
        run = sampler.run_all(w)
        roles = folds.roles_of(w)
        sizes = [len(t) for t in scores.test_rows_of_folds(roles)]
        est = scores.fold_scores(run.score_acc, w.K, w.L, run.acc.n_draws, sizes)
        tgt = scores.conjugate_targets(w.X, w.y, w.sigma, w.prior_scale, roles)
        out.append((w, est, tgt))
    return out


def test_hs_converges_to_conjugate_target(gauss_runs):
    for w, est, tgt in gauss_runs:
        err = est["hs_fold"] - tgt["hs_fold"]
        # fold-level Monte Carlo error of averages of ~1500 x 4 autocorrelated draws
        assert np.median(np.abs(err) / np.abs(tgt["hs_fold"])) < 0.02, w.K
        assert abs(est["hs"] - tgt["hs_fold"].sum()) < 0.02 * abs(tgt["hs_fold"].sum())


def test_dss_converges_to_conjugate_target(gauss_runs):
    for w, est, tgt in gauss_runs:
        err = est["dss_fold"] - tgt["dss_fold"]
        assert np.median(np.abs(err)) < 0.1, w.K
        assert abs(est["dss"] - tgt["dss_fold"].sum()) < 0.03 * abs(tgt["dss_fold"].sum()) + 0.05 * w.K


def test_predictive_draws_have_the_family_moments():
    """Many draws at fixed eta: Gaussian mean/variance, Bernoulli rate,
    Poisson mean and variance."""
    n = 200000
    eta = np.full((1, n), 0.7)
    words = scores.philox.predictive_words(123, np.array([5]), 9, n)
    g = scores.predictive_draw(0, eta, 0.5, words)
    assert abs(g.mean() - 0.7) < 4 * 0.5 / np.sqrt(n) and abs(g.var() - 0.25) < 0.01
    b = scores.predictive_draw(1, eta, 1.0, words)
    pr = 1 / (1 + np.exp(-0.7))
    assert abs(b.mean() - pr) < 4 * np.sqrt(pr * (1 - pr) / n)
    ps = scores.predictive_draw(2, eta, 1.0, words)
    lam = np.exp(0.7)
    assert abs(ps.mean() - lam) < 4 * np.sqrt(lam / n) and abs(ps.var() - lam) < 0.05 * lam
    assert np.all(ps == np.floor(ps))
