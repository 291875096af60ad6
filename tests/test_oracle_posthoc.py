"""Pins of the post-hoc diagnostics on stored draws (CPU only)."""
import numpy as np

from oracle import diagnostics, posthoc, sampler
from paper_2310_07002_amd import workloads as W


def test_rank_rhat_is_invariant_to_monotone_maps():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(4, 301)) + np.array([[0.0], [0.1], [0.0], [0.3]])
    r = posthoc.rank_rhat(x)
    assert r == posthoc.rank_rhat(2.0 * x + 3.0) == posthoc.rank_rhat(np.exp(x))
    # ties: a constant shift of all draws keeps every rank
    assert posthoc.rank_rhat(np.round(x, 1)) == posthoc.rank_rhat(np.round(x, 1) + 7.0)


def test_split_rhat_detects_a_drifting_chain():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4, 1000))
    assert abs(posthoc.split_rhat(x) - 1.0) < 0.01
    assert abs(posthoc.rhat_chains(x) - 1.0) < 0.01
    drift = x.copy()
    drift[2] += np.linspace(-1.5, 1.5, 1000)          # same chain mean, trending within
    assert posthoc.rhat_chains(drift) < 1.02 < posthoc.split_rhat(drift)
    assert posthoc.rank_rhat(drift) > 1.02


def test_stored_draws_reproduce_the_online_estimates():
    w = W.fold_subset(W.make_c1(), 0, 20)
    run = sampler.run_all(w, n_iter=w.n_warmup + 400, store_draws=True)
    on = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    ph = posthoc.fold_rhats(run.draws, w.K, w.L)
    np.testing.assert_allclose(ph["rhat_fold"], on["rhat_fold"], rtol=1e-10)
    assert ph["split_rhat_max"] < 1.1 and ph["rank_rhat_max"] < 1.1


# ---- value pins of the rank-normalised split R-hat --------------------------
# Two chains of four draws whose values are their own ranks 1..8, so every
# rank (and every tie of the folded draws) is known by inspection.  The
# expected R-hat is built here from those hand-assigned ranks: normal scores
# z(r) = Phi^-1((r - 3/8) / (8 + 1/4)) (Blom offsets, as Vehtari et al. 2021
# prescribe), then split R-hat of four half-chains of two draws, for which the
# within-chain variance of (a, b) is (a - b)^2 / 2 and
# R-hat^2 = (n - 1)/n + B/(n W) with n = 2 and B = n * var(half-chain means).
from scipy.special import ndtri  # noqa: E402


def _z(r):
    return ndtri((np.asarray(r, dtype=float) - 0.375) / 8.25)


def _split_rhat_of_pairs(pairs):
    """R-hat over half-chains of exactly two draws each (pairs of scores)."""
    pairs = np.asarray(pairs, dtype=float)
    means = pairs.mean(axis=1)
    W = np.mean((pairs[:, 0] - pairs[:, 1]) ** 2 / 2.0)
    gm = means.mean()
    B = 2.0 * np.sum((means - gm) ** 2) / (len(pairs) - 1)
    return float(np.sqrt(0.5 + B / (2.0 * W)))


def test_rank_rhat_value_shifted_chain():
    # chain 1 sits above chain 0: the bulk (location) R-hat dominates
    x = np.array([[1.0, 2.0, 3.0, 4.0], [5.0, 6.0, 7.0, 8.0]])
    bulk = _split_rhat_of_pairs([_z([1, 2]), _z([3, 4]), _z([5, 6]), _z([7, 8])])
    # |x - 4.5|: 3.5 2.5 1.5 0.5 | 0.5 1.5 2.5 3.5; each value occurs twice,
    # so the average ranks are 0.5 -> 1.5, 1.5 -> 3.5, 2.5 -> 5.5, 3.5 -> 7.5
    folded = _split_rhat_of_pairs([_z([7.5, 5.5]), _z([3.5, 1.5]), _z([1.5, 3.5]), _z([5.5, 7.5])])
    assert bulk > folded
    np.testing.assert_allclose(posthoc.rank_rhat(x), max(bulk, folded), rtol=1e-12)
    # the bulk value itself, worked by hand from normal-table quantiles
    # z(1..4) = -1.4342, -0.8525, -0.4728, -0.1525 (z(9 - r) = -z(r)):
    # half-chain means -1.1434, -0.3127, 0.3127, 1.1434; W = 0.11025;
    # B = 2 var(means) = 1.8733; R-hat^2 = 1/2 + B / (2 W) = 8.996
    np.testing.assert_allclose(bulk, 2.9993, atol=5e-4)


def test_rank_rhat_value_wide_chain():
    # same location, chain 1 holds the extreme ranks: the folded (scale)
    # R-hat dominates, so dropping the folded half changes the result
    x = np.array([[3.0, 5.0, 4.0, 6.0], [1.0, 8.0, 2.0, 7.0]])
    bulk = _split_rhat_of_pairs([_z([3, 5]), _z([4, 6]), _z([1, 8]), _z([2, 7])])
    # |x - 4.5|: 1.5 0.5 0.5 1.5 | 3.5 3.5 2.5 2.5
    folded = _split_rhat_of_pairs([_z([3.5, 1.5]), _z([1.5, 3.5]), _z([7.5, 7.5]), _z([5.5, 5.5])])
    assert folded > 1.5 > 1.0 > bulk - 0.2
    np.testing.assert_allclose(posthoc.rank_rhat(x), max(bulk, folded), rtol=1e-12)


def test_split_drops_the_middle_draw_of_odd_chains():
    # N = 5: halves are draws {0,1} and {3,4}; the middle draw (index 2) of
    # each chain must not influence the split R-hat
    a = np.array([[1.0, 2.0, 100.0, 3.0, 4.0], [5.0, 6.0, -100.0, 7.0, 8.0]])
    b = a.copy()
    b[:, 2] = [0.0, 0.0]
    assert posthoc.split_rhat(a) == posthoc.split_rhat(b)
    # and the halves are the first and last two draws
    np.testing.assert_allclose(posthoc.split_rhat(a),
                               _split_rhat_of_pairs([[1, 2], [3, 4], [5, 6], [7, 8]]), rtol=1e-12)
