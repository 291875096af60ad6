"""Pins of the oracle's counter-based random numbers (CPU only)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            words = [int(t, 16) for t in line.split()]
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = philox.philox4x32_10(tuple(np.uint64(c) for c in ctr), key)
    assert [int(o) for o in out] == expect


def test_uniform_mapping_edges_and_exactness():
    u_min = philox.uniform_from_words(np.uint64(0), np.uint64(0))
    u_max = philox.uniform_from_words(np.uint64(0xFFFFFFFF), np.uint64(0xFFFFFFFF))
    assert u_min == 2.0 ** -53
    assert u_max == 1.0 - 2.0 ** -53
    # the mapping is exact: (2k+1) * 2^-53 for the top 52 bits k
    w0, w1 = np.uint64(0x12345678), np.uint64(0x9ABCDEF0)
    k = ((int(w0) << 32) | int(w1)) >> 12
    assert philox.uniform_from_words(w0, w1) == (2 * k + 1) * 2.0 ** -53


def test_accept_uniforms_distribution():
    u = philox.accept_uniforms(1234, np.arange(200000), 7)
    assert np.all((u > 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_momentum_normals_distribution_and_independence():
    z = philox.momentum_normals(99, np.arange(20000), 3, 7)
    assert z.shape == (20000, 7)
    flat = z.ravel()
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    corr = np.corrcoef(z.T)
    assert np.max(np.abs(corr - np.eye(7))) < 0.03
    # different iterations, tags and chains give different streams
    z2 = philox.momentum_normals(99, np.arange(20000), 4, 7)
    assert abs(np.corrcoef(z[:, 0], z2[:, 0])[0, 1]) < 0.03


def test_streams_depend_only_on_global_chain_id():
    full = philox.momentum_normals(5, np.arange(100), 11, 3)
    part = philox.momentum_normals(5, np.arange(40, 60), 11, 3)
    np.testing.assert_array_equal(full[40:60], part)


def test_shuffle_indices_uniform():
    idx = np.concatenate([philox.shuffle_indices(3, 0, r, 4, 5).ravel() for r in range(4000)])
    counts = np.bincount(idx, minlength=4)
    assert stats.chisquare(counts).pvalue > 1e-3
