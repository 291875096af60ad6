"""The allocation-free block-shuffle benchmark (static device scratch) gives
the same replicates as the allocating entry point, on two calls in a row,
the second with a smaller input, and refuses sizes beyond its scratch."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2310_07002_amd import binding, workloads as W


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    binding.load_library()
    return torch.device("cuda:0")


def _run(w, n_iter):
    s = binding.PCV.from_workload(w)
    s.step(n_iter)
    return s


@pytest.mark.gpu
def test_noalloc_shuffle_benchmark_matches_allocating_entry_point(dev):
    base = W.make_c1()
    # first call: 40 folds x 4 chains, 60 replicates
    w1 = dataclasses.replace(W.fold_subset(base, 0, 40), n_warmup=20)
    _say("no-alloc shuffle: c1 LOO, 40 folds x 4 chains, 120 transitions, R = 60")
    s1 = _run(w1, 120)
    mx_a, rep_a = s1.shuffle_benchmark(60, seed=11, per_fold=True)
    mx_b, rep_b = s1.shuffle_benchmark_noalloc(60, seed=11, per_fold=True)
    assert np.all(np.isfinite(mx_a)) and np.all(mx_a >= 1.0 - 1e-12)
    np.testing.assert_array_equal(mx_b, mx_a)
    np.testing.assert_array_equal(rep_b, rep_a)
    # second call in a row, smaller input: 12 folds, 7 replicates (the
    # scratch still holds the first call's larger contents)
    w2 = dataclasses.replace(W.fold_subset(base, 50, 62), n_warmup=10)
    _say("no-alloc shuffle: c1 LOO, 12 folds x 4 chains, 70 transitions, R = 7")
    s2 = _run(w2, 70)
    mx_c, rep_c = s2.shuffle_benchmark_noalloc(7, seed=3, per_fold=True)
    mx_d, rep_d = s2.shuffle_benchmark(7, seed=3, per_fold=True)
    np.testing.assert_array_equal(mx_c, mx_d)
    np.testing.assert_array_equal(rep_c, rep_d)
    # the first context again, without per-fold output
    np.testing.assert_array_equal(s1.shuffle_benchmark_noalloc(60, seed=11), mx_a)
    s2.close()
    s1.close()


@pytest.mark.gpu
def test_noalloc_shuffle_benchmark_refuses_oversized_requests(dev):
    w = dataclasses.replace(W.fold_subset(W.make_c1(), 0, 40), n_warmup=5)
    s = _run(w, 20)
    limit = 1 << 20
    R = limit // (w.K + 1) + 1          # (K + 1) R just above the scratch
    with pytest.raises(binding.PcvError) as e:
        s.shuffle_benchmark_noalloc(R, seed=1)
    assert e.value.status == 1 and "static scratch" in str(e.value)
    # the context stays usable and the largest fitting request still works
    R_ok = limit // (w.K + 1)
    np.testing.assert_array_equal(s.shuffle_benchmark_noalloc(R_ok, seed=2), s.shuffle_benchmark(R_ok, seed=2))
    s.close()
