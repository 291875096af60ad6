"""The C ABI library loads, exports every declared entry point, and rejects
invalid input before touching the device (CPU only)."""
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_2310_07002_amd import binding, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcv.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pcv_status|void|const char\*)\s+(pcv_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("pcv_init", "pcv_step", "pcv_diagnostics", "pcv_elpd", "pcv_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(binding.EXPORTED) == _declared()


def test_status_strings():
    lib = binding.load_library()
    assert lib.pcv_status_str(0) == b"ok"
    assert lib.pcv_status_str(1) == b"invalid argument"


def _expect_invalid(w, **over):
    w = dataclasses.replace(w, **over)
    with pytest.raises(binding.PcvError) as e:
        binding.PCV.from_workload(w)
    return e.value.status


@pytest.fixture(scope="module")
def small():
    return W.fold_subset(W.make("c1"), 0, 5)


def test_invalid_inputs_are_rejected(small):
    w = small
    assert _expect_invalid(w, L=1) == 1
    bad_y = w.y.copy()
    bad_y[3] = np.nan
    assert _expect_invalid(w, y=bad_y) == 1
    assert _expect_invalid(w, step_size=-0.1) == 1
    bad_m = w.inv_mass.copy()
    bad_m[0] = 0.0
    assert _expect_invalid(w, inv_mass=bad_m) == 1
    bad_f = w.fold_index.copy()
    bad_f[0] = w.K + 3
    assert _expect_invalid(w, fold_index=bad_f) == 1
    # a fold with no test row
    empty = w.fold_index.copy()
    empty[empty == 2] = -1
    assert _expect_invalid(w, fold_index=empty) == 1
    assert _expect_invalid(w, n_leapfrog=0) == 1


def test_family_support_is_checked():
    w = W.fold_subset(W.make("c4"), 0, 3)
    y = w.y.copy()
    y[0] = 0.5
    assert _expect_invalid(w, y=y) == 1
    w5 = W.fold_subset(W.make("c5"), 0, 3)
    y5 = w5.y.copy()
    y5[1] = 2.0
    assert _expect_invalid(w5, y=y5) == 1


def test_unsupported_shapes_are_reported():
    """The matrix-core kernels go up to 128 covariates, the VALU kernels to
    64: wider designs are refused before any device work."""
    w = W.fold_subset(W.make("c1"), 0, 3)
    rng = np.random.default_rng(0)
    wide = dataclasses.replace(w, X=rng.standard_normal((w.n, 130)), prior_scale=np.ones(130),
                               inv_mass=np.ones(130), init_pos=np.zeros((w.C, 130)), x_hi=None, x_lo=None)
    assert _expect_invalid(wide, precision=W.PREC_BF16X3) == 5
    assert _expect_invalid(wide, precision=W.PREC_FP32) == 5


def test_model_masks_are_validated():
    """Several models in one launch: masks must be 0/1 and present; scores
    are refused, and hierarchical families off the fp64 / fp32 paths (host
    checks, no device)."""
    w = W.fold_subset(W.make("c1"), 0, 3)
    m = np.ones((2, w.p), dtype=np.uint8)
    w2 = W.with_models(w, m)
    assert _expect_invalid(w2, model_mask=np.full_like(m, 3)) == 1
    assert _expect_invalid(w2, model_mask=None) == 1
    assert _expect_invalid(w2, scores=2) == 5                  # PCV_ERR_UNSUPPORTED
    h = W.fold_subset(W.make("c2"), 0, 2)
    h2 = dataclasses.replace(h, n_models=2, model_mask=np.ones((2, h.p), dtype=np.uint8),
                             init_pos=np.concatenate([h.init_pos] * 2))
    assert _expect_invalid(h2, precision=W.PREC_BF16X3) == 5
    e = W.make_ex1_ab()
    assert _expect_invalid(e, precision=W.PREC_BF16X3) == 5
    assert _expect_invalid(e, scores=2) == 5
    assert _expect_invalid(W.make_ex1(), scores=1) == 5


def test_init_positions_rejects_bad_arguments():
    lib = binding.load_library()
    d = np.zeros((3, 2))
    out = np.zeros((4, 2))
    ptr = lambda a: a.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_double))
    assert lib.pcv_init_positions(ptr(d), 0, 2, 4, 1, 0, ptr(out)) == 1
    assert lib.pcv_init_positions(None, 3, 2, 4, 1, 0, ptr(out)) == 1
    assert lib.pcv_init_positions(ptr(d), 3, 2, 4, 1, 2 ** 32 - 2, ptr(out)) == 1
    assert lib.pcv_init_positions(ptr(d), 3, 2, 4, 1, 0, ptr(out)) == 0


def test_interval_folds_need_one_non_train_range():
    """Interval folds: a test block and an exclusion range that neither
    overlap nor touch would give a fold two non-train ranges; refused on the
    host (the touching and empty-exclusion forms are accepted and checked
    against the oracle on the device)."""
    w = W.fold_subset(W.make("c3"), 0, 4)
    iv = w.intervals.copy()
    k = 2
    lo, hi = int(iv[k, 0]), int(iv[k, 1])
    iv[k] = (lo, hi, hi + 3, hi + 6)
    assert _expect_invalid(w, intervals=iv) == 1
    iv[k] = (lo, hi, max(0, lo - 9), lo - 4)
    assert _expect_invalid(w, intervals=iv) == 1


def test_mfma_calibration_rejects_bad_arguments():
    """Argument checks come before any device call."""
    lib = binding.load_library()
    import ctypes
    out = ctypes.c_double(0.0)
    assert lib.pcv_calib_mfma(2, 10, ctypes.byref(out)) == 1
    assert lib.pcv_calib_mfma(1, 0, ctypes.byref(out)) == 1
    assert lib.pcv_calib_mfma(0, 10, None) == 1
