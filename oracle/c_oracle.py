"""ctypes wrapper of the plain C oracle (oracle/c/pcv_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package header).

The C file restates the hot path of the method in plain fp64 loops: the
masked fold log density, its gradient and the fold log predictive
(Appendix B), fixed-trajectory HMC (Section 3.3), Algorithm A2's online
accumulators and the estimates and diagnostics computed from them
(Sections 2.4, 4).  It is a second oracle, written independently of the
numpy one in this package; tests/test_oracle_c.py holds the two to each
other and the C one to closed forms and published Philox vectors.  This
module only marshals arguments and compiles the file with the system C
compiler when its shared library is missing or older than the source.

Single-model runs only (no nested-model masks, no HS/DSS scores).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "pcv_oracle.c")
LIB = os.path.join(HERE, "c", "libpcv_oracle.so")
CC = os.environ.get("CC", "gcc")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (IEEE fp64: no fast-math) into LIB."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = f"{LIB}.{os.getpid()}.tmp"    # per process: parallel test workers may build at once
        cmd = [CC, "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("C oracle build failed: " + r.stderr)
        os.replace(tmp, LIB)
    return LIB


class _Model(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("n", ctypes.c_int64), ("p", ctypes.c_int64), ("d", ctypes.c_int64),
                ("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("fold_kind", ctypes.c_int32), ("fold_index", ctypes.c_void_p), ("intervals", ctypes.c_void_p),
                ("roles", ctypes.c_void_p), ("n_groups", ctypes.c_int32), ("group_of", ctypes.c_void_p),
                ("sigma", ctypes.c_double), ("prior_scale", ctypes.c_void_p), ("inv_mass", ctypes.c_void_p),
                ("step_size", ctypes.c_double), ("n_leapfrog", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("chain_offset", ctypes.c_int64), ("n_warmup", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("batches_per_block", ctypes.c_int32), ("rhat_mode", ctypes.c_int32)]


class _Acc(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_void_p), ("U", ctypes.c_void_p), ("U2", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("V2", ctypes.c_void_p), ("blk_n", ctypes.c_void_p), ("blk_mean", ctypes.c_void_p),
                ("blk_m2", ctypes.c_void_p), ("n_accept", ctypes.c_void_p), ("n_divergent", ctypes.c_void_p),
                ("wsum", ctypes.c_void_p), ("center", ctypes.c_void_p), ("n_wu", ctypes.c_int64),
                ("n_draws", ctypes.c_int64)]


def library():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build(force=False))
        P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.pco_philox.argtypes = [ctypes.c_uint64, U32, U32, U32, U32, P]
        lib.pco_philox.restype = None
        lib.pco_log_density.argtypes = [P, I64, P, P, P, P, ctypes.c_int]
        lib.pco_start.argtypes = [P, P, P, P, P, P, P, ctypes.c_int]
        lib.pco_advance.argtypes = [P, I64, I64, P, P, P, P, P, ctypes.c_int]
        lib.pco_diagnostics.argtypes = [P, P, P, P, P, P, P]
        for f in (lib.pco_log_density, lib.pco_start, lib.pco_advance, lib.pco_diagnostics):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Bound:
    """A pco_model struct and the arrays it points into (kept alive)."""

    def __init__(self, w):
        if getattr(w, "n_models", 1) != 1:
            raise ValueError("the C oracle runs single-model workloads only")
        self.X = np.ascontiguousarray(w.X, dtype=np.float64)
        self.y = np.ascontiguousarray(w.y, dtype=np.float64)
        self.fi = None if w.fold_index is None else np.ascontiguousarray(w.fold_index, dtype=np.int32)
        self.iv = None if w.intervals is None else np.ascontiguousarray(w.intervals, dtype=np.int64)
        self.roles = None if w.roles is None else np.ascontiguousarray(w.roles, dtype=np.int8)
        self.go = None if w.group_of is None else np.ascontiguousarray(w.group_of, dtype=np.int32)
        self.ps = None if w.prior_scale is None else np.ascontiguousarray(w.prior_scale, dtype=np.float64)
        self.im = np.ascontiguousarray(w.inv_mass, dtype=np.float64)
        n, p = self.X.shape
        self.C = w.K * w.L
        self.d = w.d
        self.D = w.n_blocks
        self.m = _Model(family=w.family, n=n, p=p, d=w.d, K=w.K, L=w.L, X=_ptr(self.X), y=_ptr(self.y),
                        fold_kind=w.fold_kind, fold_index=_ptr(self.fi), intervals=_ptr(self.iv),
                        roles=_ptr(self.roles), n_groups=int(w.n_groups or 0), group_of=_ptr(self.go),
                        sigma=float(w.sigma), prior_scale=_ptr(self.ps), inv_mass=_ptr(self.im),
                        step_size=float(w.step_size), n_leapfrog=int(w.n_leapfrog), seed=int(w.seed),
                        chain_offset=int(w.chain_offset), n_warmup=int(w.n_warmup), batch_size=int(w.batch_size),
                        n_blocks=int(w.n_blocks), batches_per_block=int(w.batches_per_block),
                        rhat_mode=int(getattr(w, "rhat_mode", 0)))

    @property
    def ref(self):
        return ctypes.byref(self.m)


def philox(seed: int, c0: int, c1: int, c2: int, c3: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    library().pco_philox(int(seed), c0, c1, c2, c3, _ptr(out))
    return out


def log_density_grad(w, theta: np.ndarray, threads: int = 1):
    """(log pi[C], grad[C, d], s[C]) of every chain at theta[C, d]."""
    b = _Bound(w)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    C = th.shape[0]
    assert th.shape == (C, b.d) and C <= b.C
    logp, grad, s = np.zeros(C), np.zeros((C, b.d)), np.zeros(C)
    if library().pco_log_density(b.ref, C, _ptr(th), _ptr(logp), _ptr(grad), _ptr(s), threads) != 0:
        raise RuntimeError("pco_log_density failed")
    return logp, grad, s


class Run:
    """State and accumulators of a C-oracle run; advance() continues it."""

    def __init__(self, w, threads: int = 1):
        self.b = _Bound(w)
        self.threads = threads
        C, d, D = self.b.C, self.b.d, self.b.D
        self.q, self.logp, self.grad, self.s = np.zeros((C, d)), np.zeros(C), np.zeros((C, d)), np.zeros(C)
        self.arr = {k: np.zeros(C) for k in ("Z", "U", "U2", "V", "V2", "wsum", "center")}
        self.arr["blk_n"] = np.zeros((C, D), dtype=np.int64)
        self.arr["blk_mean"] = np.zeros((C, D))
        self.arr["blk_m2"] = np.zeros((C, D))
        self.arr["n_accept"] = np.zeros(C, dtype=np.int64)
        self.arr["n_divergent"] = np.zeros(C, dtype=np.int64)
        self.acc = _Acc(**{k: _ptr(v) for k, v in self.arr.items()}, n_wu=0, n_draws=0)
        init = np.ascontiguousarray(w.init_pos, dtype=np.float64)
        assert init.shape == (C, d)
        self.t = 0
        if library().pco_start(self.b.ref, _ptr(init), _ptr(self.q), _ptr(self.logp), _ptr(self.grad),
                               _ptr(self.s), ctypes.byref(self.acc), threads) != 0:
            raise RuntimeError("pco_start failed")

    def advance(self, n_iter: int) -> "Run":
        if library().pco_advance(self.b.ref, self.t, int(n_iter), _ptr(self.q), _ptr(self.logp), _ptr(self.grad),
                                 _ptr(self.s), ctypes.byref(self.acc), self.threads) != 0:
            raise RuntimeError("pco_advance failed")
        self.t += int(n_iter)
        return self

    @property
    def n_draws(self) -> int:
        return int(self.acc.n_draws)

    def diagnostics(self) -> dict:
        K = self.b.m.K
        ef, mf, rf, sf, out = np.zeros(K), np.zeros(K), np.zeros(K), np.zeros(K), np.zeros(6)
        if library().pco_diagnostics(self.b.ref, ctypes.byref(self.acc), _ptr(ef), _ptr(mf), _ptr(rf), _ptr(sf),
                                     _ptr(out)) != 0:
            raise RuntimeError("pco_diagnostics failed")
        return {"elpd_fold": ef, "mcse_fold": mf, "rhat_fold": rf, "ess_fold": sf, "elpd": out[0], "mcse": out[1],
                "rhat_max": out[2], "ess": out[3], "accept_rate": out[4], "n_divergent": int(out[5]),
                "n_draws": self.n_draws}


def run_all(w, n_iter=None, threads: int = 1) -> Run:
    r = Run(w, threads)
    return r.advance(w.n_iter if n_iter is None else n_iter)
