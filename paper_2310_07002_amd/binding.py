"""ctypes binding of libpcv.so (include/pcv.h), same names as the C ABI.

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  Device arrays for the lower-level calls are torch tensors on the
current HIP device; host arrays are numpy arrays.  The library is loaded from
this package directory; importing works without a GPU, but calls that touch
the device fail loudly if there is none.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcv.so")

PCV_OK = 0
STATUS_NAMES = {0: "PCV_OK", 1: "PCV_ERR_INVALID_ARG", 2: "PCV_ERR_NOMEM", 3: "PCV_ERR_DEVICE",
                4: "PCV_ERR_STATE", 5: "PCV_ERR_UNSUPPORTED"}

EXPORTED = ["pcv_init", "pcv_set_stream", "pcv_step", "pcv_diagnostics", "pcv_elpd",
            "pcv_shuffle_benchmark", "pcv_shuffle_benchmark_noalloc", "pcv_scores", "pcv_get_draws",
            "pcv_posthoc", "pcv_compare",
            "pcv_destroy", "pcv_last_error", "pcv_status_str",
            "pcv_logdensity_grad", "pcv_leapfrog", "pcv_get_state", "pcv_set_state",
            "pcv_get_accumulators", "pcv_autotune", "pcv_save", "pcv_load", "pcv_philox",
            "pcv_adapt", "pcv_init_positions", "pcv_elpd_model", "pcv_compare_models",
            "pcv_timing_enable", "pcv_timing_read", "pcv_set_launch_config", "pcv_get_launch_config",
            "pcv_calib_mfma"]


class PcvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pcv_folds(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32),
                ("fold_index", ctypes.POINTER(ctypes.c_int32)),
                ("intervals", ctypes.POINTER(ctypes.c_int64)),
                ("roles", ctypes.POINTER(ctypes.c_int8))]


class pcv_model(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("group_of", ctypes.POINTER(ctypes.c_int32)),
                ("sigma", ctypes.c_double), ("prior_scale", ctypes.POINTER(ctypes.c_double)),
                ("step_size", ctypes.c_double), ("n_leapfrog", ctypes.c_int32),
                ("inv_mass", ctypes.POINTER(ctypes.c_double)),
                ("init_pos", ctypes.POINTER(ctypes.c_double)),
                ("n_warmup", ctypes.c_int64), ("batch_size", ctypes.c_int32),
                ("batches_per_block", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("chain_offset", ctypes.c_int64),
                ("x_format", ctypes.c_int32), ("rhat_mode", ctypes.c_int32),
                ("scores", ctypes.c_int32), ("store_draws", ctypes.c_int64),
                ("n_models", ctypes.c_int32), ("model_mask", ctypes.POINTER(ctypes.c_uint8))]

X_FP64, X_BF16_HILO = 0, 1
RHAT_WELFORD, RHAT_SHIFTED_SUMS = 0, 1
SCORE_HS, SCORE_DSS = 1, 2


class pcv_comparison(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("prob_a_better", ctypes.c_double), ("mcse", ctypes.c_double),
                ("delta_fold", ctypes.POINTER(ctypes.c_double))]


class pcv_posthoc_diag(ctypes.Structure):
    _fields_ = [("elpd", ctypes.c_double), ("mcse", ctypes.c_double), ("ess", ctypes.c_double),
                ("rhat_max", ctypes.c_double), ("split_rhat_max", ctypes.c_double),
                ("rank_rhat_max", ctypes.c_double), ("n_draws", ctypes.c_int64),
                ("rhat_fold", ctypes.POINTER(ctypes.c_double)),
                ("split_rhat_fold", ctypes.POINTER(ctypes.c_double)),
                ("rank_rhat_fold", ctypes.POINTER(ctypes.c_double))]


class pcv_diag(ctypes.Structure):
    _fields_ = [("rhat_max", ctypes.c_double), ("ess", ctypes.c_double),
                ("elpd", ctypes.c_double), ("mcse", ctypes.c_double),
                ("accept_rate", ctypes.c_double), ("n_divergent", ctypes.c_int64),
                ("n_draws", ctypes.c_int64), ("n_iter", ctypes.c_int64),
                ("rhat_fold", ctypes.POINTER(ctypes.c_double)),
                ("ess_fold", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libpcv.so from this package (raises if it has not been built).
    PCV_LIBRARY may name another build of the same library (experiments)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("PCV_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2310_07002_amd.build")
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "pcv_init": ([ctypes.POINTER(P), ctypes.POINTER(pcv_model), P, dp, ctypes.POINTER(pcv_folds)], I32),
        "pcv_set_stream": ([P, P], I32),
        "pcv_step": ([P, I64], I32),
        "pcv_diagnostics": ([P, ctypes.POINTER(pcv_diag)], I32),
        "pcv_elpd": ([P, dp, dp, dp, dp], I32),
        "pcv_shuffle_benchmark": ([P, I32, U64, dp, dp], I32),
        "pcv_shuffle_benchmark_noalloc": ([P, I32, U64, dp, dp], I32),
        "pcv_compare": ([P, P, ctypes.POINTER(pcv_comparison)], I32),
        "pcv_scores": ([P, dp, dp, dp, dp], I32),
        "pcv_get_draws": ([P, dp, I64, ctypes.POINTER(I64)], I32),
        "pcv_posthoc": ([P, ctypes.POINTER(pcv_posthoc_diag)], I32),
        "pcv_destroy": ([P], None),
        "pcv_last_error": ([P], ctypes.c_char_p),
        "pcv_status_str": ([I32], ctypes.c_char_p),
        "pcv_logdensity_grad": ([P, P, P, P, I32], I32),
        "pcv_leapfrog": ([P, P, P, I32, P, P, P, P], I32),
        "pcv_get_state": ([P, dp, dp, dp], I32),
        "pcv_set_state": ([P, dp], I32),
        "pcv_get_accumulators": ([P, dp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "pcv_autotune": ([P, ctypes.c_char_p, ctypes.POINTER(I32), dp], I32),
        "pcv_set_launch_config": ([P, I32], I32),
        "pcv_get_launch_config": ([P, ctypes.POINTER(I32)], I32),
        "pcv_save": ([P, ctypes.c_char_p], I32),
        "pcv_load": ([P, ctypes.c_char_p], I32),
        "pcv_philox": ([U64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, I64,
                        ctypes.POINTER(ctypes.c_uint32)], I32),
        "pcv_adapt": ([P, I64, D, dp, dp], I32),
        "pcv_elpd_model": ([P, I32, dp, dp, dp, dp], I32),
        "pcv_compare_models": ([P, I32, I32, ctypes.POINTER(pcv_comparison)], I32),
        "pcv_init_positions": ([dp, I64, I64, I64, U64, I64, dp], I32),
        "pcv_timing_enable": ([P, I32], I32),
        "pcv_timing_read": ([P, dp, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_char_p), I32], I32),
        "pcv_calib_mfma": ([I32, I32, dp], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dev(t) -> ctypes.c_void_p:
    if t is None:
        return None
    if not t.is_cuda or t.dtype != __import__("torch").float64 or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def init_positions(draws: np.ndarray, C: int, seed: int, chain_offset: int = 0) -> np.ndarray:
    """Starting positions [C, d] drawn from full-data draws [n_draws, d]
    (pcv_init_positions)."""
    lib = load_library()
    draws = np.ascontiguousarray(draws, dtype=np.float64)
    n_draws, d = draws.shape
    out = np.zeros((C, d))
    st = lib.pcv_init_positions(_dptr(draws), n_draws, d, C, seed, chain_offset, _dptr(out))
    if st != PCV_OK:
        raise PcvError(st, "pcv_init_positions failed")
    return out


def pcv_philox(seed: int, c0: int, c1: int, c2: int, c3: int, n: int) -> np.ndarray:
    lib = load_library()
    out = np.zeros(4 * n, dtype=np.uint32)
    st = lib.pcv_philox(seed, c0, c1, c2, c3, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if st != PCV_OK:
        raise PcvError(st, "pcv_philox failed")
    return out.reshape(n, 4)


def pcv_calib_mfma(data_kind: int, launches: int = 50) -> float:
    """Sustained bf16 32x32x16 MFMA rate in TFLOP/s on constant (0) or random (1) operands."""
    lib = load_library()
    out = ctypes.c_double(0.0)
    st = lib.pcv_calib_mfma(int(data_kind), int(launches), ctypes.byref(out))
    if st != PCV_OK:
        raise PcvError(st, "pcv_calib_mfma failed")
    return out.value


class PCV:
    """One sampler context (pcv_ctx).  Thin wrapper; see include/pcv.h."""

    def __init__(self, *, family: int, precision: int, X: np.ndarray, y: np.ndarray, K: int, L: int,
                 fold_kind: int, fold_index=None, intervals=None, roles=None, group_of=None,
                 n_groups: int = 0, sigma: float = 1.0, prior_scale=None, step_size: float,
                 n_leapfrog: int, inv_mass, init_pos, n_warmup: int, batch_size: int,
                 batches_per_block: int, n_blocks: int, seed: int, chain_offset: int = 0,
                 x_format: int = X_FP64, rhat_mode: int = RHAT_WELFORD, scores: int = 0,
                 store_draws: int = 0, n_models: int = 1, model_mask=None, stream=None):
        """X: [n, p] float64, or with x_format=X_BF16_HILO a [2, n, p] uint16
        array of bf16 bit patterns (hi plane, lo plane).  n_models > 1 with
        model_mask [n_models, p] (0/1): several nested models in one launch,
        n_models * K * L chains, model-major."""
        self._lib = load_library()
        if x_format == X_BF16_HILO:
            X = np.ascontiguousarray(X, dtype=np.uint16)
            assert X.ndim == 3 and X.shape[0] == 2, "bf16 planes must be [2, n, p]"
            n, p = X.shape[1:]
        else:
            X = np.ascontiguousarray(X, dtype=np.float64)
            n, p = X.shape
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.n, self.p, self.K, self.L = n, p, int(K), int(L)
        self.M = max(1, int(n_models))
        self.C = self.M * self.K * self.L
        self._scores = int(scores)
        # parameters per chain: GLMs p; hierarchical logistic p + 2 + groups;
        # hierarchical Gaussian p + 3 + groups (its extra log sigma_y)
        self.d = p + (3 if family == 4 else 2) + n_groups if group_of is not None else p
        keep = []

        def arr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        inv_mass = arr(inv_mass, np.float64)
        init_pos = arr(init_pos, np.float64)
        prior_scale = arr(prior_scale, np.float64)
        go = arr(group_of, np.int32)
        fi = arr(fold_index, np.int32)
        iv = arr(intervals, np.int64)
        rl = arr(roles, np.int8)
        mm = arr(model_mask, np.uint8) if self.M > 1 else None
        m = pcv_model()
        m.family, m.precision = family, precision
        m.n, m.p, m.K, m.L = n, p, K, L
        m.n_groups = n_groups
        m.group_of = go.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if go is not None else None
        m.sigma = sigma
        m.prior_scale = _dptr(prior_scale)
        m.step_size, m.n_leapfrog = step_size, n_leapfrog
        m.inv_mass = _dptr(inv_mass)
        m.init_pos = _dptr(init_pos)
        m.n_warmup, m.batch_size = n_warmup, batch_size
        m.batches_per_block, m.n_blocks = batches_per_block, n_blocks
        m.seed, m.chain_offset = seed, chain_offset
        m.x_format, m.rhat_mode, m.scores = x_format, rhat_mode, scores
        m.store_draws = store_draws
        m.n_models = self.M
        m.model_mask = mm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if mm is not None else None
        f = pcv_folds()
        f.kind = fold_kind
        f.fold_index = fi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if fi is not None else None
        f.intervals = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if iv is not None else None
        f.roles = rl.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)) if rl is not None else None
        self._ctx = ctypes.c_void_p()
        st = self._lib.pcv_init(ctypes.byref(self._ctx), ctypes.byref(m), X.ctypes.data_as(ctypes.c_void_p),
                                _dptr(y), ctypes.byref(f))
        if st != PCV_OK:
            self._ctx = None
            raise PcvError(st, "pcv_init failed (details on stderr)")
        if stream is not None:
            self.set_stream(stream)

    @classmethod
    def from_workload(cls, w, precision: Optional[int] = None, stream=None, x_planes: bool = False,
                      rhat_mode: Optional[int] = None) -> "PCV":
        """x_planes: pass the design as its stored bf16 hi/lo planes (w.x_hi, w.x_lo).
        rhat_mode: default the workload's."""
        X, xf = (np.stack([w.x_hi, w.x_lo]), X_BF16_HILO) if x_planes else (w.X, X_FP64)
        if rhat_mode is None:
            rhat_mode = getattr(w, "rhat_mode", RHAT_WELFORD)
        return cls(family=w.family, precision=w.precision if precision is None else precision,
                   X=X, x_format=xf, rhat_mode=rhat_mode, scores=getattr(w, "scores", 0),
                   store_draws=getattr(w, "store_draws", 0), y=w.y,
                   K=w.K, L=w.L, fold_kind=w.fold_kind,
                   fold_index=w.fold_index,
                   intervals=w.intervals, roles=w.roles, group_of=w.group_of, n_groups=w.n_groups,
                   sigma=w.sigma, prior_scale=w.prior_scale, step_size=w.step_size,
                   n_leapfrog=w.n_leapfrog, inv_mass=w.inv_mass, init_pos=w.init_pos,
                   n_warmup=w.n_warmup, batch_size=w.batch_size,
                   batches_per_block=w.batches_per_block, n_blocks=w.n_blocks, seed=w.seed,
                   chain_offset=w.chain_offset, n_models=getattr(w, "n_models", 1),
                   model_mask=getattr(w, "model_mask", None), stream=stream)

    # -- helpers ---------------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != PCV_OK:
            msg = self._lib.pcv_last_error(self._ctx)
            raise PcvError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pcv_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI -----------------------------------------------------------------
    def set_stream(self, stream):
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._check(self._lib.pcv_set_stream(self._ctx, ctypes.c_void_p(handle)), "pcv_set_stream")

    def step(self, n_iter: int):
        self._check(self._lib.pcv_step(self._ctx, int(n_iter)), "pcv_step")

    def diagnostics(self) -> dict:
        rf = np.zeros(self.M * self.K)
        ef = np.zeros(self.M * self.K)
        d = pcv_diag()
        d.rhat_fold = _dptr(rf)
        d.ess_fold = _dptr(ef)
        self._check(self._lib.pcv_diagnostics(self._ctx, ctypes.byref(d)), "pcv_diagnostics")
        return {"rhat_max": d.rhat_max, "ess": d.ess, "elpd": d.elpd, "mcse": d.mcse,
                "accept_rate": d.accept_rate, "n_divergent": d.n_divergent, "n_draws": d.n_draws,
                "n_iter": d.n_iter, "rhat_fold": rf, "ess_fold": ef}

    def elpd(self) -> dict:
        e = ctypes.c_double()
        s = ctypes.c_double()
        ef = np.zeros(self.M * self.K)
        sf = np.zeros(self.M * self.K)
        self._check(self._lib.pcv_elpd(self._ctx, ctypes.byref(e), ctypes.byref(s), _dptr(ef), _dptr(sf)),
                    "pcv_elpd")
        return {"elpd": e.value, "mcse": s.value, "elpd_fold": ef, "mcse_fold": sf}

    def elpd_model(self, model: int) -> dict:
        """elpd and MCSE of one model of a multi-model run, in total and per fold."""
        e = ctypes.c_double()
        s = ctypes.c_double()
        ef = np.zeros(self.K)
        sf = np.zeros(self.K)
        self._check(self._lib.pcv_elpd_model(self._ctx, model, ctypes.byref(e), ctypes.byref(s), _dptr(ef),
                                             _dptr(sf)), "pcv_elpd_model")
        return {"elpd": e.value, "mcse": s.value, "elpd_fold": ef, "mcse_fold": sf}

    def compare_models(self, a: int, b: int) -> dict:
        """Model a against model b of this run (pcv_compare_models)."""
        out = pcv_comparison()
        df = np.zeros(self.K)
        out.delta_fold = _dptr(df)
        self._check(self._lib.pcv_compare_models(self._ctx, a, b, ctypes.byref(out)), "pcv_compare_models")
        return {"delta": out.delta, "sigma2": out.sigma2, "prob_a_better": out.prob_a_better,
                "mcse": out.mcse, "delta_fold": df}

    def shuffle_benchmark(self, R: int, seed: int, per_fold: bool = False):
        mx = np.zeros(R)
        rep = np.zeros(self.M * self.K * R) if per_fold else None
        self._check(self._lib.pcv_shuffle_benchmark(self._ctx, R, seed, _dptr(mx), _dptr(rep)),
                    "pcv_shuffle_benchmark")
        return (mx, rep.reshape(self.M * self.K, R)) if per_fold else mx

    def shuffle_benchmark_noalloc(self, R: int, seed: int, per_fold: bool = False):
        """The same benchmark on the library's static device scratch (no
        device allocation; at most PCV_SHUFFLE_NOALLOC_MAX_DOUBLES doubles)."""
        mx = np.zeros(R)
        rep = np.zeros(self.M * self.K * R) if per_fold else None
        self._check(self._lib.pcv_shuffle_benchmark_noalloc(self._ctx, R, seed, _dptr(mx), _dptr(rep)),
                    "pcv_shuffle_benchmark_noalloc")
        return (mx, rep.reshape(self.M * self.K, R)) if per_fold else mx

    def logdensity_grad(self, theta, want_grad: bool = True):
        """theta: [C, d] float64 cuda tensor -> (logp [C], grad [C, d] or None)."""
        import torch
        logp = torch.empty(self.C, dtype=torch.float64, device=theta.device)
        grad = torch.empty_like(theta) if want_grad else None
        self._check(self._lib.pcv_logdensity_grad(self._ctx, _dev(theta), _dev(logp), _dev(grad),
                                                  1 if want_grad else 0), "pcv_logdensity_grad")
        return logp, grad

    def leapfrog(self, q, p, n_steps: int):
        import torch
        q_out = torch.empty_like(q)
        p_out = torch.empty_like(p)
        logp = torch.empty(self.C, dtype=torch.float64, device=q.device)
        grad = torch.empty_like(q)
        self._check(self._lib.pcv_leapfrog(self._ctx, _dev(q), _dev(p), int(n_steps), _dev(q_out),
                                           _dev(p_out), _dev(logp), _dev(grad)), "pcv_leapfrog")
        return q_out, p_out, logp, grad

    def get_state(self):
        th = np.zeros((self.C, self.d))
        lp = np.zeros(self.C)
        s = np.zeros(self.C)
        self._check(self._lib.pcv_get_state(self._ctx, _dptr(th), _dptr(lp), _dptr(s)), "pcv_get_state")
        return th, lp, s

    def set_state(self, theta: np.ndarray):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self._check(self._lib.pcv_set_state(self._ctx, _dptr(th)), "pcv_set_state")

    def get_accumulators(self, n_blocks: int) -> dict:
        C = self.C
        out = {k: np.zeros(C) for k in ("Z", "U", "U2", "V", "V2")}
        out["blk_mean"] = np.zeros(n_blocks * C)
        out["blk_m2"] = np.zeros(n_blocks * C)
        out["n_accept"] = np.zeros(C, dtype=np.int64)
        out["n_divergent"] = np.zeros(C, dtype=np.int64)
        i64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self._check(self._lib.pcv_get_accumulators(
            self._ctx, _dptr(out["Z"]), _dptr(out["U"]), _dptr(out["U2"]), _dptr(out["V"]),
            _dptr(out["V2"]), _dptr(out["blk_mean"]), _dptr(out["blk_m2"]), i64(out["n_accept"]),
            i64(out["n_divergent"])), "pcv_get_accumulators")
        out["blk_mean"] = out["blk_mean"].reshape(n_blocks, C).T.copy()
        out["blk_m2"] = out["blk_m2"].reshape(n_blocks, C).T.copy()
        return out

    def scores(self) -> dict:
        """HS and/or DSS (those enabled in the model), total and per fold."""
        out = {}
        hs, dss = ctypes.c_double(), ctypes.c_double()
        hf, df = np.zeros(self.K), np.zeros(self.K)
        want_h, want_d = bool(self._scores & SCORE_HS), bool(self._scores & SCORE_DSS)
        self._check(self._lib.pcv_scores(self._ctx, ctypes.byref(hs) if want_h else None,
                                         _dptr(hf) if want_h else None,
                                         ctypes.byref(dss) if want_d else None,
                                         _dptr(df) if want_d else None), "pcv_scores")
        if want_h:
            out.update(hs=hs.value, hs_fold=hf)
        if want_d:
            out.update(dss=dss.value, dss_fold=df)
        return out

    def get_draws(self, n_max: int) -> np.ndarray:
        """Stored post-warm-up draws of s, [C, n] (n <= n_max)."""
        buf = np.zeros(self.C * int(n_max))
        n = ctypes.c_int64()
        self._check(self._lib.pcv_get_draws(self._ctx, _dptr(buf), int(n_max), ctypes.byref(n)), "pcv_get_draws")
        return buf[: self.C * n.value].reshape(self.C, n.value)

    def posthoc(self) -> dict:
        """Two-pass estimates and R-hats (paper's, split, rank-normalised) from the stored draws."""
        out = pcv_posthoc_diag()
        f = {k: np.zeros(self.M * self.K) for k in ("rhat_fold", "split_rhat_fold", "rank_rhat_fold")}
        for k, a in f.items():
            setattr(out, k, _dptr(a))
        self._check(self._lib.pcv_posthoc(self._ctx, ctypes.byref(out)), "pcv_posthoc")
        res = {k: getattr(out, k) for k in ("elpd", "mcse", "ess", "rhat_max", "split_rhat_max",
                                            "rank_rhat_max", "n_draws")}
        res.update(f)
        return res

    def compare(self, other: "PCV") -> dict:
        """This run as model A against `other` as model B on the same folds."""
        df = np.zeros(self.K)
        out = pcv_comparison()
        out.delta_fold = _dptr(df)
        self._check(self._lib.pcv_compare(self._ctx, other._ctx, ctypes.byref(out)), "pcv_compare")
        return {"delta": out.delta, "sigma2": out.sigma2, "prob_a_better": out.prob_a_better,
                "mcse": out.mcse, "delta_fold": df}

    def autotune(self, cache_path: Optional[str] = None) -> dict:
        """Time candidate launch shapes of the hot kernel and keep the fastest
        (row splits on the matrix-core and row-split VALU paths, waves per
        workgroup on the fused VALU path); cache_path: JSON cache of tuned
        shapes."""
        cfg = ctypes.c_int32()
        ms = ctypes.c_double()
        self._check(self._lib.pcv_autotune(self._ctx, os.fsencode(cache_path) if cache_path else None,
                                           ctypes.byref(cfg), ctypes.byref(ms)), "pcv_autotune")
        return {"config": cfg.value, "ms": ms.value}

    def set_launch_config(self, config: int):
        """Apply a launch shape in pcv_autotune's encoding."""
        self._check(self._lib.pcv_set_launch_config(self._ctx, int(config)), "pcv_set_launch_config")

    def launch_config(self) -> int:
        cfg = ctypes.c_int32()
        self._check(self._lib.pcv_get_launch_config(self._ctx, ctypes.byref(cfg)), "pcv_get_launch_config")
        return cfg.value

    def adapt(self, n_adapt: int, target_accept: float = 0.8) -> dict:
        """Window adaptation of the step size and diagonal inverse mass over
        n_adapt transitions of this (full-data) context (pcv_adapt); the
        context keeps the adapted values."""
        eps = ctypes.c_double()
        minv = np.zeros(self.d)
        self._check(self._lib.pcv_adapt(self._ctx, n_adapt, target_accept, ctypes.byref(eps), _dptr(minv)),
                    "pcv_adapt")
        return {"step_size": eps.value, "inv_mass": minv}

    def save(self, path: str):
        """Checkpoint the run (state, accumulators, transition count) to `path`."""
        self._check(self._lib.pcv_save(self._ctx, os.fsencode(path)), "pcv_save")

    def load(self, path: str):
        """Resume from a checkpoint of the same model, data, folds and precision."""
        self._check(self._lib.pcv_load(self._ctx, os.fsencode(path)), "pcv_load")

    def timing_enable(self, on: bool = True):
        self._check(self._lib.pcv_timing_enable(self._ctx, 1 if on else 0), "pcv_timing_enable")

    def timing_read(self, reset: bool = True):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        name = ctypes.c_char_p()
        self._check(self._lib.pcv_timing_read(self._ctx, ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(name), 1 if reset else 0), "pcv_timing_read")
        return ms.value, n.value, name.value.decode()
