"""Parity of the HIP library against the CPU oracle (needs an MI355X).

Every comparison uses the same seeded inputs on both sides; expected values
come only from the oracle.  Tolerances:
  fp64 paths            1e-12 relative (log pi; normwise per chain for vectors)
  fp32 VALU path        1e-5
  bf16 split paths      leapfrog positions/momenta 1e-5 normwise per chain;
                        log pi 1e-5 relative; gradient 1e-5 (BF16X5) and 5e-5
                        (BF16X3, whose two-term theta carries ~2^-17 relative
                        error into eta and from there into the residuals)
"""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import closed_form, diagnostics, folds, hmc, model, philox, sampler
from paper_2310_07002_amd import binding, workloads as W

pytestmark = pytest.mark.gpu

PREC = {"fp64": W.PREC_FP64, "fp32": W.PREC_FP32, "bf16x3": W.PREC_BF16X3, "bf16x5": W.PREC_BF16X5,
        "fp64u": W.PREC_FP64_UNFUSED}


def _say(msg):
    print(msg, flush=True)


def _normwise(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _oracle_eval(w, theta):
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    return (model.log_density(w, theta, roles, foc), model.grad_log_density(w, theta, roles, foc))


def _theta_near_init(w, scale=0.3, seed=0):
    rng = np.random.default_rng(seed)
    return w.init_pos + scale * np.sqrt(w.inv_mass)[None, :] * rng.standard_normal(w.init_pos.shape)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


# ---------------------------------------------------------------- random streams

def test_philox_bit_exact(dev):
    for seed, ctr in [(0, (0, 0, 0, 0)), (0xFFFFFFFFFFFFFFFF, (0xFFFFFFFF,) * 4),
                      (0x299F31D0A4093822, (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344)),
                      (20231007 * 10 + 2, (7, 123, 1, 0))]:
        got = binding.pcv_philox(seed, *ctr, 64)
        k = philox.seed_key(seed)
        want = np.stack([np.asarray(x, dtype=np.uint64) for x in philox.philox4x32_10(
            (np.uint64(ctr[0]), np.uint64(ctr[1]), np.uint64(ctr[2]),
             (np.uint64(ctr[3]) + np.arange(64, dtype=np.uint64)) & np.uint64(0xFFFFFFFF)), k)], axis=1)
        np.testing.assert_array_equal(got.astype(np.uint64), want)


# ---------------------------------------------------------------- value and gradient

CASES = [
    ("c1", "fp64", None, 1e-12, 1e-12),
    ("c3", "fp64", (0, 40), 1e-12, 1e-12),
    ("c2", "fp32", None, 1e-5, 1e-5),
    ("c4", "fp64u", (0, 16), 1e-12, 1e-12),
    ("c4", "fp64", (0, 16), 1e-12, 1e-12),
    ("c4", "bf16x5", (0, 16), 1e-5, 1e-5),
    ("c4", "bf16x3", (0, 16), 1e-5, 5e-5),
    ("c4", "fp32", (0, 16), 1e-5, 1e-5),
    ("c5", "bf16x5", (100, 140), 1e-5, 1e-5),
    ("c5", "bf16x3", (100, 140), 1e-5, 5e-5),
]


@pytest.mark.parametrize("name,prec,folds_,tol_v,tol_g", CASES)
def test_logdensity_grad_matches_oracle(dev, name, prec, folds_, tol_v, tol_g):
    w = W.make(name)
    if folds_:
        w = W.fold_subset(w, *folds_)
    _say(f"[logdensity] {name} {prec} C={w.C}")
    theta = _theta_near_init(w)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    rel_v = np.abs(lp - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g, g_o)
    _say(f"    logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e} median {np.median(rel_g):.2e}")
    assert rel_v.max() < tol_v
    assert rel_g.max() < tol_g


def test_ragged_chain_tile_and_row_tail(dev):
    """C not a multiple of the 256-chain tile, n not a multiple of the 32-row tile."""
    w = W.fold_subset(W.make("c4"), 3, 40)          # 296 chains
    w = dataclasses.replace(w, X=w.X[:19990], y=w.y[:19990], fold_index=w.fold_index[:19990])
    _say(f"[ragged] C={w.C} n={w.n}")
    theta = _theta_near_init(w, seed=3)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=W.PREC_BF16X5)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    assert (np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)).max() < 1e-5
    assert _normwise(g.cpu().numpy(), g_o).max() < 1e-5


def _intervals_of_blocks(w, h):
    """The blocked folds of w in the interval encoding, with h excluded rows
    on each side of every test block."""
    iv = np.zeros((w.K, 4), dtype=np.int64)
    for k in range(w.K):
        rows = np.flatnonzero(w.fold_index == k)
        lo, hi = int(rows.min()), int(rows.max()) + 1
        assert hi - lo == rows.size               # blocked folds are contiguous
        iv[k] = (lo, hi, max(0, lo - h), min(w.n, hi + h))
    return dataclasses.replace(w, fold_kind=W.FOLDS_INTERVALS, intervals=iv, fold_index=None)


SHAPE_CASES = [
    # (label, workload builder, precision, tol_v, tol_g)
    ("c4-index", lambda: W.fold_subset(W.make("c4"), 0, 16), "bf16x3", 1e-5, 5e-5),
    ("c4-index", lambda: W.fold_subset(W.make("c4"), 0, 16), "bf16x5", 1e-5, 1e-5),
    ("c5-index", lambda: W.fold_subset(W.make("c5"), 100, 140), "bf16x3", 1e-5, 5e-5),
    ("c5-intervals", lambda: _intervals_of_blocks(W.fold_subset(W.make("c5"), 100, 140), 7), "bf16x3", 1e-5, 5e-5),
    ("c5-intervals", lambda: _intervals_of_blocks(W.fold_subset(W.make("c5"), 100, 140), 7), "bf16x5", 1e-5, 1e-5),
    ("c4-ragged", lambda: (lambda w: dataclasses.replace(w, X=w.X[:19990], y=w.y[:19990],
                                                         fold_index=w.fold_index[:19990]))(
        W.fold_subset(W.make("c4"), 3, 40)), "bf16x3", 1e-5, 5e-5),
]


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("label,make_w,prec,tol_v,tol_g", SHAPE_CASES)
def test_mfma_tile_shapes_match_oracle(dev, shape, label, make_w, prec, tol_v, tol_g):
    """Every launch shape of the matrix-core kernel (16x16x32 tiles with 32 or
    16 chains per wave; 32x32x16 tiles in program order or scheduled by the
    compiler) at several row-split counts: value and gradient against the
    oracle, index and interval folds, a ragged chain tile and row tail.  The
    16-chain shape exists for designs of up to 64 columns only and is refused
    at width 128."""
    w = make_w()
    theta = _theta_near_init(w, seed=7)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    if shape == 3 and w.p > 64:
        cfg = s.launch_config()
        with pytest.raises(binding.PcvError):
            s.set_launch_config(256 * 3 + 1)
        assert s.launch_config() == cfg
        s.close()
        return
    n_tiles = (w.n + 31) // 32
    for ns in (1, 7, min(64, n_tiles)):
        s.set_launch_config(256 * shape + ns)
        cfg = s.launch_config()
        assert cfg // 256 == shape
        lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
        rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
        rel_g = _normwise(g.cpu().numpy(), g_o)
        _say(f"[shape {shape}] {label} {prec} C={w.C} n={w.n} config {cfg}: logp rel max {rel_v.max():.2e}  "
             f"grad normwise max {rel_g.max():.2e}")
        assert rel_v.max() < tol_v
        assert rel_g.max() < tol_g
    with pytest.raises(binding.PcvError):
        s.set_launch_config(256 * 4 + 1)
    assert s.launch_config() == cfg
    s.close()


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("label,make_w,prec", [(c[0], c[1], c[2]) for c in SHAPE_CASES if c[2] == "bf16x3"])
def test_leapfrog_every_tile_shape_matches_oracle(dev, shape, label, make_w, prec):
    """Eight leapfrog steps in every launch shape: seven gradient-only
    launches (where the masks are applied after the tile's MFMAs, on tiles
    whose flag marks the wave) and one value launch, against the oracle's
    trajectory at the 8-step BF16X3 bound."""
    w = make_w()
    if shape == 3 and w.p > 64:
        pytest.skip("the 16-chain shape is for designs of up to 64 columns")
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    q0 = _theta_near_init(w, seed=11)
    p0 = philox.momentum_normals(w.seed, w.chain_offset + np.arange(w.C), 0, w.d) / np.sqrt(w.inv_mass)
    g0 = model.grad_log_density(w, q0, roles, foc)
    q1, p1, _, lp1 = hmc.leapfrog(w, q0, p0, g0, 8, w.step_size, roles, foc)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    s.set_launch_config(256 * shape + 7)
    qg, pg, lpg, _ = s.leapfrog(torch.tensor(q0, device=dev), torch.tensor(p0, device=dev), 8)
    eq = _normwise(qg.cpu().numpy(), q1)
    ep = _normwise(pg.cpu().numpy(), p1)
    ev = np.abs(lpg.cpu().numpy() - lp1) / np.abs(lp1)
    _say(f"[leapfrog shape {shape}] {label}: q {eq.max():.2e}  p {ep.max():.2e}  logp {ev.max():.2e}")
    assert eq.max() < 2e-5 and ep.max() < 2e-5 and ev.max() < 2e-5
    s.close()


@pytest.mark.parametrize("name,folds_,prec,tol", [("c2", (0, 10), "fp32", 2e-6), ("c3", (0, 40), "fp64", 1e-12)])
def test_row_split_waves_and_splits_match_oracle(dev, name, folds_, prec, tol):
    """The row-split VALU path at several launch shapes, 1024 x waves per
    workgroup + row splits (the hierarchical family and interval folds):
    value and gradient against the oracle at each; shapes the path cannot
    run are refused and leave the context as it was."""
    w = W.fold_subset(W.make(name), *folds_)
    theta = _theta_near_init(w, seed=6)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    for W_, ns in ((1, 3), (2, 17), (4, 1), (8, 9), (8, 40)):
        cfg = 1024 * W_ + ns
        s.set_launch_config(cfg)
        assert s.launch_config() == cfg
        lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
        rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
        rel_g = _normwise(g.cpu().numpy(), g_o)
        _say(f"[row-split shape] {name} {prec} waves {W_} splits {ns}: logp rel max {rel_v.max():.2e}  "
             f"grad normwise max {rel_g.max():.2e}")
        assert rel_v.max() < tol and rel_g.max() < tol
    for bad in (1024 * 3 + 4, 1024 * 16 + 4, 1024 * 4 + 0, 1024 * 8 + 1000):   # waves 3, 16; no split; too many
        with pytest.raises(binding.PcvError):
            s.set_launch_config(bad)
    assert s.launch_config() == 1024 * 8 + 40
    s.step(2)
    th, lp2, _ = s.get_state()
    assert np.isfinite(th).all() and np.isfinite(lp2).all()
    s.close()


@pytest.mark.parametrize("prec,tol_v,tol_g", [("bf16x3", 1e-5, 5e-5), ("bf16x5", 1e-5, 1e-5)])
def test_interval_folds_on_matrix_cores(dev, prec, tol_v, tol_g):
    """hv-block style folds (test block plus a buffer of h rows each side,
    interval encoding) through the matrix-core path: rows excluded for a
    chain's fold must drop out of its value and gradient."""
    w = W.fold_subset(W.make("c5"), 100, 140)
    h = 7
    iv = np.zeros((w.K, 4), dtype=np.int64)
    for k in range(w.K):
        rows = np.flatnonzero(w.fold_index == k)
        lo, hi = int(rows.min()), int(rows.max()) + 1
        assert hi - lo == rows.size               # blocked folds are contiguous
        iv[k] = (lo, hi, max(0, lo - h), min(w.n, hi + h))
    w = dataclasses.replace(w, fold_kind=W.FOLDS_INTERVALS, intervals=iv, fold_index=None)
    _say(f"[intervals] {prec} C={w.C} K={w.K} h={h}")
    theta = _theta_near_init(w, seed=5)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g.cpu().numpy(), g_o)
    _say(f"    logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
    assert rel_v.max() < tol_v
    assert rel_g.max() < tol_g


def _mixed_intervals(w, h=6):
    """Interval folds in four forms, cycling over the folds so that one
    wave's lanes mix them: no exclusion range, an exclusion range touching
    the test block from above or from below, and a buffer on both sides."""
    iv = w.intervals.copy()
    for k in range(w.K):
        lo, hi = int(iv[k, 0]), int(iv[k, 1])
        iv[k] = [(lo, hi, lo, lo), (lo, hi, hi, min(w.n, hi + 3)), (lo, hi, max(0, lo - 4), lo),
                 (lo, hi, max(0, lo - h), min(w.n, hi + h))][k % 4]
    return dataclasses.replace(w, intervals=iv)


@pytest.mark.parametrize("path", ["split", "fused", "mfma"])
def test_interval_fold_forms(dev, path):
    """The four interval forms on the row-split VALU path (all 4996 rows),
    the fused VALU path (rows cut under 2048) and the matrix cores (blocked
    folds recoded as intervals): value and gradient against the oracle, and
    on the VALU paths three whole transitions replayed."""
    if path == "mfma":
        w = W.fold_subset(W.make("c5"), 100, 132)
        iv = np.zeros((w.K, 4), dtype=np.int64)
        for k in range(w.K):
            rows = np.flatnonzero(w.fold_index == k)
            iv[k] = (rows.min(), rows.max() + 1, 0, 0)
        w = dataclasses.replace(w, fold_kind=W.FOLDS_INTERVALS, intervals=iv, fold_index=None)
        tol, prec = 1e-5, W.PREC_BF16X5
    else:
        w = W.fold_subset(W.make("c3"), 296, 336)
        if path == "fused":
            n = 1800
            w = dataclasses.replace(w, X=w.X[:n], y=w.y[:n],
                                    intervals=np.minimum(w.intervals, n))
        tol, prec = 1e-12, W.PREC_FP64
    w = dataclasses.replace(_mixed_intervals(w), n_warmup=2)
    _say(f"[interval forms] {path} n={w.n} C={w.C}")
    theta = _theta_near_init(w, seed=6)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=prec)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g.cpu().numpy(), g_o)
    _say(f"    logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
    assert rel_v.max() < tol
    assert rel_g.max() < tol
    if path != "mfma":
        run, s2 = _replay(w, 3, dev, prec=prec)
        th, _, sv = s2.get_state()
        np.testing.assert_allclose(th, run.state.q, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(sv, run.state.s, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
@pytest.mark.parametrize("lagged", [True, False])
def test_autoregressive_rows_on_split_path(dev, prec, lagged):
    """The AR(4) design (every row's lags are the previous row's response and
    lags, which the row-split kernel slides in registers) with index-coded
    contiguous folds, and the same design one ulp off that identity (the
    general row loop): value and gradient against the oracle, and in fp64
    three whole transitions replayed."""
    w = W.fold_subset(W.make("c3"), 296, 336)
    X = w.X.copy()
    if not lagged:
        X[700, 2] = np.nextafter(X[700, 2], np.inf)
    fi = (np.arange(w.n) * w.K // w.n).astype(np.int32)
    w = dataclasses.replace(w, X=X, fold_kind=W.FOLDS_INDEX, fold_index=fi, intervals=None, n_warmup=2)
    _say(f"[autoregressive rows] lagged={lagged} prec={prec} n={w.n} C={w.C}")
    theta = _theta_near_init(w, seed=8)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=prec)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g.cpu().numpy(), g_o)
    _say(f"    logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
    tol = 1e-12 if prec == W.PREC_FP64 else 1e-5
    assert rel_v.max() < tol
    assert rel_g.max() < tol
    if prec == W.PREC_FP64:
        run, s2 = _replay(w, 3, dev, prec=prec)
        th, _, sv = s2.get_state()
        np.testing.assert_allclose(th, run.state.q, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(sv, run.state.s, rtol=1e-10, atol=1e-12)


def test_dense_fold_encoding_matches_index(dev):
    w = W.fold_subset(W.make("c1"), 0, 30)
    wd = W.with_dense_roles(w)
    theta = _theta_near_init(w, seed=4)
    t = torch.tensor(theta, device=dev)
    lp1, g1 = binding.PCV.from_workload(w).logdensity_grad(t)
    lp2, g2 = binding.PCV.from_workload(wd).logdensity_grad(t)
    np.testing.assert_allclose(lp2.cpu().numpy(), lp1.cpu().numpy(), rtol=1e-14)
    np.testing.assert_allclose(g2.cpu().numpy(), g1.cpu().numpy(), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- single leapfrog trajectories

@pytest.mark.parametrize("name,prec,folds_,tol", [("c1", "fp64", None, 1e-12), ("c3", "fp64", (0, 30), 1e-12),
                                                 ("c2", "fp32", (0, 10), 1e-5),
                                                 ("c4", "fp64", (0, 16), 1e-12),
                                                 ("c4", "bf16x3", (0, 16), 1e-5),
                                                 ("c5", "bf16x3", (0, 32), 1e-5),
                                                 ("c5", "bf16x5", (0, 32), 1e-5)])
@pytest.mark.parametrize("n_steps", [1, 8])
def test_leapfrog_matches_oracle(dev, name, prec, folds_, tol, n_steps):
    """One step at the stated tolerance.  Over a whole 8-step trajectory the
    BF16X3 gradient error (~2e-5 normwise) enters the momentum once per step,
    so its bound there is 2e-5."""
    if prec == "bf16x3" and n_steps > 1:
        tol = 2e-5
    w = W.make(name)
    if folds_:
        w = W.fold_subset(w, *folds_)
    _say(f"[leapfrog] {name} {prec} steps={n_steps}")
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    q0 = _theta_near_init(w, seed=5)
    p0 = philox.momentum_normals(w.seed, w.chain_offset + np.arange(w.C), 0, w.d) / np.sqrt(w.inv_mass)
    g0 = model.grad_log_density(w, q0, roles, foc)
    q1, p1, g1, lp1 = hmc.leapfrog(w, q0, p0, g0, n_steps, w.step_size, roles, foc)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    qg, pg, lpg, gg = s.leapfrog(torch.tensor(q0, device=dev), torch.tensor(p0, device=dev), n_steps)
    eq = _normwise(qg.cpu().numpy(), q1)
    ep = _normwise(pg.cpu().numpy(), p1)
    ev = np.abs(lpg.cpu().numpy() - lp1) / np.abs(lp1)
    _say(f"    q {eq.max():.2e}  p {ep.max():.2e}  logp {ev.max():.2e}")
    assert eq.max() < tol and ep.max() < tol and ev.max() < tol


# ---------------------------------------------------------------- whole runs

def _replay(w, n_iter, dev, prec=None):
    run = sampler.run_all(w, n_iter=n_iter)
    s = binding.PCV.from_workload(w, precision=prec)
    s.step(n_iter)
    return run, s


def test_fp64_run_replays_oracle_c1(dev):
    w = dataclasses.replace(W.make("c1"), n_warmup=100)
    _say("[replay] c1 fp64 300 iterations")
    run, s = _replay(w, 300, dev)
    th, lp, sv = s.get_state()
    np.testing.assert_allclose(th, run.state.q, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(sv, run.state.s, rtol=1e-9, atol=1e-10)
    acc = s.get_accumulators(w.n_blocks)
    np.testing.assert_array_equal(acc["n_accept"], run.acc.n_accept)
    for k in ("Z", "U", "U2", "V", "V2"):
        np.testing.assert_allclose(acc[k], getattr(run.acc, k), rtol=1e-9, err_msg=k)
    np.testing.assert_allclose(acc["blk_mean"], run.acc.blk_mean, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(acc["blk_m2"], run.acc.blk_m2, rtol=1e-8, atol=1e-9)
    # diagnostics from the device accumulators vs the oracle's own
    d = s.diagnostics()
    o = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    assert abs(d["elpd"] - o["elpd"]) < 1e-9 * abs(o["elpd"])
    assert abs(d["rhat_max"] - o["rhat_max"]) < 1e-9
    assert abs(d["mcse"] - o["mcse"]) < 1e-8 * o["mcse"]
    assert abs(d["ess"] - o["ess"]) < 1e-8 * o["ess"]
    np.testing.assert_allclose(d["rhat_fold"], o["rhat_fold"], rtol=1e-9)
    np.testing.assert_allclose(d["ess_fold"], o["ess_fold"], rtol=1e-7)
    e = s.elpd()
    np.testing.assert_allclose(e["elpd_fold"], o["elpd_fold"], rtol=1e-10)
    np.testing.assert_allclose(e["mcse_fold"], o["mcse_fold"], rtol=1e-7)
    assert d["accept_rate"] == pytest.approx(o["accept_rate"], rel=1e-12)
    rep_g = s.shuffle_benchmark(20, seed=17)
    _, rep_o = diagnostics.shuffle_benchmark(run.acc, w.K, w.L, w.n_blocks, 20, seed=17)
    np.testing.assert_allclose(rep_g, rep_o, rtol=1e-9)


def test_shifted_sums_rhat_replays_oracle(dev):
    """rhat_mode = shifted sums (Algorithm A2): the fold centres are fixed when
    the warm-up ends (here inside a pcv_step call), then the device's block
    sums, Rhat and block-shuffle benchmark follow the oracle's."""
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 30), n_warmup=60, rhat_mode=1)
    run = sampler.run_all(w, n_iter=260)
    s = binding.PCV.from_workload(w)
    for n in (37, 100, 123):
        s.step(n)
    acc = s.get_accumulators(w.n_blocks)
    np.testing.assert_allclose(acc["blk_mean"], run.acc.blk_mean, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(acc["blk_m2"], run.acc.blk_m2, rtol=1e-9, atol=1e-9)
    d = s.diagnostics()
    o = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
    np.testing.assert_allclose(d["rhat_fold"], o["rhat_fold"], rtol=1e-9)
    rep_g = s.shuffle_benchmark(20, seed=5)
    _, rep_o = diagnostics.shuffle_benchmark(run.acc, w.K, w.L, w.n_blocks, 20, seed=5)
    np.testing.assert_allclose(rep_g, rep_o, rtol=1e-9)


def test_shifted_sums_equal_welford_on_matrix_cores(dev):
    w = dataclasses.replace(W.fold_subset(W.make("c4"), 0, 30), n_warmup=20, batch_size=10)
    a = binding.PCV.from_workload(w, precision=W.PREC_BF16X3, rhat_mode=binding.RHAT_WELFORD)
    b = binding.PCV.from_workload(w, precision=W.PREC_BF16X3, rhat_mode=binding.RHAT_SHIFTED_SUMS)
    for x in (a, b):
        x.step(15)
        x.step(60)
    np.testing.assert_array_equal(a.get_state()[0], b.get_state()[0])
    da, db = a.diagnostics(), b.diagnostics()
    assert da["elpd"] == db["elpd"]
    np.testing.assert_allclose(db["rhat_fold"], da["rhat_fold"], rtol=1e-9)
    np.testing.assert_allclose(b.shuffle_benchmark(10, seed=2), a.shuffle_benchmark(10, seed=2), rtol=1e-9)


def test_fp64_run_replays_oracle_hvblock(dev):
    w = dataclasses.replace(W.fold_subset(W.make("c3"), 0, 25), n_warmup=40)
    _say("[replay] c3 fp64 subset 120 iterations")
    run, s = _replay(w, 120, dev)
    th, lp, sv = s.get_state()
    np.testing.assert_allclose(th, run.state.q, rtol=1e-9, atol=1e-10)
    acc = s.get_accumulators(w.n_blocks)
    np.testing.assert_array_equal(acc["n_accept"], run.acc.n_accept)
    np.testing.assert_allclose(acc["U"], run.acc.U, rtol=1e-9)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x5"])
def test_bf16_run_tracks_oracle_c5(dev, prec):
    """Split-precision transitions: accept decisions may differ where the
    energy error decides; every other chain must track the fp64 oracle."""
    w = dataclasses.replace(W.fold_subset(W.make("c5"), 0, 32), n_warmup=2)
    _say(f"[replay] c5 {prec} subset 4 iterations")
    run, s = _replay(w, 4, dev, prec=PREC[prec])
    th, lp, sv = s.get_state()
    err = _normwise(th, run.state.q)
    acc = s.get_accumulators(w.n_blocks)
    same = acc["n_accept"] == run.acc.n_accept
    _say(f"    same decisions {same.mean():.3f}  max err (same) {err[same].max():.2e}")
    assert same.mean() > 0.97
    assert err[same].max() < 1e-5


def _regrouped(w):
    """The hierarchical design of w with its groups relabelled so that row 0
    is a group of its own, every original group g becomes group 2g+1, and
    the even groups in between (and one past the end) have no rows: only
    their prior informs them.  Rows stay sorted by group."""
    g = 2 * w.group_of.astype(np.int64) + 1
    g[0] = 0
    G2 = 2 * w.n_groups + 2
    p = w.p
    z_of = np.zeros(G2, dtype=np.int64) - 1          # original group behind each new group
    z_of[2 * np.arange(w.n_groups) + 1] = np.arange(w.n_groups)
    z_of[0] = w.group_of[0]
    def expand(a, fill):                              # [..., p + 2 + G] -> [..., p + 2 + G2]
        out = np.full(a.shape[:-1] + (p + 2 + G2,), fill, dtype=np.float64)
        out[..., :p + 2] = a[..., :p + 2]
        has = z_of >= 0
        out[..., p + 2:][..., has] = a[..., p + 2 + z_of[has]]
        return out
    return dataclasses.replace(w, group_of=g.astype(np.int32), n_groups=G2,
                               init_pos=expand(w.init_pos, 0.0), inv_mass=expand(w.inv_mass, 1.0),
                               prior_scale=expand(w.prior_scale, 1.0),
                               truth=expand(w.truth, 0.0) if w.truth is not None else None)


@pytest.mark.parametrize("n_keep", [22, 12])
def test_hier_empty_and_single_row_groups(dev, n_keep):
    """Hierarchical groups with no rows and with one row, and groups that
    straddle waves and row splits, on the rows of the first n_keep groups of
    the LOGO workload: 22 groups (over 2048 rows, 64 chains) run on the
    row-split path, 12 groups (under 2048 rows) on the fused path.  fp64,
    against the oracle."""
    base = W.make("c2")
    rows = int(np.searchsorted(base.group_of, n_keep))
    base = dataclasses.replace(base, X=base.X[:rows], y=base.y[:rows], fold_index=base.fold_index[:rows],
                               group_of=base.group_of[:rows], n_groups=n_keep, K=n_keep,
                               init_pos=base.init_pos[:n_keep * base.L, :base.p + 2 + n_keep],
                               inv_mass=base.inv_mass[:base.p + 2 + n_keep],
                               prior_scale=base.prior_scale[:base.p + 2 + n_keep],
                               truth=base.truth[:base.p + 2 + n_keep])
    assert (rows >= 2048) == (n_keep == 22)
    w = dataclasses.replace(_regrouped(W.fold_subset(base, 0, 4)), precision=W.PREC_FP64, n_warmup=2)
    _say(f"[hier groups] n={w.n} groups={w.n_groups} C={w.C}")
    theta = _theta_near_init(w, seed=11)
    lp_o, g_o = _oracle_eval(w, theta)
    s = binding.PCV.from_workload(w, precision=W.PREC_FP64)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g.cpu().numpy(), g_o)
    _say(f"    logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
    assert rel_v.max() < 1e-12
    assert rel_g.max() < 1e-12
    # three whole transitions replay the oracle
    run, s2 = _replay(w, 3, dev, prec=W.PREC_FP64)
    th, _, sv = s2.get_state()
    np.testing.assert_allclose(th, run.state.q, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(sv, run.state.s, rtol=1e-10, atol=1e-12)


def test_hier_fp32_run_tracks_oracle(dev):
    w = dataclasses.replace(W.make("c2"), n_warmup=2)
    w = W.fold_subset(w, 0, 10)
    _say("[replay] c2 fp32 subset 4 iterations")
    run, s = _replay(w, 4, dev)
    th, lp, sv = s.get_state()
    err = _normwise(th, run.state.q)
    acc = s.get_accumulators(w.n_blocks)
    same = acc["n_accept"] == run.acc.n_accept
    _say(f"    same decisions {same.mean():.3f}  max err (same) {err[same].max():.2e}")
    assert same.mean() > 0.95
    assert err[same].max() < 1e-4


def test_loo_elpd_within_mcse_of_closed_form(dev):
    """Full first configuration on the device: elpd within 4 MCSE of the exact LOO."""
    w = W.make("c1")
    s = binding.PCV.from_workload(w)
    s.step(w.n_iter)
    d = s.diagnostics()
    roles = folds.roles_of(w)
    exact = sum(closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1, roles[k] == 2)["elpd"]
                for k in range(w.K))
    _say(f"[c1 full] elpd {d['elpd']:.4f} exact {exact:.4f} mcse {d['mcse']:.4f} rhat_max {d['rhat_max']:.4f}")
    assert abs(d["elpd"] - exact) < 4 * d["mcse"]
    assert d["n_draws"] == w.n_samples


@pytest.mark.parametrize("name,prec,folds_", [("c1", "fp64", (0, 8)), ("c3", "fp64", (0, 16)),
                                              ("c4", "fp64", (0, 4)), ("c4", "fp64u", (0, 4)),
                                              ("c2", "fp64", (0, 3))])
def test_autograd_function_matches_finite_differences(dev, name, prec, folds_):
    """PCVLogDensity's backward is the hand-written adjoint: against central
    differences (h = 1e-6) of the same kernel's fp64 log density on every
    fp64 path -- the fused VALU kernel (c1), the row-split VALU kernel for
    interval folds (c3), for the Poisson GLM at p = 64 (c4) and for the
    hierarchical family (c2, the groups' chain rule), and the plain
    library-GEMM path.  A central difference of a smooth f errs by about
    h^2/6 times its third derivative plus 2^-52 |f| / h of rounding; with
    |log pi| <= 3e4 here that is below 2e-4 absolute."""
    from paper_2310_07002_amd.autograd import log_density
    w = W.fold_subset(W.make(name), *folds_)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    _say(f"[autograd FD] {name} {prec} C={w.C} d={w.d}")
    theta = torch.tensor(_theta_near_init(w, seed=9), device=dev, requires_grad=True)
    weights = torch.linspace(0.5, 1.5, w.C, dtype=torch.float64, device=dev)
    (log_density(theta, s) * weights).sum().backward()
    g = theta.grad.cpu().numpy()
    h = 1e-6
    th = theta.detach().cpu().numpy()
    rng = np.random.default_rng(1)
    for j in sorted(rng.choice(w.d, size=min(6, w.d), replace=False).tolist()) + [w.d - 1]:
        e = np.zeros_like(th)
        e[:, j] = h
        lp_p, _ = s.logdensity_grad(torch.tensor(th + e, device=dev), want_grad=False)
        lp_m, _ = s.logdensity_grad(torch.tensor(th - e, device=dev), want_grad=False)
        fd = (lp_p - lp_m).cpu().numpy() / (2 * h) * weights.cpu().numpy()
        np.testing.assert_allclose(g[:, j], fd, rtol=2e-5, atol=2e-4, err_msg=f"coordinate {j}")


@pytest.mark.parametrize("name,prec,folds_,tol", [("c4", "bf16x5", (0, 16), 1e-5), ("c4", "bf16x3", (0, 16), 5e-5),
                                                 ("c5", "bf16x3", (0, 8), 5e-5), ("c2", "fp32", (0, 4), 1e-5)])
def test_autograd_function_matches_fp64_reference(dev, name, prec, folds_, tol):
    """PCVLogDensity over the split-precision matrix-core adjoint and the fp32
    VALU adjoint: the backward (weighted by grad_out) equals the fp64
    oracle's gradient at the normwise tolerance stated for each precision."""
    from paper_2310_07002_amd.autograd import log_density
    w = W.fold_subset(W.make(name), *folds_)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    th = _theta_near_init(w, seed=12)
    theta = torch.tensor(th, device=dev, requires_grad=True)
    weights = torch.linspace(0.5, 1.5, w.C, dtype=torch.float64, device=dev)
    lp = log_density(theta, s)
    (lp * weights).sum().backward()
    lp_o, g_o = _oracle_eval(w, th)
    wv = weights.cpu().numpy()[:, None]
    err = _normwise(theta.grad.cpu().numpy(), wv * g_o)
    _say(f"[autograd ref] {name} {prec}: grad normwise max {err.max():.2e}")
    assert err.max() < tol
    assert (np.abs(lp.detach().cpu().numpy() - lp_o) / np.abs(lp_o)).max() < 1e-5


def test_state_roundtrip_and_divergence_counting(dev):
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 8), n_warmup=0, step_size=5.0)
    s = binding.PCV.from_workload(w)
    th0, lp0, s0 = s.get_state()
    np.testing.assert_allclose(th0, w.init_pos, rtol=0, atol=0)
    s.step(10)
    d = s.diagnostics()
    assert d["n_divergent"] > 0
    s.set_state(w.init_pos)
    th1, lp1, s1 = s.get_state()
    np.testing.assert_array_equal(th1, th0)
    np.testing.assert_allclose(lp1, lp0, rtol=1e-15)


@pytest.mark.parametrize("name,prec,folds_,tol_v,tol_g", [("c1", "fp64", None, 1e-12, 1e-12),
                                                        ("c2", "fp32", None, 1e-5, 1e-5),
                                                        ("c4", "bf16x3", (0, 64), 1e-5, 5e-5)])
def test_autotune_keeps_parity_and_caches(dev, tmp_path, name, prec, folds_, tol_v, tol_g):
    """The tuned launch shape changes only the order of sums: the log density
    and gradient still match the oracle, the shape is cached in JSON, a second
    context takes it from the cache, and the sampler steps with it."""
    import json
    w = W.make(name)
    if folds_:
        w = W.fold_subset(w, *folds_)
    cache = str(tmp_path / "tune.json")
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    r = s.autotune(cache)
    _say(f"[autotune] {name} {prec}: config {r['config']} {r['ms']:.4f} ms")
    assert r["config"] >= 1 and r["ms"] > 0
    theta = _theta_near_init(w, seed=7)
    lp_o, g_o = _oracle_eval(w, theta)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    assert (np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)).max() < tol_v
    assert _normwise(g.cpu().numpy(), g_o).max() < tol_g
    entries = json.load(open(cache))
    assert len(entries) == 1 and list(entries.values())[0]["cfg"] == r["config"]
    s2 = binding.PCV.from_workload(w, precision=PREC[prec])
    r2 = s2.autotune(cache)
    assert r2["config"] == r["config"] and r2["ms"] == pytest.approx(r["ms"], rel=1e-6)
    s2.step(3)
    th, lp2, _ = s2.get_state()
    assert np.isfinite(th).all() and np.isfinite(lp2).all()


def test_design_as_bf16_planes_matches_fp64_design(dev, tmp_path):
    """X handed over as its stored bf16 hi/lo planes is the same design as its
    fp64 sum: identical results, and checkpoints are interchangeable."""
    w = W.fold_subset(W.make("c4"), 0, 24)
    a = binding.PCV.from_workload(w, precision=W.PREC_BF16X3)
    b = binding.PCV.from_workload(w, precision=W.PREC_BF16X3, x_planes=True)
    theta = torch.tensor(_theta_near_init(w, seed=2), device=dev)
    for x, y in zip(a.logdensity_grad(theta), b.logdensity_grad(theta)):
        torch.testing.assert_close(x, y, rtol=0, atol=0)
    a.step(3)
    a.save(str(tmp_path / "a.ckpt"))
    b.load(str(tmp_path / "a.ckpt"))
    b.step(2)
    a.step(2)
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x5"])
def test_general_fp64_design_on_matrix_cores(dev, prec):
    """A design that is not a stored bf16 pair (a generic fp64 matrix) on the
    matrix-core path: the library rounds each entry to fp32 and keeps it as a
    bf16 hi + lo pair, 16 significant bits, so |x - x_kept| <= 2^-16 |x|
    (fp32 rounding 2^-24 plus the lo term's rounding 2^-17 of |x|, rounded
    up).  That moves eta and the gradient by at most 2^-16 times the sums of
    |x theta| and |x r|; the tolerances below are that bound times the
    cancellation these sums show on the workload, with a factor 4 to spare,
    on top of the stored-pair tolerances."""
    w = W.fold_subset(W.make("c4"), 0, 16)
    rng = np.random.default_rng(12)
    X = w.X * (1.0 + 1e-3 * rng.standard_normal(w.X.shape))     # no longer a bf16 pair
    w = dataclasses.replace(w, X=X, x_hi=None, x_lo=None)
    theta = _theta_near_init(w, seed=4)
    lp_o, g_o = _oracle_eval(w, theta)
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    eta = model.linear_predictor(w, theta)
    train = roles[foc].T == folds.ROLE_TRAIN
    r = train * model.dloglik_deta(w.family, w.y[:, None], eta, w.sigma)
    h = 1e-6
    dr = train * np.abs(model.dloglik_deta(w.family, w.y[:, None], eta + h, w.sigma)
                        - model.dloglik_deta(w.family, w.y[:, None], eta - h, w.sigma)) / (2 * h)
    u = 2.0 ** -16
    deta = u * (np.abs(w.X) @ np.abs(theta.T))                     # |eta change| per row and chain
    bound_v = np.sum(np.abs(r) * deta, axis=0) / np.abs(lp_o)
    bound_g = np.linalg.norm(u * (np.abs(w.X).T @ np.abs(r)) + np.abs(w.X).T @ (dr * deta), axis=0) \
        / np.linalg.norm(g_o, axis=1)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
    rel_g = _normwise(g.cpu().numpy(), g_o)
    base_v, base_g = 1e-5, (5e-5 if prec == "bf16x3" else 1e-5)
    _say(f"[general design] {prec}: logp rel max {rel_v.max():.2e} (bound {bound_v.max():.1e}), "
         f"grad normwise max {rel_g.max():.2e} (bound {bound_g.max():.1e})")
    assert np.all(rel_v < base_v + 4 * bound_v)
    assert np.all(rel_g < base_g + 4 * bound_g)
    s.close()


@pytest.mark.parametrize("name,prec,folds_,mode", [("c1", "fp64", (0, 12), 0), ("c4", "bf16x3", (0, 40), 0),
                                                  ("c1", "fp64", (0, 12), 1)])
def test_checkpoint_resume_is_exact(dev, tmp_path, name, prec, folds_, mode):
    """Run A: 30 transitions, save, 25 more.  Run B: a fresh context loads the
    checkpoint and runs 25.  Everything must agree bit for bit (random
    numbers are keyed by chain and transition).  With shifted sums the save
    falls inside the warm-up, so the resumed run fixes the fold centres from
    restored warm-up sums.  Checkpoints of another run and damaged files are
    refused and leave the context usable."""
    w = dataclasses.replace(W.fold_subset(W.make(name), *folds_), n_warmup=40 if mode else 12,
                            batch_size=4, rhat_mode=mode)
    path = str(tmp_path / "run.ckpt")
    _say(f"[checkpoint] {name} {prec} C={w.C}")
    a = binding.PCV.from_workload(w, precision=PREC[prec])
    a.step(30)
    a.save(path)
    a.step(25)
    b = binding.PCV.from_workload(w, precision=PREC[prec])
    b.load(path)
    b.step(25)
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)
    acc_a, acc_b = a.get_accumulators(w.n_blocks), b.get_accumulators(w.n_blocks)
    for k in acc_a:
        np.testing.assert_array_equal(acc_a[k], acc_b[k])
    da, db = a.diagnostics(), b.diagnostics()
    assert da["n_iter"] == db["n_iter"] == 55
    assert da["elpd"] == db["elpd"] and da["rhat_max"] == db["rhat_max"]

    other = binding.PCV.from_workload(dataclasses.replace(w, seed=w.seed + 1), precision=PREC[prec])
    with pytest.raises(binding.PcvError, match="another"):
        other.load(path)
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0x40
    bad = str(tmp_path / "flipped.ckpt")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(binding.PcvError, match="corrupted"):
        b.load(bad)
    short = str(tmp_path / "short.ckpt")
    open(short, "wb").write(bytes(raw[: len(raw) - 8]))
    with pytest.raises(binding.PcvError, match="corrupted"):
        b.load(short)
    b.step(1)                                   # still usable after refused loads
    assert b.diagnostics()["n_iter"] == 56


def test_checkpoint_guards_the_target_and_carries_the_tuning(dev, tmp_path):
    """A checkpoint is refused by a context whose target differs (noise scale
    or prior scales), and it carries the step size and inverse mass that
    window adaptation left: a fresh context created with the unadapted
    tuning resumes a post-adaptation checkpoint bit for bit."""
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 12), n_warmup=10)
    path = str(tmp_path / "t.ckpt")
    a = binding.PCV.from_workload(w)
    a.step(12)
    a.save(path)
    for other in (dataclasses.replace(w, sigma=w.sigma * 1.25),
                  dataclasses.replace(w, prior_scale=w.prior_scale * 2.0)):
        with pytest.raises(binding.PcvError, match="another"):
            binding.PCV.from_workload(other).load(path)
    f = W.full_data(W.make("c1"), L=8, n_warmup=400)
    x = binding.PCV.from_workload(f, precision=W.PREC_FP64)
    r = x.adapt(150, 0.8)
    assert r["step_size"] != f.step_size
    x.step(5)
    x.save(path)
    x.step(20)
    y = binding.PCV.from_workload(f, precision=W.PREC_FP64)     # created with the unadapted tuning
    y.load(path)
    y.step(20)
    for u, v in zip(x.get_state(), y.get_state()):
        np.testing.assert_array_equal(u, v)
    _say(f"[checkpoint] adapted eps {r['step_size']:.4f} resumed bit for bit")


@pytest.mark.parametrize("name,prec,tol_v,tol_g", [("c5", "bf16x3", 1e-5, 5e-5), ("c4", "bf16x3", 1e-5, 5e-5),
                                                   ("c5", "bf16x5", 1e-5, 1e-5), ("c3", "fp64", 1e-12, 1e-12)])
def test_full_size_sampled_parity(dev, name, prec, tol_v, tol_g):
    """The full configuration in the launch shape the benchmark times (all
    chains, all row splits, the autotuned split count), checked on sampled
    folds one at a time."""
    w = W.make(name)
    _say(f"[full size] {name} {prec} C={w.C}")
    theta = _theta_near_init(w, seed=11)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    tune = s.autotune()
    _say(f"    autotuned launch shape {tune['config']}")
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(lp)) and np.all(np.isfinite(g))
    rng = np.random.default_rng(5)
    worst_v = worst_g = 0.0
    for k in sorted(rng.choice(w.K, size=12, replace=False).tolist()) + [w.K - 1]:
        sub = W.fold_subset(w, k, k + 1)
        sl = slice(k * w.L, (k + 1) * w.L)
        lp_o, g_o = _oracle_eval(sub, theta[sl])
        worst_v = max(worst_v, float(np.max(np.abs(lp[sl] - lp_o) / np.abs(lp_o))))
        worst_g = max(worst_g, float(np.max(_normwise(g[sl], g_o))))
    _say(f"    sampled folds: logp rel max {worst_v:.2e}  grad normwise max {worst_g:.2e}")
    assert worst_v < tol_v
    assert worst_g < tol_g


def test_hvblock_elpd_within_mcse_of_closed_form(dev):
    """The full hv-block configuration (1000 folds x 8 chains, the autotuned
    launch shape): the device's elpd lies within 4 MCSE of the sum of the
    exact hv-block predictive densities (conjugate Gaussian, known sigma), and
    per fold within 4 MCSE but for the few folds that chance allows."""
    w = W.make("c3")
    s = binding.PCV.from_workload(w)
    s.autotune()
    s.step(w.n_iter)
    d = s.diagnostics()
    e = s.elpd()
    elpd_k, mcse_k = e["elpd_fold"], e["mcse_fold"]
    roles = folds.roles_of(w)
    exact_k = np.array([closed_form.fold_exact(w.X, w.y, w.sigma, w.prior_scale, roles[k] == 1,
                                               roles[k] == 2)["elpd"] for k in range(w.K)])
    z = np.abs(elpd_k - exact_k) / mcse_k
    _say(f"[c3 full] elpd {d['elpd']:.4f} exact {exact_k.sum():.4f} mcse {d['mcse']:.4f} "
         f"rhat_max {d['rhat_max']:.4f}; folds beyond 4 MCSE: {int(np.sum(z > 4))} of {w.K}, max z {z.max():.2f}")
    assert d["n_draws"] == w.n_samples
    assert abs(d["elpd"] - exact_k.sum()) < 4 * d["mcse"]
    assert np.sum(z > 4) <= 2 and z.max() < 6


@pytest.mark.parametrize("name,folds_,prec", [("c4", (0, 40), "bf16x3"), ("c3", (0, 40), "fp64"),
                                             ("c2", (0, 10), "fp32")])
def test_graph_replay_matches_eager(dev, name, folds_, prec):
    """Transitions replayed from the captured graph equal eager launches of
    the same kernels, replay after replay, with eager work in between: the
    matrix-core path (c4) and the row-split VALU path for interval folds
    (c3) and the hierarchical family (c2)."""
    w = dataclasses.replace(W.fold_subset(W.make(name), *folds_), n_warmup=3)
    _say(f"[graph] {name} {prec} C={w.C}")
    g = binding.PCV.from_workload(w, precision=PREC[prec])           # graph replays
    e = binding.PCV.from_workload(w, precision=PREC[prec])           # eager (timing on)
    e.timing_enable(True)
    for rep in range(4):
        g.step(2)
        e.step(2)
        th_g, lp_g, s_g = g.get_state()
        th_e, lp_e, s_e = e.get_state()
        np.testing.assert_array_equal(th_g, th_e)
        np.testing.assert_array_equal(s_g, s_e)
        # eager work on the graph context between replays
        lp, _ = g.logdensity_grad(torch.tensor(th_g, device=dev), want_grad=False)
        np.testing.assert_allclose(lp.cpu().numpy(), lp_g, rtol=1e-12)
    ag, ae = g.get_accumulators(w.n_blocks), e.get_accumulators(w.n_blocks)
    for k in ("U", "U2", "Z", "blk_mean", "blk_m2", "n_accept"):
        np.testing.assert_array_equal(ag[k], ae[k])


# ---------------------------------------------------------------- model comparison

def test_model_comparison_replays_oracle(dev):
    """LOO of the conjugate Gaussian: model A with all covariates, model B
    without its strongest one, both full runs; pcv_compare against the
    oracle's comparison of its own runs."""
    a = W.make("c1")
    b = W.drop_covariates(a, [int(np.argmax(np.abs(a.truth)))])
    _say("[compare] c1 fp64, full runs of both models")
    ra, rb = sampler.run_all(a), sampler.run_all(b)
    da = diagnostics.from_accumulators(ra.acc, a.K, a.L, a.batch_size)
    db = diagnostics.from_accumulators(rb.acc, b.K, b.L, b.batch_size)
    want = diagnostics.compare(da["elpd_fold"], da["mcse_fold"], db["elpd_fold"], db["mcse_fold"])
    sa, sb = binding.PCV.from_workload(a), binding.PCV.from_workload(b)
    sa.step(a.n_iter)
    sb.step(b.n_iter)
    got = sa.compare(sb)
    _say(f"    delta {got['delta']:.4f} (oracle {want['delta']:.4f}) mcse {got['mcse']:.4f} "
         f"Pr(A>B) {got['prob_a_better']:.6f}")
    assert got["delta"] == pytest.approx(want["delta"], rel=1e-9)
    assert got["sigma2"] == pytest.approx(want["sigma2"], rel=1e-8)
    assert got["prob_a_better"] == pytest.approx(want["prob_a_better"], abs=1e-9)
    assert got["mcse"] == pytest.approx(want["mcse"], rel=1e-7)
    np.testing.assert_allclose(got["delta_fold"], want["delta_fold"], rtol=1e-9, atol=1e-12)
    swapped = sb.compare(sa)
    assert swapped["delta"] == -got["delta"] and swapped["prob_a_better"] == pytest.approx(1 - got["prob_a_better"])


def test_model_comparison_on_matrix_cores(dev):
    """Nested logistic models on the bf16x3 path (model B: two columns
    zeroed); the comparison equals the oracle's formulas applied to the two
    runs' fold estimates, and runs on different folds are refused."""
    a = W.fold_subset(W.make("c5"), 0, 64)
    a = dataclasses.replace(a, n_warmup=20, batch_size=10)
    b = W.drop_covariates(a, [3, 77], zero=True)
    sa = binding.PCV.from_workload(a, precision=W.PREC_BF16X3)
    sb = binding.PCV.from_workload(b, precision=W.PREC_BF16X3, x_planes=True)
    sa.step(80)
    sb.step(80)
    ea, eb = sa.elpd(), sb.elpd()
    want = diagnostics.compare(ea["elpd_fold"], ea["mcse_fold"], eb["elpd_fold"], eb["mcse_fold"])
    got = sa.compare(sb)
    assert got["delta"] == pytest.approx(want["delta"], rel=1e-12, abs=1e-12)
    assert got["sigma2"] == pytest.approx(want["sigma2"], rel=1e-12)
    assert got["prob_a_better"] == pytest.approx(want["prob_a_better"], abs=1e-12)
    assert got["mcse"] == pytest.approx(want["mcse"], rel=1e-12)
    other = binding.PCV.from_workload(W.fold_subset(W.make("c5"), 64, 128), precision=W.PREC_BF16X3)
    other.step(25)
    with pytest.raises(binding.PcvError, match="same folds"):
        sa.compare(other)


# ---------------------------------------------------------------- HS and DSS

def _score_replay(w, n_iter, prec):
    from oracle import scores as sc
    run = sampler.run_all(w, n_iter=n_iter)
    sizes = [len(t) for t in sc.test_rows_of_folds(folds.roles_of(w))]
    want = sc.fold_scores(run.score_acc, w.K, w.L, run.acc.n_draws, sizes)
    s = binding.PCV.from_workload(w, precision=PREC[prec])
    s.step(n_iter)
    return want, s.scores()


@pytest.mark.parametrize("name,folds_,prec", [("c1", (0, 40), "fp64"), ("c3", (0, 30), "fp64")])
def test_hs_dss_replay_oracle_gaussian(dev, name, folds_, prec):
    """Gaussian: HS and DSS per fold from the device's sums equal the oracle's
    (one test row per fold for c1, five for the hv-block folds of c3)."""
    w = dataclasses.replace(W.fold_subset(W.make(name), *folds_), n_warmup=30, scores=3)
    want, got = _score_replay(w, 130, prec)
    _say(f"[scores] {name}: HS {got['hs']:.4f} (oracle {want['hs']:.4f}) DSS {got['dss']:.4f} (oracle {want['dss']:.4f})")
    np.testing.assert_allclose(got["hs_fold"], want["hs_fold"], rtol=1e-9)
    np.testing.assert_allclose(got["dss_fold"], want["dss_fold"], rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("base,v,L", [("c5", 10, 4), ("c4", 40, 8)])
def test_dss_replay_oracle_discrete(dev, base, v, L):
    """Bernoulli and Poisson predictive draws: a 2000-row design of the same
    family, 20 blocked folds of v test rows, on the plain fp64 path (which
    replays the oracle transition for transition)."""
    w0 = W.make(base)
    n, K = 2000, 20
    fi = np.where(np.arange(n) < K * v, np.arange(n) // v, -1).astype(np.int32)
    w = dataclasses.replace(w0, X=w0.X[:n], y=w0.y[:n], x_hi=None, x_lo=None, fold_index=fi, K=K, L=L,
                            init_pos=w0.init_pos[:K * L], n_warmup=10, batch_size=5, scores=2)
    want, got = _score_replay(w, 50, "fp64u")
    _say(f"[scores] {base} family {w.family}: DSS {got['dss']:.4f} (oracle {want['dss']:.4f})")
    np.testing.assert_allclose(got["dss_fold"], want["dss_fold"], rtol=1e-8, atol=1e-9)


def test_hs_refused_for_discrete_response(dev):
    w = dataclasses.replace(W.fold_subset(W.make("c5"), 0, 4), scores=1)
    with pytest.raises(binding.PcvError):
        binding.PCV.from_workload(w)


# ---------------------------------------------------------------- stored draws (Algorithm 1)

def test_stored_draws_and_posthoc_replay_oracle(dev):
    from oracle import posthoc
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 25), n_warmup=50, store_draws=300)
    run = sampler.run_all(w, n_iter=50 + 320, store_draws=True)      # more draws than the capacity
    s = binding.PCV.from_workload(w)
    s.step(370)
    d = s.get_draws(1000)
    assert d.shape == (w.C, 300)
    np.testing.assert_allclose(d, run.draws[:, :300], rtol=1e-10, atol=1e-12)
    got = s.posthoc()
    # rank statistics order near-ties differently when the values differ by
    # rounding, so the post-hoc formulas are compared on the device's draws
    want = posthoc.fold_rhats(d, w.K, w.L)
    tp = diagnostics.two_pass(d, w.K, w.L, w.batch_size)
    for k in ("rhat_fold", "split_rhat_fold", "rank_rhat_fold"):
        np.testing.assert_allclose(got[k], want[k], rtol=1e-9, err_msg=k)
    assert got["n_draws"] == 300
    assert got["elpd"] == pytest.approx(tp["elpd"], rel=1e-12)
    assert got["mcse"] == pytest.approx(tp["mcse"], rel=1e-9)
    assert got["ess"] == pytest.approx(tp["ess"], rel=1e-9)


def test_stored_draws_agree_with_online_on_matrix_cores(dev):
    w = dataclasses.replace(W.fold_subset(W.make("c5"), 0, 64), n_warmup=20, batch_size=10, store_draws=200)
    s = binding.PCV.from_workload(w, precision=W.PREC_BF16X3)
    s.step(20 + 200)
    on = s.diagnostics()
    ph = s.posthoc()
    np.testing.assert_allclose(ph["rhat_fold"], on["rhat_fold"], rtol=1e-9)
    assert ph["elpd"] == pytest.approx(on["elpd"], rel=1e-12)
    assert ph["split_rhat_max"] >= 1.0 - 1e-3 and np.isfinite(ph["rank_rhat_max"])
