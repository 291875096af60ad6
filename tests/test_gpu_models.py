"""Several nested models in one launch (Appendix B, parallel model
evaluation) against the oracle (needs an MI355X).  Model m of a run is, by
construction, the workload with its masked covariates' columns zeroed and
its own global chain ids; the oracle evaluates and runs exactly that."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import diagnostics, folds, model, sampler
from paper_2310_07002_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _normwise(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _masks(p, drop):
    m = np.ones((2, p), dtype=np.uint8)
    m[1, drop] = 0
    return m


CASES = [  # workload, precision, folds, dropped covariates of model B, tolerances (value, gradient)
    ("c1", W.PREC_FP64, None, [1, 4], 1e-12, 1e-12),          # fused VALU path
    ("c3", W.PREC_FP64, (0, 40), [2, 3], 1e-12, 1e-12),       # row-split VALU path
    ("c4", W.PREC_BF16X3, (0, 16), list(range(8)), 1e-5, 5e-5),   # matrix-core path
]


@pytest.mark.parametrize("name,prec,folds_,drop,tol_v,tol_g", CASES)
def test_masked_models_match_zeroed_columns(dev, name, prec, folds_, drop, tol_v, tol_g):
    w = W.make(name)
    if folds_:
        w = W.fold_subset(w, *folds_)
    w2 = W.with_models(w, _masks(w.p, drop))
    _say(f"[models] {name} C={w2.C}")
    rng = np.random.default_rng(4)
    theta = w2.init_pos + 0.3 * np.sqrt(w2.inv_mass)[None, :] * rng.standard_normal(w2.init_pos.shape)
    s = binding.PCV.from_workload(w2, precision=prec)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    KL = w.K * w.L
    for mi in range(2):
        wm = W.model_of(w2, mi)
        roles = folds.roles_of(wm)
        foc = np.arange(wm.C) // wm.L
        th = theta[mi * KL:(mi + 1) * KL]
        lp_o = model.log_density(wm, th, roles, foc)
        g_o = model.grad_log_density(wm, th, roles, foc)
        rel_v = np.abs(lp[mi * KL:(mi + 1) * KL] - lp_o) / np.abs(lp_o)
        rel_g = _normwise(g[mi * KL:(mi + 1) * KL], g_o)
        _say(f"    model {mi}: logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
        assert rel_v.max() < tol_v
        assert rel_g.max() < tol_g
    s.close()


def test_two_models_in_one_launch_replay_the_oracle(dev):
    """LOO of the conjugate Gaussian, model B without its two strongest
    covariates, both models in one fp64 launch: every chain replays the
    oracle's run of its own model, and the per-model elpd and the comparison
    equal the oracle's."""
    w = dataclasses.replace(W.make("c1"), n_warmup=40, n_samples=200, batch_size=20, n_blocks=5)
    drop = list(np.argsort(-np.abs(w.truth))[:2])
    w2 = W.with_models(w, _masks(w.p, drop))
    n_iter = w.n_warmup + w.n_samples
    s = binding.PCV.from_workload(w2)
    s.step(n_iter)
    th, _, sv = s.get_state()
    acc = s.get_accumulators(w.n_blocks)
    KL = w.K * w.L
    fold_est = []
    for mi in range(2):
        run = sampler.run_all(W.model_of(w2, mi), n_iter=n_iter)
        sl = slice(mi * KL, (mi + 1) * KL)
        np.testing.assert_allclose(th[sl], run.state.q, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(sv[sl], run.state.s, rtol=1e-9, atol=1e-10)
        np.testing.assert_array_equal(acc["n_accept"][sl], run.acc.n_accept)
        o = diagnostics.from_accumulators(run.acc, w.K, w.L, w.batch_size)
        e = s.elpd_model(mi)
        _say(f"[models] model {mi}: elpd {e['elpd']:.4f} +- {e['mcse']:.4f} (oracle {o['elpd']:.4f})")
        assert e["elpd"] == pytest.approx(o["elpd"], rel=1e-10)
        np.testing.assert_allclose(e["elpd_fold"], o["elpd_fold"], rtol=1e-10)
        np.testing.assert_allclose(e["mcse_fold"], o["mcse_fold"], rtol=1e-7)
        fold_est.append(o)
    want = diagnostics.compare(fold_est[0]["elpd_fold"], fold_est[0]["mcse_fold"],
                               fold_est[1]["elpd_fold"], fold_est[1]["mcse_fold"])
    got = s.compare_models(0, 1)
    _say(f"[models] delta {got['delta']:.4f} (oracle {want['delta']:.4f}) Pr(A>B) {got['prob_a_better']:.4f}")
    assert got["delta"] == pytest.approx(want["delta"], rel=1e-9)
    assert got["sigma2"] == pytest.approx(want["sigma2"], rel=1e-8)
    assert got["prob_a_better"] == pytest.approx(want["prob_a_better"], abs=1e-9)
    np.testing.assert_allclose(got["delta_fold"], want["delta_fold"], rtol=1e-9, atol=1e-12)
    # the whole-run diagnostics see 2K posteriors
    d = s.diagnostics()
    assert d["rhat_fold"].shape == (2 * w.K,) and np.isfinite(d["rhat_max"])
    s.close()


def test_masked_models_refused_where_unsupported(dev):
    w = W.fold_subset(W.make("c4"), 0, 4)
    w2 = W.with_models(w, _masks(w.p, [0]))
    with pytest.raises(binding.PcvError):
        binding.PCV.from_workload(w2, precision=W.PREC_FP64_UNFUSED)
    bad = dataclasses.replace(w2, model_mask=np.full_like(w2.model_mask, 2))
    with pytest.raises(binding.PcvError):
        binding.PCV.from_workload(bad, precision=W.PREC_BF16X3)


def test_two_model_run_resumes_from_a_checkpoint(dev, tmp_path):
    """A two-model launch saved after 30 transitions and resumed in a fresh
    context continues bit for bit; a context with a different mask refuses
    the checkpoint."""
    w = dataclasses.replace(W.fold_subset(W.make("c1"), 0, 30), n_warmup=10, batch_size=10)
    w2 = W.with_models(w, _masks(w.p, [0, 2]))
    a = binding.PCV.from_workload(w2)
    a.step(30)
    path = str(tmp_path / "two_models.ckpt")
    a.save(path)
    a.step(25)
    b = binding.PCV.from_workload(w2)
    b.load(path)
    b.step(25)
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)
    assert a.elpd_model(1)["elpd"] == b.elpd_model(1)["elpd"]
    other = binding.PCV.from_workload(W.with_models(w, _masks(w.p, [1])))
    with pytest.raises(binding.PcvError):
        other.load(path)


def test_two_models_on_matrix_cores_track_separate_runs(dev):
    """Two nested Poisson GLMs (p=64) in one bf16x3 launch stepping through
    captured transition graphs, against each model run alone (its columns
    zeroed, its global chain ids): the row-split count may differ between
    the runs, so positions agree to the bf16x3 tolerance wherever the
    accept decisions agree, which is nearly everywhere; so do the
    accepted states' test-row log predictives (each model's selection mask
    applied when they are formed)."""
    w = dataclasses.replace(W.fold_subset(W.make("c4"), 0, 16), n_warmup=3)
    w2 = W.with_models(w, _masks(w.p, list(range(0, 64, 5))))
    s = binding.PCV.from_workload(w2, precision=W.PREC_BF16X3)
    s.step(6)
    th, _, sv = s.get_state()
    acc = s.get_accumulators(w.n_blocks)["n_accept"]
    KL = w.K * w.L
    for mi in range(2):
        one = binding.PCV.from_workload(W.model_of(w2, mi), precision=W.PREC_BF16X3)
        one.step(6)
        t1, _, s1 = one.get_state()
        a1 = one.get_accumulators(w.n_blocks)["n_accept"]
        sl = slice(mi * KL, (mi + 1) * KL)
        same = acc[sl] == a1
        err = _normwise(th[sl], t1)
        serr = np.abs(sv[sl] - s1) / np.abs(s1)
        _say(f"[models] c4 model {mi}: same decisions {same.mean():.3f}, max err (same) {err[same].max():.2e}, "
             f"log predictive {serr[same].max():.2e}")
        assert same.mean() > 0.95
        assert err[same].max() < 1e-4
        assert serr[same].max() < 1e-4
        one.close()
    s.close()
