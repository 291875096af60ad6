"""The paper's Example 1 on the device against the oracle (needs an MI355X):
LOGO-CV of a grouped Gaussian regression with hierarchical intercepts
alpha_j = mu + sigma_a z_j and unknown noise scale sigma_y, model A (all four
group-level covariates) and model B (one dropped) in one launch (Section 2,
Example 1; Section 2.3, eqs sel-cv and norm-approx; Appendix B, parallel
model evaluation).  Model m of the launch is, by construction, the workload
with its masked covariate's column zeroed and its own global chain ids; the
oracle evaluates and runs exactly that."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import diagnostics, folds, hmc, model, sampler
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


def _theta(w, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return w.init_pos + scale * np.sqrt(w.inv_mass)[None, :] * rng.standard_normal(w.init_pos.shape)


def _split_path_workload():
    """50 groups of 45 rows (n = 2250), the first 8 folds: few chains and
    many rows, so the library takes its row-split path."""
    return W.fold_subset(W.make_ex1(Nj=45), 0, 8)


CASES = [  # label, builder, precision, tol value, tol gradient
    ("ex1 fp64 fused", lambda: W.make_ex1(), W.PREC_FP64, 1e-12, 1e-12),
    ("ex1 fp32 fused", lambda: W.make_ex1(), W.PREC_FP32, 1e-5, 1e-5),
    ("ex1 A+B fp64 fused", lambda: W.make_ex1_ab(), W.PREC_FP64, 1e-12, 1e-12),
    ("ex1 A+B fp32 fused", lambda: W.make_ex1_ab(), W.PREC_FP32, 1e-5, 1e-5),
    ("ex1 Nj=45 fp64 row-split", _split_path_workload, W.PREC_FP64, 1e-12, 1e-12),
    ("ex1 Nj=45 fp32 row-split", _split_path_workload, W.PREC_FP32, 1e-5, 1e-5),
    ("ex1 Nj=45 A+B fp64 row-split",
     lambda: W.with_models(_split_path_workload(), np.array([[1, 1, 1, 1], [0, 1, 1, 1]], dtype=np.uint8)),
     W.PREC_FP64, 1e-12, 1e-12),
]


def _oracle_models(w):
    """(model workload, chain slice) of every model of w."""
    if w.n_models == 1:
        return [(w, slice(0, w.C))]
    KL = w.K * w.L
    return [(W.model_of(w, m), slice(m * KL, (m + 1) * KL)) for m in range(w.n_models)]


@pytest.mark.parametrize("label,make_w,prec,tol_v,tol_g", CASES)
def test_ex1_logdensity_grad_matches_oracle(dev, label, make_w, prec, tol_v, tol_g):
    w = make_w()
    theta = _theta(w, seed=3)
    s = binding.PCV.from_workload(w, precision=prec)
    lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    for wm, sl in _oracle_models(w):
        roles = folds.roles_of(wm)
        foc = np.arange(wm.C) // wm.L
        lp_o = model.log_density(wm, theta[sl], roles, foc)
        g_o = model.grad_log_density(wm, theta[sl], roles, foc)
        rel_v = np.abs(lp[sl] - lp_o) / np.abs(lp_o)
        rel_g = _normwise(g[sl], g_o)
        _say(f"[{label}] C={w.C} n={w.n} d={w.d}: logp rel max {rel_v.max():.2e}  grad normwise max {rel_g.max():.2e}")
        assert rel_v.max() < tol_v
        assert rel_g.max() < tol_g
    s.close()


@pytest.mark.parametrize("make_w,n_steps", [(lambda: W.make_ex1(), 8), (_split_path_workload, 8)])
def test_ex1_leapfrog_matches_oracle(dev, make_w, n_steps):
    """n_steps leapfrog steps from the same (q, p) in fp64, fused and
    row-split paths (the latter: per-step partials, their reduction and the
    log sigma_a value the partials were taken at)."""
    w = make_w()
    q = _theta(w, seed=5)
    rng = np.random.default_rng(6)
    p = rng.standard_normal(q.shape) / np.sqrt(w.inv_mass)[None, :]
    s = binding.PCV.from_workload(w, precision=W.PREC_FP64)
    qd, pd, lpd, gd = s.leapfrog(torch.tensor(q, device=dev), torch.tensor(p, device=dev), n_steps)
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    g0 = model.grad_log_density(w, q, roles, foc)
    qo, po, go, lpo = hmc.leapfrog(w, q, p, g0, n_steps, w.step_size, roles, foc)
    eq = _normwise(qd.cpu().numpy(), qo).max()
    ep = _normwise(pd.cpu().numpy(), po).max()
    ev = (np.abs(lpd.cpu().numpy() - lpo) / np.abs(lpo)).max()
    _say(f"[ex1 leapfrog] n={w.n} C={w.C}: q {eq:.2e} p {ep:.2e} logp {ev:.2e}")
    assert eq < 1e-12 and ep < 1e-11 and ev < 1e-12
    s.close()


def test_ex1_two_models_replay_the_oracle(dev):
    """Both models of Example 1 in one fp64 launch, 150 transitions: every
    chain replays the oracle's run of its own model accept for accept; the
    per-model elpd and pcv_compare_models equal the oracle's."""
    w2 = dataclasses.replace(W.make_ex1_ab(), n_warmup=50, n_samples=100, batch_size=20)
    n_iter = w2.n_warmup + w2.n_samples
    s = binding.PCV.from_workload(w2)
    s.step(n_iter)
    th, _, sv = s.get_state()
    acc = s.get_accumulators(w2.n_blocks)
    est = []
    for mi, (wm, sl) in enumerate(_oracle_models(w2)):
        run = sampler.run_all(wm, n_iter=n_iter)
        np.testing.assert_allclose(th[sl], run.state.q, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(sv[sl], run.state.s, rtol=1e-9, atol=1e-10)
        np.testing.assert_array_equal(acc["n_accept"][sl], run.acc.n_accept)
        o = diagnostics.from_accumulators(run.acc, wm.K, wm.L, wm.batch_size)
        e = s.elpd_model(mi)
        _say(f"[ex1 replay] model {'AB'[mi]}: elpd {e['elpd']:.4f} +- {e['mcse']:.4f} (oracle {o['elpd']:.4f}), "
             f"accept {o['accept_rate']:.3f}")
        assert e["elpd"] == pytest.approx(o["elpd"], rel=1e-10)
        np.testing.assert_allclose(e["elpd_fold"], o["elpd_fold"], rtol=1e-10)
        np.testing.assert_allclose(e["mcse_fold"], o["mcse_fold"], rtol=1e-7)
        est.append(o)
    want = diagnostics.compare(est[0]["elpd_fold"], est[0]["mcse_fold"], est[1]["elpd_fold"], est[1]["mcse_fold"])
    got = s.compare_models(0, 1)
    _say(f"[ex1 replay] delta {got['delta']:.4f} (oracle {want['delta']:.4f}) Pr(A>B) {got['prob_a_better']:.4f}")
    assert got["delta"] == pytest.approx(want["delta"], rel=1e-9)
    assert got["sigma2"] == pytest.approx(want["sigma2"], rel=1e-8)
    assert got["prob_a_better"] == pytest.approx(want["prob_a_better"], abs=1e-9)
    np.testing.assert_allclose(got["delta_fold"], want["delta_fold"], rtol=1e-9, atol=1e-12)
    s.close()


def test_ex1_full_comparison_favours_the_true_model(dev):
    """The full Example 1 (50 groups, 4 chains per fold, both models in one
    fp64 launch, 250 + 1000 transitions): converged (R-hat_max below 1.05 for
    each model), Delta's Monte Carlo error far below its epistemic spread,
    and the comparison favours model A, which generated the data (the
    paper's Figure 1 reports Pr(M_A better) near one)."""
    w2 = W.make_ex1_ab()
    s = binding.PCV.from_workload(w2)
    s.step(w2.n_iter)
    d = s.diagnostics()
    rk = d["rhat_fold"]
    got = s.compare_models(0, 1)
    ea, eb = s.elpd_model(0), s.elpd_model(1)
    _say(f"[ex1 full] elpd A {ea['elpd']:.3f} +- {ea['mcse']:.3f}, B {eb['elpd']:.3f} +- {eb['mcse']:.3f}; "
         f"delta {got['delta']:.3f} mcse {got['mcse']:.3f} sd {np.sqrt(w2.K * got['sigma2']):.3f} "
         f"Pr(A>B) {got['prob_a_better']:.4f}; rhat_max A {rk[:w2.K].max():.4f} B {rk[w2.K:].max():.4f}; "
         f"accept {d['accept_rate']:.3f} divergent {d['n_divergent']}")
    assert rk.max() < 1.05
    assert got["mcse"] < 0.25 * np.sqrt(w2.K * got["sigma2"])
    assert got["delta"] > 0 and got["prob_a_better"] > 0.9
    s.close()


def test_ex1_refusals(dev):
    w = W.make_ex1()
    for prec in (W.PREC_BF16X3, W.PREC_FP64_UNFUSED):
        with pytest.raises(binding.PcvError) as e:
            binding.PCV.from_workload(w, precision=prec)
        assert e.value.status == 5
    with pytest.raises(binding.PcvError) as e:
        binding.PCV.from_workload(dataclasses.replace(w, scores=2))
    assert e.value.status == 5
