"""The matrix-core path at design widths other than 64 and 128 (needs an
MI355X).  The bf16 kernels are built for widths 64 and 128; a design of
1 <= p <= 128 columns runs on the next one with zero columns past p, zero
coefficients there, and only the first p gradient rows written.  Checked
against the oracle like the full-width cases: the log density and gradient
of every chain in three launch shapes and several row-split counts, leapfrog
trajectories, and two nested models in one launch at an odd width (their
selection masks are read per coefficient)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import folds, hmc, model, philox
from paper_2310_07002_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _narrow(name, p, folds_):
    """The workload's fold subset with only its first p covariates (the
    stored bf16 design planes keep X = hi + lo exact)."""
    w = W.fold_subset(W.make(name), *folds_)
    return W.drop_covariates(w, np.arange(p, w.p)) if p < w.p else w


def _theta(w, seed):
    rng = np.random.default_rng(seed)
    return w.init_pos + 0.3 * np.sqrt(w.inv_mass)[None, :] * rng.standard_normal(w.init_pos.shape)


def _normwise(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _grad_bound(w, theta, g_o):
    """Normwise gradient error the split arithmetic allows per chain: with
    u = 2^-16 (the relative error of the hi + lo pairs of theta and of the
    residuals), |delta grad| <= u |X|'|r| + |X|'(|dr/deta| u |X||theta|).
    With many covariates the normwise error averages far below this; with
    one or a few, the gradient is a short sum whose cancellation the bound
    follows."""
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    eta = model.linear_predictor(w, theta)
    train = roles[foc].T == folds.ROLE_TRAIN
    r = train * model.dloglik_deta(w.family, w.y[:, None], eta, w.sigma)
    h = 1e-6
    dr = train * np.abs(model.dloglik_deta(w.family, w.y[:, None], eta + h, w.sigma)
                        - model.dloglik_deta(w.family, w.y[:, None], eta - h, w.sigma)) / (2 * h)
    u = 2.0 ** -16
    deta = u * (np.abs(w.X) @ np.abs(theta.T))
    return np.linalg.norm(u * (np.abs(w.X).T @ np.abs(r)) + np.abs(w.X).T @ (dr * deta), axis=0) \
        / np.linalg.norm(g_o, axis=1)


WIDTHS = [("c4", 1, (0, 16)), ("c4", 17, (0, 16)), ("c4", 40, (0, 16)), ("c5", 65, (100, 140)),
          ("c5", 100, (100, 140))]


@pytest.mark.parametrize("shape", [0, 1, 3])
@pytest.mark.parametrize("name,p,folds_", WIDTHS)
def test_any_width_matches_oracle(dev, shape, name, p, folds_):
    if shape == 3 and p > 64:
        pytest.skip("the 16-chain shape is for designs of up to 64 columns")
    w = _narrow(name, p, folds_)
    assert w.p == p and w.x_hi.shape[1] == p
    theta = _theta(w, seed=8)
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    lp_o = model.log_density(w, theta, roles, foc)
    g_o = model.grad_log_density(w, theta, roles, foc)
    bound = _grad_bound(w, theta, g_o)
    s = binding.PCV.from_workload(w, precision=W.PREC_BF16X3)
    for ns in (1, 7):
        s.set_launch_config(256 * shape + ns)
        lp, g = s.logdensity_grad(torch.tensor(theta, device=dev))
        rel_v = np.abs(lp.cpu().numpy() - lp_o) / np.abs(lp_o)
        rel_g = _normwise(g.cpu().numpy(), g_o)
        _say(f"[width] {name} p={p} shape {shape} splits {ns}: logp rel max {rel_v.max():.2e}, "
             f"grad normwise max {rel_g.max():.2e} (bound max {bound.max():.1e})")
        assert rel_v.max() < 1e-5
        if p >= 8:
            assert rel_g.max() < 5e-5
        else:
            # one coefficient: its gradient is a single cancelling sum, held
            # to the bound (the comparison with the zero-padded run below is
            # exact)
            assert np.all(rel_g < 5e-5 + bound)
    s.close()


@pytest.mark.parametrize("shape", [0, 1, 3])
@pytest.mark.parametrize("name,p,folds_", WIDTHS)
def test_any_width_equals_the_zero_padded_design(dev, shape, name, p, folds_):
    """The narrow design against the same design padded to the kernel width
    with zero columns (coefficients past p set to zero), at the same launch
    shape: the first p gradient entries agree bit for bit, the padded ones
    are zero, and the log densities differ by the padded coefficients'
    prior terms at zero."""
    if shape == 3 and p > 64:
        pytest.skip("the 16-chain shape is for designs of up to 64 columns")
    full = W.fold_subset(W.make(name), *folds_)
    P = 64 if p <= 64 else 128
    w = _narrow(name, p, folds_)
    wp = W.drop_covariates(W.drop_covariates(full, np.arange(P, full.p)) if P < full.p else full,
                           np.arange(p, P), zero=True)
    assert wp.p == P
    theta = _theta(w, seed=9)
    theta_p = np.zeros((w.C, P))
    theta_p[:, :p] = theta
    s = binding.PCV.from_workload(w, precision=W.PREC_BF16X3)
    sp = binding.PCV.from_workload(wp, precision=W.PREC_BF16X3)
    for ns in (1, 7):
        s.set_launch_config(256 * shape + ns)
        sp.set_launch_config(256 * shape + ns)
        lp, g = (a.cpu().numpy() for a in s.logdensity_grad(torch.tensor(theta, device=dev)))
        lpp, gp = (a.cpu().numpy() for a in sp.logdensity_grad(torch.tensor(theta_p, device=dev)))
        np.testing.assert_array_equal(gp[:, :p], g)
        np.testing.assert_array_equal(gp[:, p:], 0.0)
        extra = float(np.sum(-0.5 * np.log(2 * np.pi) - np.log(wp.prior_scale[p:])))
        np.testing.assert_allclose(lpp - extra, lp, rtol=1e-12)
    _say(f"[width padded] {name} p={p} shape {shape}: equal to the zero-padded width-{P} run")
    s.close()
    sp.close()


@pytest.mark.parametrize("name,p,folds_", [("c4", 40, (0, 16)), ("c5", 100, (100, 140))])
def test_any_width_leapfrog_matches_oracle(dev, name, p, folds_):
    """Four leapfrog steps (gradient-only launches in between) at the
    multi-step BF16X3 bound of the full-width cases."""
    w = _narrow(name, p, folds_)
    roles = folds.roles_of(w)
    foc = np.arange(w.C) // w.L
    q0 = _theta(w, seed=5)
    p0 = philox.momentum_normals(w.seed, w.chain_offset + np.arange(w.C), 0, w.d) / np.sqrt(w.inv_mass)
    g0 = model.grad_log_density(w, q0, roles, foc)
    q1, p1, _, lp1 = hmc.leapfrog(w, q0, p0, g0, 4, w.step_size, roles, foc)
    s = binding.PCV.from_workload(w, precision=W.PREC_BF16X3)
    qg, pg, lpg, _ = s.leapfrog(torch.tensor(q0, device=dev), torch.tensor(p0, device=dev), 4)
    eq = _normwise(qg.cpu().numpy(), q1)
    ep = _normwise(pg.cpu().numpy(), p1)
    ev = np.abs(lpg.cpu().numpy() - lp1) / np.abs(lp1)
    _say(f"[width leapfrog] {name} p={p}: q {eq.max():.2e}  p {ep.max():.2e}  logp {ev.max():.2e}")
    assert eq.max() < 2e-5 and ep.max() < 2e-5 and ev.max() < 2e-5
    s.close()


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_two_models_at_an_odd_width(dev, shape):
    """p = 17: model B drops covariates 3, 9 and 16 (the last one); both
    models in one bf16x3 launch, in every launch shape (the kernels read the
    selection masks when they split theta), match the oracle's separate
    evaluations."""
    w = _narrow("c4", 17, (0, 16))
    m = np.ones((2, w.p), dtype=np.uint8)
    m[1, [3, 9, 16]] = 0
    w2 = W.with_models(w, m)
    theta = _theta(w2, seed=4)
    s = binding.PCV.from_workload(w2, precision=W.PREC_BF16X3)
    s.set_launch_config(256 * shape + 7)
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
        _say(f"[width models] shape {shape} model {mi}: logp rel max {rel_v.max():.2e}  "
             f"grad normwise max {rel_g.max():.2e}")
        assert rel_v.max() < 1e-5
        assert rel_g.max() < 5e-5
    s.close()
