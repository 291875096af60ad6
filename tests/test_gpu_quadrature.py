"""The device's elpd on non-conjugate models against brute force (needs an
MI355X).  The two-coefficient logistic and Poisson GLMs of the oracle's
quadrature pin, run whole on the device in fp64 (fused VALU path), fp32 and
bf16x3 (matrix cores, the design padded to width 64): every fold's elpd lies
within 4 Monte Carlo standard errors of the exact K-fold predictive density."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import model
from paper_2310_07002_amd import binding, workloads as W
from test_oracle_quadrature import _exact_fold_elpd, _workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("family,seed", [(model.LOGISTIC, 0), (model.POISSON, 1)])
def test_device_elpd_matches_quadrature(dev, family, seed, prec):
    w = _workload(family, seed)
    exact = np.array([_exact_fold_elpd(w, k)[0] for k in range(w.K)])
    code = {"fp64": W.PREC_FP64, "fp32": W.PREC_FP32, "bf16x3": W.PREC_BF16X3}[prec]
    s = binding.PCV.from_workload(w, precision=code)
    s.step(w.n_iter)
    d = s.diagnostics()
    e = s.elpd()
    z = np.abs(e["elpd_fold"] - exact) / e["mcse_fold"]
    print(f"[quadrature] family {family} {prec}: elpd {d['elpd']:.4f} exact {exact.sum():.4f} "
          f"mcse {d['mcse']:.4f} fold z max {z.max():.2f} rhat_max {d['rhat_max']:.4f}", flush=True)
    assert d["n_draws"] == w.n_samples
    assert np.all(z < 4)
    assert abs(d["elpd"] - exact.sum()) < 4 * d["mcse"]
    assert d["rhat_max"] < 1.05
    s.close()
