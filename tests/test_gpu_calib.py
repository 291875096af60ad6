"""The bf16 MFMA calibration kernel behind bench.py's roofline.mfma_ceiling
(needs an MI355X): both rates are positive, below the published dense peak,
and random operands never sustain more than constant ones by more than the
run-to-run spread."""
import pytest

torch = pytest.importorskip("torch")

from paper_2310_07002_amd import binding

pytestmark = pytest.mark.gpu

BF16_DENSE_PEAK_TFLOPS = 2500.0


def test_mfma_calibration_rates():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    rnd = binding.pcv_calib_mfma(1, 10)
    cst = binding.pcv_calib_mfma(0, 10)
    print(f"[calib] bf16 32x32x16 MFMA: random operands {rnd:.0f} TFLOP/s, constant {cst:.0f}", flush=True)
    for r in (rnd, cst):
        assert 0.0 < r < 1.05 * BF16_DENSE_PEAK_TFLOPS
    assert rnd < 1.05 * cst
