"""MI355X (gfx950) library for parallel brute-force Bayesian cross-validation.

The sampler itself lives in the HIP library libpcv.so (C ABI in include/pcv.h);
`binding` exposes it to Python, `autograd` wraps its hand-written adjoint as a
torch.autograd.Function, and `workloads` generates the seeded synthetic
inputs.
"""
from . import workloads  # noqa: F401
