"""torch.autograd.Function around the library's hand-written adjoint.

forward(theta[C, d]) -> log pi[C] for every fold x chain state (the masked log
density of Appendix B); backward(grad_out[C]) -> grad_out[:, None] * grad log pi,
with the gradient produced by the same kernel launch as the value (the adjoint
contraction X' R), not by a tape.
"""
from __future__ import annotations

import torch


class PCVLogDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, sampler) -> torch.Tensor:
        theta = theta.detach().contiguous()
        logp, grad = sampler.logdensity_grad(theta, want_grad=True)
        ctx.save_for_backward(grad)
        return logp

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad_out[:, None] * grad, None


def log_density(theta: torch.Tensor, sampler) -> torch.Tensor:
    return PCVLogDensity.apply(theta, sampler)
