"""torch.autograd.Function for the bandlimited NFFT-like transform.

f = A(x) fhat with A the factorisation Psi F D_psihat of (4.11).  The backward pass is
hand-written in the library: grad_fhat = A^H grad_f (bl_adjoint: spreading, forward
FFT, truncation to I_M, deconvolution) and grad_x[j, t] = Re(conj(grad_f_j) d f_j /
d x_jt) (bl_grad_x, psi' short sums on the samples theta of the forward pass).  PyTorch's
complex convention passes grad_f = dL/dRe f + i dL/dIm f, for which both formulas are the
exact gradients.
"""
from __future__ import annotations

import torch

from .plan import Plan


class BandlimitedNFFT(torch.autograd.Function):
    """f = BandlimitedNFFT.apply(fhat, x, plan)."""

    @staticmethod
    def forward(ctx, fhat: torch.Tensor, x: torch.Tensor, plan: Plan):
        plan.bind_nodes(x.detach().contiguous())
        f = plan.forward(fhat.detach().contiguous())
        ctx.plan = plan
        ctx.state = plan.state()
        ctx.save_for_backward(fhat, x)
        return f

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        plan: Plan = ctx.plan
        fhat, x = ctx.saved_tensors
        g = grad_f.contiguous().to(plan.complex_dtype)
        if plan.state() != ctx.state:
            # a later call rebound the nodes or replaced the samples theta: restore them
            plan.set_nodes(x.detach().contiguous())
            plan.forward(fhat.detach().contiguous())
        grad_fhat = grad_x = None
        if ctx.needs_input_grad[1]:
            grad_x = plan.grad_x(g)
        if ctx.needs_input_grad[0]:
            grad_fhat = plan.adjoint(g)
        return grad_fhat, grad_x, None


def bandlimited_nfft(fhat: torch.Tensor, x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable f_j ~ f(x_j) from fhat(k), k in I_M (Algorithm 4.2)."""
    return BandlimitedNFFT.apply(fhat, x, plan)
