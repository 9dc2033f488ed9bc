"""Differentiable NFFT: ``f = nfft(x, fhat, plan)`` with gradients for the coefficients
and the node positions.

For a real loss L and y = A(x) fhat, PyTorch passes the upstream gradient
v = dL/dRe(y) + i dL/dIm(y).  Then

* dL/dfhat (same convention) = A^H v, which is the adjoint NFFT (Algorithm 2.2) of v;
* dL/dx_{j,t} = Re(conj(v_j) d y_j / d x_{j,t}), where the derivative is taken through
  the window of Algorithm 2.1 step 3 (nfft_grad_x), using the grid of the forward pass.

Both run in the HIP library; this module only wires them into autograd.
"""
import torch

from ._lib import NFFT_KEEP_GRID
from .nfft import Plan


class _NfftFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, fhat, plan):
        plan.set_nodes(x.detach())
        f = plan.trafo(fhat.detach())
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.node_generation = plan.node_generation
        ctx.save_for_backward(x, fhat)
        return f

    @staticmethod
    def backward(ctx, v):
        plan = ctx.plan
        x, fhat = ctx.saved_tensors
        v = v.contiguous().to(plan.dtype)
        gx = gfhat = None
        # The plan may have been used with other nodes or coefficients since this forward
        # ran: both gradients need this call's nodes, the node gradient also its grid.
        stale_nodes = plan.node_generation != ctx.node_generation or plan.nodes_version != x._version
        stale_grid = stale_nodes or plan.generation != ctx.generation
        if stale_nodes:
            plan.set_nodes(x.detach())
        if ctx.needs_input_grad[0]:
            if stale_grid:
                plan.trafo(fhat.detach())
            gx = plan.grad_x(v).to(x.dtype)
        if ctx.needs_input_grad[1]:
            gfhat = plan.adjoint(v)
        return gx, gfhat, None


def nfft(x, fhat, plan):
    """NFFT f_j ~ sum_k fhat_k exp(-2 pi i k.x_j) of the (M, d) float64 nodes x and the
    coefficients fhat (shape N, the plan's complex dtype), differentiable in both.  The
    plan must have been created with NFFT_KEEP_GRID (see ``differentiable_plan``)."""
    if not (plan.flags & NFFT_KEEP_GRID):
        raise ValueError("the plan needs NFFT_KEEP_GRID for gradients with respect to x")
    return _NfftFunction.apply(x, fhat, plan)


def differentiable_plan(N, M, n=None, m=8, dtype=torch.complex64, device="cuda", window="kaiser-bessel"):
    """A plan set up for ``nfft`` (keeps the forward grid for the node gradient)."""
    return Plan(N, M, n=n, m=m, dtype=dtype, flags=NFFT_KEEP_GRID, device=device, window=window)
