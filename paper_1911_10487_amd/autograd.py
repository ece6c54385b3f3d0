"""PyTorch autograd wrapper and power iteration over the C-ABI derivatives.

``invert(W, u0, delta, plan)`` is a torch.autograd.Function: the forward is
fl_invert and the backward is the hand-written adjoint fl_invert_vjp (the
gradient convention is PyTorch's: dL/dRe + i dL/dIm for complex tensors).
``power_iteration`` estimates the largest singular value of J = d xi / d W
(as a real-linear map) by repeated J^T J products, each one fl_invert_jvp
followed by fl_invert_vjp.
"""
from __future__ import annotations

import torch


class FlInvert(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W, u0, plan, delta):
        ctx.plan = plan
        ctx.delta = float(delta)
        ctx.save_for_backward(W, u0)
        return plan.invert(W, u0, delta)

    @staticmethod
    def backward(ctx, grad_xi):
        W, u0 = ctx.saved_tensors
        gW, gu = ctx.plan.vjp(W, u0, ctx.delta, grad_xi, want_u0=ctx.needs_input_grad[1])
        gW = gW.to(W.dtype) if ctx.needs_input_grad[0] else None
        gu = gu.to(u0.dtype) if gu is not None else None
        return gW, gu, None, None


def invert(W, u0, delta, plan):
    return FlInvert.apply(W, u0, plan, delta)


def power_iteration(plan, W, u0, delta, iters=20, seed=0):
    """Returns (sigma estimates per iteration, unit right singular direction).

    Each iteration: y = J x (tangent), z = J^T y (adjoint), sigma^2 ~ <x, z>,
    x <- z / ||z||; the Rayleigh quotients increase monotonically to
    ||J||_2^2."""
    g = torch.Generator(device=W.device)
    g.manual_seed(seed)
    x = torch.randn(W.shape, dtype=W.dtype, device=W.device, generator=g)
    x = x / torch.linalg.vector_norm(x)
    est = []
    for _ in range(iters):
        y = plan.jvp(W, u0, delta, x)
        z, _ = plan.vjp(W, u0, delta, y)
        lam = torch.real(torch.vdot(x.reshape(-1).to(torch.complex128), z.reshape(-1))).item()
        est.append(max(lam, 0.0) ** 0.5)
        x = (z / torch.linalg.vector_norm(z)).to(W.dtype)
    return est, x
