"""Differentiable unrolled mean field: T proximal steps behind torch.autograd.

The forward runs the steps in the HIP library (one step per launch, so the
backward's recomputation reproduces it bitwise) and keeps log q at every
``ckpt_every``-th iteration; the backward calls the library's hand-written
adjoint, which recomputes the iterates between checkpoints.  Gradients flow
to the unaries and to every entry of Theta as it appears in m = u + Theta S.
"""
from __future__ import annotations

import torch

from . import mf


class _UnrolledMeanField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, unary, theta, graph, height, width, alpha, iters, ckpt_every, precision):
        u = unary.detach().contiguous()
        th = theta.detach().contiguous()
        solver = mf.MeanField(u, graph, height=height, width=width, theta=th, alpha=alpha,
                              precision=precision, steps_per_launch=1)
        n_ckpt = max(1, (iters + ckpt_every - 1) // ckpt_every)
        B, L, N = solver.shape
        ckpts = torch.empty((n_ckpt, B, L, N), dtype=torch.float32, device=u.device)
        t = 0
        for k in range(n_ckpt):
            ckpts[k].copy_(solver.current_state())
            n = min(ckpt_every, iters - t)
            solver.step(n)
            t += n
        out = solver.current_state().clone()
        ctx.solver = solver
        ctx.iters = iters
        ctx.ckpt_every = ckpt_every
        ctx.theta_shape = theta.shape
        ctx.save_for_backward(ckpts)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (ckpts,) = ctx.saved_tensors
        g = grad_out.contiguous().to(torch.float32)
        gu, gt = ctx.solver.backward(ckpts, ctx.iters, ctx.ckpt_every, g)
        return gu, gt.reshape(ctx.theta_shape), None, None, None, None, None, None, None


def unrolled_mean_field(unary: torch.Tensor, theta: torch.Tensor, *, height: int, width: int,
                        connectivity: int = 8, alpha: float = 0.5, iters: int = 10, ckpt_every: int = 5,
                        precision: str = "f32") -> torch.Tensor:
    """log q after ``iters`` parallel proximal steps from q0 = softmax(-u).

    unary: [B, L, N] energies; theta: [L, L].  Differentiable in both.
    """
    if precision != "f32":
        # the library's adjoint differentiates the step with FP32 messages
        raise mf.MFError(mf.MF_EUNSUPPORTED, "the adjoint runs with FP32 messages only")
    graph = "grid4" if connectivity == 4 else "grid8"
    return _UnrolledMeanField.apply(unary, theta, graph, height, width, alpha, iters, ckpt_every, precision)
