"""Differentiable wrappers of the line solves and the ADI time loop.

The backward passes are the library's hand-written adjoint kernels:
  - a line solve x = A^{-1} d has dL/dd = A^{-T} dL/dx (a tridiagonal solve with
    the transposed rows) and dL/dA = -lambda x^T restricted to the three
    diagonals;
  - one ADI step (Alg. 3 of arxiv 2201.03950 with per-point s) is reversed from
    its input checkpoint: the step is recomputed, then the transposed solves run
    z -> y -> x and the stencil's adjoint closes the step.
ADIFn keeps one checkpoint per step (the field entering it) and nothing else.
"""

from __future__ import annotations

import torch

from . import _binding as B


class TridSolveFn(torch.autograd.Function):
    """x = A^{-1} d along ``axis`` with per-point coefficient arrays a, b, c."""

    @staticmethod
    def forward(ctx, a, b, c, d, axis):
        a, b, c = a.contiguous(), b.contiguous(), c.contiguous()
        x = d.contiguous().clone()
        B.gtsv(a, b, c, x, axis)
        ctx.save_for_backward(a, b, c, x)
        ctx.axis = axis
        return x

    @staticmethod
    def backward(ctx, gx):
        a, b, c, x = ctx.saved_tensors
        g = gx.contiguous().clone()
        ga, gb, gc = torch.empty_like(g), torch.empty_like(g), torch.empty_like(g)
        B.gtsv_adjoint(a, b, c, x, g, ctx.axis, ga, gb, gc)
        return ga, gb, gc, g, None


class TridSolveSFn(torch.autograd.Function):
    """x = A(s)^{-1} d along ``axis`` with rows (-s, 1 + 2 s, -s)."""

    @staticmethod
    def forward(ctx, s, d, axis):
        s = s.contiguous()
        x = d.contiguous().clone()
        B.gtsv_s(s, x, axis)
        ctx.save_for_backward(s, x)
        ctx.axis = axis
        return x

    @staticmethod
    def backward(ctx, gx):
        s, x = ctx.saved_tensors
        g = gx.contiguous().clone()
        gs = torch.zeros_like(s)
        B.gtsv_s_adjoint(s, x, g, gs, ctx.axis)
        return gs, g, None


class ADIFn(torch.autograd.Function):
    """``nsteps`` ADI steps with per-point s, differentiable in u0 and s.

    Memory: one checkpoint (the field entering the step) per step.
    """

    @staticmethod
    def forward(ctx, u0, s, nsteps):
        s = s.contiguous()
        u = u0.detach().contiguous().clone()
        ckpts = []
        for _ in range(int(nsteps)):
            ckpts.append(u.clone())
            B.adi_step(u, s=s, nsteps=1)
        ctx.save_for_backward(s, *ckpts)
        return u

    @staticmethod
    def backward(ctx, gu):
        s, *ckpts = ctx.saved_tensors
        ubar = gu.contiguous().clone()
        sbar = torch.zeros_like(s)
        for u_t in reversed(ckpts):
            B.adi_step_adjoint(u_t, s, ubar, sbar)
        return ubar, sbar, None


def gtsv(a, b, c, d, axis):
    """Differentiable batched solve (arrays form)."""
    return TridSolveFn.apply(a, b, c, d, axis)


def gtsv_s(s, d, axis):
    """Differentiable batched solve with rows (-s, 1 + 2 s, -s)."""
    return TridSolveSFn.apply(s, d, axis)


def adi(u0, s, nsteps):
    """Differentiable ADI time loop (per-point s), per-step checkpointing."""
    return ADIFn.apply(u0, s, nsteps)
