"""Differentiable wrappers of the line solves and the ADI time loop.

The backward passes are the library's hand-written adjoint kernels:
  - a line solve x = A^{-1} d has dL/dd = A^{-T} dL/dx (a tridiagonal solve with
    the transposed rows) and dL/dA = -lambda x^T restricted to the three
    diagonals;
  - one ADI step (Alg. 3 of arxiv 2201.03950 with per-point s) is reversed
    with its intermediates -- kept by the forward pass, or recomputed from the
    step's input checkpoint -- by the transposed solves z -> y -> x, and the
    stencil's adjoint closes the step.
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

    keep=False: one checkpoint per step (the field entering it); the reverse
    pass recomputes the step's intermediates from it.
    keep=True: each step also keeps its intermediates (2 or 3 mesh-sized
    arrays more per step), so the reverse pass recomputes nothing.
    """

    @staticmethod
    def forward(ctx, u0, s, nsteps, keep):
        s = s.contiguous()
        u = u0.detach().contiguous().clone()
        saved = []
        for _ in range(int(nsteps)):
            saved.append(u.clone())
            if keep:
                ws = [torch.empty_like(u) for _ in range(u.dim() - 1)]
                B.adi_step_keep(u, s, *ws)
                saved.extend(ws)
            else:
                B.adi_step(u, s=s, nsteps=1)
        ctx.keep = bool(keep)
        ctx.per = 1 + (u.dim() - 1 if keep else 0)  # saved tensors per step
        ctx.save_for_backward(s, *saved)
        return u

    @staticmethod
    def backward(ctx, gu):
        s, *saved = ctx.saved_tensors
        ubar = gu.contiguous().clone()
        sbar = torch.zeros_like(s)
        steps = [saved[i:i + ctx.per] for i in range(0, len(saved), ctx.per)]
        for step in reversed(steps):
            if ctx.keep:
                u_t, *ws = step
                w3 = ws[2] if len(ws) == 3 else None
                B.adi_step_adjoint_kept(u_t, s, ws[0], ws[1], w3, ubar, sbar)
            else:
                B.adi_step_adjoint(step[0], s, ubar, sbar)
        return ubar, sbar, None, None


def gtsv(a, b, c, d, axis):
    """Differentiable batched solve (arrays form)."""
    return TridSolveFn.apply(a, b, c, d, axis)


def gtsv_s(s, d, axis):
    """Differentiable batched solve with rows (-s, 1 + 2 s, -s)."""
    return TridSolveSFn.apply(s, d, axis)


def adi(u0, s, nsteps, keep=True):
    """Differentiable ADI time loop (per-point s).  keep=True keeps each step's
    intermediates (no recomputation in the reverse pass); keep=False keeps one
    checkpoint per step and recomputes."""
    return ADIFn.apply(u0, s, nsteps, keep)
