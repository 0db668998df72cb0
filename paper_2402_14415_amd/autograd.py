"""Differentiation form: the TaylorGrid forward/adjoint behind torch.autograd.

``f, grad_f = taylor_grid(grid, q)`` returns the field value and its analytic spatial
gradient (needed for normals and the eikonal term of Sec. 3.2, Eq. 8).  Gradients flow to
``grid.master`` (the FP32 parameters; with 16-bit storage the forward reads the rounded
copy and the gradient is applied to the master) and, if requested, to the queries.  Both
adjoints run in the HIP kernels (tg_backward); this module only routes tensors.  The
backward is differentiable once: the adjoint kernels have no adjoint of their own, so a
second-order graph (``create_graph=True``) raises instead of returning wrong gradients.
"""
from __future__ import annotations

import torch

from .grid import TaylorGrid


class TaylorGridFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, master, q, grid: TaylorGrid, ws):
        grid.sort(q, ws)
        f, g = grid.forward(q, ws, want_grad=True)
        ctx.grid = grid
        ctx.ws = ws
        ctx.save_for_backward(q)
        return f, g

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_f, g_grad):
        (q,) = ctx.saved_tensors
        grid, ws = ctx.grid, ctx.ws
        grid.ensure_sorted(q, ws)
        g_f = None if g_f is None else g_f.contiguous().float()
        g_grad = None if g_grad is None else g_grad.contiguous().float()
        d_master = None
        if ctx.needs_input_grad[0]:
            d_master = torch.empty_like(grid.master)
        want_dq = bool(ctx.needs_input_grad[1])
        dq = None
        if d_master is not None or want_dq:
            scratch = d_master if d_master is not None else torch.empty_like(grid.master)
            dq = grid.backward(q, ws, g_f, g_grad, want_dq=want_dq, grad_out=scratch)
        return d_master, dq, None, None


def taylor_grid(grid: TaylorGrid, q: torch.Tensor, ws: torch.Tensor | None = None):
    """Differentiable (f, grad f) of the grid at queries q [n, dim]."""
    if ws is None:
        ws = grid.workspace(q.shape[0])
    return TaylorGridFn.apply(grid.master, q, grid, ws)
