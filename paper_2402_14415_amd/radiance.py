"""Radiance-field form (Sec. 3.3): a density TaylorGrid (K=2, ReLU) and a three-channel colour
TaylorGrid (K=1, the three channels' series stored per vertex) on the same vertices, rendered
along rays by the Max optical model (Eq. 10) and fitted to observed ray colours by the
photometric loss (Eq. 11).

Argument marshalling only: the bucketing (once per batch, shared by both grids), the grid
evaluations, the compositing with its adjoint and the fused adjoint + Adam of every grid run in
the library (``tg_sort_queries``, ``tg_share_sort``, ``tg_forward``, ``tg_composite``,
``tg_backward_adam``).
"""
from __future__ import annotations

import torch

from . import _lib
from .grid import TaylorGrid, _check_tensor, _ptr, _stream


def composite(f, c, delta, n_samples, ws, target=None, rgb=None, loss=None, g_f=None, g_c=None):
    """Eq. 10 along rays of ``n_samples`` samples (ray-major): f [N] density-grid values, c
    [3, N] colour channels, delta [N] sample spacings.  Returns (rgb [R, 3], loss, g_f, g_c);
    with ``target`` [R, 3] also the loss (device float64 [1]) of Eq. 11 and the upstream
    gradients g_f [N] and g_c [3, N] for the grids' adjoints (else None)."""
    dev = f.device
    n = f.numel()
    if n_samples < 1 or n % n_samples:
        raise ValueError("the sample count must be a multiple of n_samples")
    n_rays = n // n_samples
    _check_tensor("f", f, torch.float32, dev, n)
    _check_tensor("c", c, torch.float32, dev, 3 * n)
    _check_tensor("delta", delta, torch.float32, dev, n)
    rgb = torch.empty((n_rays, 3), dtype=torch.float32, device=dev) if rgb is None else rgb
    _check_tensor("rgb", rgb, torch.float32, dev, 3 * n_rays)
    if target is not None:
        _check_tensor("target", target, torch.float32, dev, 3 * n_rays)
        loss = torch.empty(1, dtype=torch.float64, device=dev) if loss is None else loss
        g_f = torch.empty(n, dtype=torch.float32, device=dev) if g_f is None else g_f
        g_c = torch.empty((3, n), dtype=torch.float32, device=dev) if g_c is None else g_c
        _check_tensor("loss", loss, torch.float64, dev, 1)
        _check_tensor("g_f", g_f, torch.float32, dev, n)
        _check_tensor("g_c", g_c, torch.float32, dev, 3 * n)
    else:
        loss = g_f = g_c = None
    _lib.call("tg_composite", n_rays, n_samples, _ptr(f), _ptr(c), _ptr(delta), _ptr(target), _ptr(rgb), _ptr(loss),
              _ptr(g_f), _ptr(g_c), _ptr(ws), ws.numel(), _stream(dev))
    return rgb, loss, g_f, g_c


class RadianceField:
    """Density grid (K=2) and a three-channel colour grid (K=1, 12 coefficients per vertex in
    3D) on one vertex lattice over [lo, hi]^3.  ``coeffs`` optionally gives the initial FP32
    coefficients: (density [res_z, res_y, res_x, 10], colour [res_z, res_y, res_x, 12] or a
    list of the three channels' [res_z, res_y, res_x, 4])."""

    def __init__(self, res=(160, 160, 160), lo=(-1.0,) * 3, hi=(1.0,) * 3, device="cuda", coeffs=None):
        dens, col = coeffs if coeffs is not None else (None, None)
        if isinstance(col, (list, tuple)):
            col = torch.cat([torch.as_tensor(c) for c in col], dim=-1)
        self.density = TaylorGrid(3, res, 2, lo, hi, coeffs=dens, device=device)
        self.colour = TaylorGrid(3, res, 1, lo, hi, coeffs=col, device=device, channels=3)
        self.device = self.density.device
        self.reduce_ws = torch.empty(_lib.lib().tg_reduce_workspace_bytes(), dtype=torch.uint8, device=self.device)

    @property
    def grids(self):
        return [self.density, self.colour]

    def workspace(self, n):
        """One workspace for both grids: they share one vertex lattice, so the samples are
        bucketed once (by the density grid) and the colour grid reuses that sort.  It is sized
        for the grid with the most coefficients per vertex."""
        nb = max(g.workspace_bytes(n) for g in self.grids)
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    def evaluate(self, q, ws, f=None, c=None):
        """Sort the samples once and evaluate both grids: f [N] density values, c [3, N] colours."""
        n = q.shape[0]
        f = torch.empty(n, dtype=torch.float32, device=self.device) if f is None else f
        c = torch.empty((3, n), dtype=torch.float32, device=self.device) if c is None else c
        self.density.sort(q, ws)
        self.density.forward(q, ws, want_grad=False, out=(f, None))
        self.colour.share_sort(self.density, q, ws)
        self.colour.forward(q, ws, out=(c, None))
        return f, c

    def render(self, q, delta, n_samples, ws):
        f, c = self.evaluate(q, ws)
        return composite(f, c, delta, n_samples, self.reduce_ws)[0]

    def train_step(self, q, delta, n_samples, target, ws, lr=1e-2, step=None, bufs=None, stage_events=None):
        """One step: evaluate, composite with the loss and its adjoint, then the fused adjoint
        + Adam of both grids.  Returns the loss (device float64 [1]).  ``bufs`` optionally
        carries preallocated (f, c, rgb, loss, g_f, g_c); ``stage_events`` optionally three
        recorded torch.cuda.Events, re-recorded after the evaluation, the compositing and the
        updates."""
        f, c, rgb, loss, g_f, g_c = bufs if bufs is not None else (None,) * 6
        f, c = self.evaluate(q, ws, f, c)
        if stage_events is not None:
            stage_events[0].record()
        _, loss, g_f, g_c = composite(f, c, delta, n_samples, self.reduce_ws, target, rgb, loss, g_f, g_c)
        if stage_events is not None:
            stage_events[1].record()
        self.density.backward_adam(q, ws, g_f, None, lr=lr, step=step)
        self.colour.backward_adam(q, ws, g_c, None, lr=lr, step=step)
        if stage_events is not None:
            stage_events[2].record()
        return loss
