"""SDF quality measures on the GPU (the paper reports IoU and Chamfer distance, Sec. 4.1):
IoU of the inside sets on sample points, the zero-level-set mesh of a sampled field
(marching tetrahedra), and the Chamfer distance between point sets.

Argument marshalling only: the counting, the meshing and the distances run in the library
(``tg_iou_counts``, ``tg_mesh``, ``tg_chamfer``).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .grid import _check_tensor, _ptr, _stream


def _reduce_ws(dev):
    return torch.empty(_lib.lib().tg_reduce_workspace_bytes(), dtype=torch.uint8, device=dev)


def iou(f, d, ws=None):
    """IoU of {f < 0} and {d < 0}; returns (iou, |A and B|, |A or B|)."""
    dev = f.device
    n = f.numel()
    _check_tensor("f", f, torch.float32, dev)
    _check_tensor("d", d, torch.float32, dev, n)
    ws = _reduce_ws(dev) if ws is None else ws
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    _lib.call("tg_iou_counts", n, _ptr(f), _ptr(d), _ptr(counts), _ptr(ws), ws.numel(), _stream(dev))
    inter, union = (int(x) for x in counts.cpu())
    return (1.0 if union == 0 else inter / union), inter, union


def mesh(values, lo, hi, max_tris=None):
    """Zero-level-set triangles [T, 3, 3] of values [nz, ny, nx] sampled on the lattice over
    [lo, hi]^3 (marching tetrahedra, in the library's documented order)."""
    dev = values.device
    nz, ny, nx = values.shape
    _check_tensor("values", values, torch.float32, dev)
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    lo_c = (ctypes.c_float * 3)(*[float(v) for v in lo])
    hi_c = (ctypes.c_float * 3)(*[float(v) for v in hi])
    wsb = _lib.lib().tg_mesh_workspace_bytes(n)
    if wsb == 0:
        raise ValueError("lattice too small or too large")
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = 0 if max_tris is None else int(max_tris)
    tri = torch.empty((max(cap, 1), 3, 3), dtype=torch.float32, device=dev)
    _lib.call("tg_mesh", n, lo_c, hi_c, _ptr(values), _ptr(tri), cap, _ptr(count), _ptr(ws), ws.numel(), _stream(dev))
    total = int(count.item())
    if max_tris is None and total > 0:  # size the output from the first call's count
        tri = torch.empty((total, 3, 3), dtype=torch.float32, device=dev)
        _lib.call("tg_mesh", n, lo_c, hi_c, _ptr(values), _ptr(tri), total, _ptr(count), _ptr(ws), ws.numel(),
                  _stream(dev))
        cap = total
    return tri[: min(total, cap)], total


def chamfer(a, b, ws=None):
    """Chamfer distance of point sets a [Na, 3], b [Nb, 3]: (total, mean a->b, mean b->a)."""
    dev = a.device
    _check_tensor("a", a, torch.float32, dev)
    _check_tensor("b", b, torch.float32, dev)
    ws = _reduce_ws(dev) if ws is None else ws
    out = torch.empty(3, dtype=torch.float64, device=dev)
    _lib.call("tg_chamfer", _ptr(a), a.shape[0], _ptr(b), b.shape[0], _ptr(out), _ptr(ws), ws.numel(), _stream(dev))
    return tuple(float(x) for x in out.cpu())
