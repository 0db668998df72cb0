"""SDF quality measures on the GPU (the paper reports IoU and the Chamfer-L1 distance of the
mesh that marching cubes extracts from the field, Sec. 4.1): IoU of the inside sets on sample
points, a grid's field on a lattice finer than the grid, the zero-level-set mesh of a sampled
field (marching cubes), and the Chamfer distance between point sets (L1 or Euclidean).

Argument marshalling only: the counting, the sampling, the meshing and the distances run in
the library (``tg_iou_counts``, ``tg_field_lattice``, ``tg_mesh``, ``tg_chamfer``).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .grid import _check_tensor, _ptr, _stream


def _reduce_ws(dev):
    return torch.empty(_lib.lib().tg_reduce_workspace_bytes(), dtype=torch.uint8, device=dev)


def iou_counts(f, d, ws=None, counts=None):
    """Device int64 [2]: (|A and B|, |A or B|) of A = {f < 0}, B = {d < 0} (no host sync)."""
    dev = f.device
    n = f.numel()
    _check_tensor("f", f, torch.float32, dev)
    _check_tensor("d", d, torch.float32, dev, n)
    ws = _reduce_ws(dev) if ws is None else ws
    counts = torch.empty(2, dtype=torch.int64, device=dev) if counts is None else counts
    _lib.call("tg_iou_counts", n, _ptr(f), _ptr(d), _ptr(counts), _ptr(ws), ws.numel(), _stream(dev))
    return counts


def iou(f, d, ws=None):
    """IoU of {f < 0} and {d < 0}; returns (iou, |A and B|, |A or B|)."""
    inter, union = (int(x) for x in iou_counts(f, d, ws).cpu())
    return (1.0 if union == 0 else inter / union), inter, union


def field_lattice(grid, s, out=None):
    """The grid's field on the lattice s times finer than the grid: values [nz, ny, nx] with
    n = s (res - 1) + 1 per axis (point i at lo + i h / s, located exactly: a point on a cell
    face takes the cell above)."""
    n = [s * (r - 1) + 1 for r in grid.res]
    shape = (n[2], n[1], n[0])
    out = torch.empty(shape, dtype=torch.float32, device=grid.device) if out is None else out
    _check_tensor("out", out, torch.float32, grid.device, n[0] * n[1] * n[2])
    _lib.call("tg_field_lattice", grid.handle, int(s), _ptr(out), _stream(grid.device))
    return out


class MeshLattice:
    """The lattice arguments and workspace of tg_mesh for values [nz, ny, nx] over [lo, hi]^3."""

    def __init__(self, shape, lo, hi, device):
        nz, ny, nx = shape
        self.n = (ctypes.c_int32 * 3)(nx, ny, nz)
        self.lo = (ctypes.c_float * 3)(*[float(v) for v in lo])
        self.hi = (ctypes.c_float * 3)(*[float(v) for v in hi])
        wsb = _lib.lib().tg_mesh_workspace_bytes(self.n)
        if wsb == 0:
            raise ValueError("lattice too small or too large")
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)

    def run(self, values, tri, max_tris):
        """Enqueue the mesh into tri (capacity max_tris); the total goes to self.count (no sync)."""
        _check_tensor("values", values, torch.float32, values.device)
        _lib.call("tg_mesh", self.n, self.lo, self.hi, _ptr(values), _ptr(tri), int(max_tris), _ptr(self.count),
                  _ptr(self.ws), self.ws.numel(), _stream(values.device))


def mesh(values, lo, hi, max_tris=None):
    """Zero-level-set triangles [T, 3, 3] of values [nz, ny, nx] sampled on the lattice over
    [lo, hi]^3 (marching cubes, in the library's documented order), and the total count."""
    dev = values.device
    lat = MeshLattice(values.shape, lo, hi, dev)
    cap = 0 if max_tris is None else int(max_tris)
    tri = torch.empty((max(cap, 1), 3, 3), dtype=torch.float32, device=dev)
    lat.run(values, tri, cap)
    total = int(lat.count.item())
    if max_tris is None and total > 0:  # size the output from the first call's count
        tri = torch.empty((total, 3, 3), dtype=torch.float32, device=dev)
        lat.run(values, tri, total)
        cap = total
    return tri[: min(total, cap)], total


def chamfer_workspace(na, nb, device):
    """A workspace for the Chamfer distance of na and nb points (tg_chamfer_workspace_bytes)."""
    nbytes = _lib.lib().tg_chamfer_workspace_bytes(int(na), int(nb))
    if nbytes == 0:
        raise ValueError(f"chamfer: point counts {na}, {nb} out of range")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def chamfer_into(a, b, out, ws, norm=1):
    """Enqueue the Chamfer distance of a [Na, 3] and b [Nb, 3] into out (device float64 [3]);
    norm 1: L1 point distances (the paper's CD-L1), 2: Euclidean; ws: chamfer_workspace(Na, Nb)."""
    dev = a.device
    _check_tensor("a", a, torch.float32, dev)
    _check_tensor("b", b, torch.float32, dev)
    _check_tensor("out", out, torch.float64, dev, 3)
    _lib.call("tg_chamfer", _ptr(a), a.shape[0], _ptr(b), b.shape[0], int(norm), _ptr(out), _ptr(ws), ws.numel(),
              _stream(dev))
    return out


def chamfer(a, b, ws=None, norm=1):
    """Chamfer distance of point sets a [Na, 3], b [Nb, 3]: (total, mean a->b, mean b->a)."""
    ws = chamfer_workspace(a.shape[0], b.shape[0], a.device) if ws is None else ws
    out = torch.empty(3, dtype=torch.float64, device=a.device)
    return tuple(float(x) for x in chamfer_into(a, b, out, ws, norm).cpu())
