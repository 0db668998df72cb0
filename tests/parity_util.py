"""Shared helpers for the GPU parity tests (comparison rule and oracle plumbing).

Tolerance rule.  Element-wise relative error is ill-posed at the zero level set, where
surface queries put f near 0, so each output tensor is compared by its normalised maximum
error  err(x, ref) = max_i |x_i - ref_i| / max_i |ref_i|  (per component for vectors):
  f, SDF loss terms, Adam master ........................ <= 1e-5
  grad f, dC (coefficient adjoint), dq, g_f, g_grad ..... <= 1e-4
The FP32 kernels are compared with the FP64 oracle run on the same FP32-rounded inputs.
"""
import numpy as np
import torch

import oracle

TOL_VALUE = 1e-5
TOL_GRAD = 1e-4


def nerr(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (scale if scale > 0 else 1.0))


def nerr_cols(x, ref):
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    return max(nerr(x[:, a], ref[:, a]) for a in range(ref.shape[1]))


def to_np(t):
    return t.detach().cpu().double().numpy()


def geometry(grid):
    return oracle.Geometry(grid.dim, grid.res, grid.order, grid.lo, grid.hi)


def nudge_off_faces(q, lo, hi, res, gap=1e-9):
    """Move the rare queries whose cell coordinate lies within `gap` of an integer slightly
    into the cell, so that both sides pick the same cell (the gradient is discontinuous
    across faces, so on a face either adjacent cell is a valid answer)."""
    q = np.array(q, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / (np.asarray(res) - 1)
    s = (np.clip(q, lo, hi) - lo) / h
    near = np.abs(s - np.round(s)) < gap
    inside = (q > lo) & (q < hi)
    fix = near & inside
    if fix.any():
        q[fix] = q[fix] + 1e-6 * np.broadcast_to(h, q.shape)[fix]
    return q.astype(np.float32).astype(np.float64)


def device():
    return torch.device("cuda", 0)
