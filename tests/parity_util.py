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


# Rule for queries on a face.  The field is continuous across an interior face of the grid,
# but its gradient (and so dq and a query's share of dC) is not: for a query on a face,
# either adjacent cell's one-sided value is correct (Sec. 3.1 does not say which cell owns a
# face).  The kernels locate cells in FP32 two-float arithmetic that agrees with the FP64
# oracle except within about 2^-46 s of a face; FACE_GAP (in cell units) covers that band
# with a wide margin.  Queries within FACE_GAP of an interior face are counted, and for them
# the comparison accepts the oracle's value on either side of every such face.
FACE_GAP = 1e-8


def face_alternatives(q64, lo, hi, res, gap=FACE_GAP):
    """(indices of the queries within `gap` of an interior vertex plane on some unclamped
    axis, and for each the query moved 4 gap h to either side along every such axis, in
    every combination of sides, as an [m, dim] array)."""
    q = np.asarray(q64, dtype=np.float64)
    dim = q.shape[1]
    lo = np.asarray(lo, dtype=np.float64)[:dim]
    hi = np.asarray(hi, dtype=np.float64)[:dim]
    res = np.asarray(res)[:dim]
    h = (hi - lo) / (res - 1)
    s = (q - lo) / h
    k = np.round(s)
    near = (np.abs(s - k) < gap) & (k >= 1) & (k <= res - 2) & (q > lo) & (q < hi)
    idx = np.nonzero(near.any(axis=1))[0]
    alts = []
    for i in idx:
        axes = np.nonzero(near[i])[0]
        rows = []
        for signs in np.ndindex(*(2,) * len(axes)):
            r = q[i].copy()
            for a, sg in zip(axes, signs):
                r[a] += (4 * gap if sg else -4 * gap) * h[a]
            rows.append(r)
        alts.append(np.array(rows))
    return idx, alts


class FaceRule:
    """Comparisons of one query set under the face rule; ``count`` is the number of queries
    within FACE_GAP of an interior face."""

    def __init__(self, geom, C64, q64):
        self.geom = geom
        self.C = C64
        self.q = np.asarray(q64, dtype=np.float64)
        self.idx, self.alts = face_alternatives(self.q, geom.lo, geom.hi, geom.res)
        self.count = len(self.idx)

    def _err_rows(self, x, ref, alt_rows):
        x = np.asarray(x, dtype=np.float64).reshape(len(self.q), -1)
        ref = np.asarray(ref, dtype=np.float64).reshape(len(self.q), -1)
        err = np.abs(x - ref)
        for i, qa in zip(self.idx, self.alts):
            rows = alt_rows(qa, i).reshape(len(qa), -1)
            cand = np.abs(x[i] - rows)
            j = int(np.argmin(cand.max(axis=1)))
            if cand[j].max() < err[i].max():
                err[i] = cand[j]
        scale = np.max(np.abs(ref), axis=0)
        scale[scale == 0] = 1.0
        return float(np.max(err.max(axis=0) / scale)) if len(ref) else 0.0

    def grad_err(self, x, ref):
        """Per-component normalised error of grad f against the oracle's."""
        return self._err_rows(x, ref, lambda qa, i: oracle.forward(self.geom, self.C, qa)[1])

    def dq_err(self, x, ref, gf, gg):
        """Per-component normalised error of dq; gf [n] / gg [n, dim] (either may be None)."""
        def rows(qa, i):
            m = len(qa)
            a = None if gf is None else np.repeat(np.asarray(gf, dtype=np.float64)[i : i + 1], m)
            b = None if gg is None else np.repeat(np.asarray(gg, dtype=np.float64)[i : i + 1], m, axis=0)
            return oracle.backward(self.geom, self.C, qa, a, b, want_dq=True)[1]
        return self._err_rows(x, ref, rows)

    def dC_slack(self, gf, gg):
        """Per coefficient, the largest change of dC that moving the near-face queries to
        either side can make (0 everywhere when no query is near a face)."""
        slack = np.zeros(self.C.size)
        for i, qa in zip(self.idx, self.alts):
            a = None if gf is None else np.asarray(gf, dtype=np.float64)[i : i + 1]
            b = None if gg is None else np.asarray(gg, dtype=np.float64)[i : i + 1]
            base = oracle.backward(self.geom, self.C, self.q[i : i + 1], a, b)[0].reshape(-1)
            worst = np.zeros_like(slack)
            for r in qa:
                other = oracle.backward(self.geom, self.C, r[None], a, b)[0].reshape(-1)
                worst = np.maximum(worst, np.abs(other - base))
            slack += worst
        return slack

    def dC_err(self, x, ref, gf, gg):
        """Normalised error of dC with the near-face queries' slack taken off."""
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        ref = np.asarray(ref, dtype=np.float64).reshape(-1)
        slack = self.dC_slack(gf, gg) if self.count else 0.0
        scale = np.max(np.abs(ref)) if ref.size else 1.0
        return float(np.max(np.maximum(np.abs(x - ref) - slack, 0.0)) / (scale if scale > 0 else 1.0))


def device():
    return torch.device("cuda", 0)
