"""FP64 CPU oracle of the rest of the paper's SDF objective (Sec. 3.2, Eq. 6-8) and of the
coarse-to-fine resolution step of its training schedule (Sec. 4.1).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU-baseline leg use
it; the GPU library never imports, links or calls it, and it shares nothing with the GPU path.

* Adaptive surface weight (Eq. 7): w'(d) = 1 - |2 sigmoid(k d) - 1| and
  w(x) = max(w'(f(x)), w'(d(x))), applied to the L1 term of Eq. 6:
      L_recon = (1/n) sum_i w_i |f_i - d_i|.
  The weight is a per-sample importance and is held fixed when differentiating (no gradient
  flows through w'(f)); k = 0 makes every weight 1, the unweighted loss.
* Total variation (Eq. 8's L_TV, Plenoxels' regulariser): over every vertex v of the grid and
  every stored coefficient channel c,
      Delta_a(v, c) = C(v + e_a, c) - C(v, c)   (0 where v + e_a is outside the grid),
      TV = (1/|V|) sum_v sum_c sqrt(sum_a Delta_a(v, c)^2),
  with the gradient of a term whose differences are all zero taken as 0.
* Coarse-to-fine step: the fine grid's coefficients at each fine vertex are the value,
  gradient and Hessian of the coarse field there (Eq. 1's series of the field that the coarse
  grid already represents), truncated to the fine grid's order.

Parity status: pinned by ``tests/test_oracle_objective.py`` (the weight's closed form and
limits, the unweighted special case, finite differences with the weight held fixed; TV of a
linear ramp in closed form, invariances and finite differences; exact upsampling of a
quadratic); none is unpinned.
"""
from __future__ import annotations

import numpy as np

from . import Geometry, forward, sdf_loss


def surface_weight_1(d, k):
    """w'(d) of Eq. 7, written as the paper defines it (sigmoid(z) = 1 / (1 + exp(-z)))."""
    z = k * np.asarray(d, dtype=np.float64)
    with np.errstate(over="ignore"):
        sig = 1.0 / (1.0 + np.exp(-z))
    return 1.0 - np.abs(2.0 * sig - 1.0)


def surface_weight(f, d, k):
    """w(x) of Eq. 7: the larger of the predicted and the true distance's weights."""
    return np.maximum(surface_weight_1(f, k), surface_weight_1(d, k))


def weighted_sdf_loss(f, grad, d, w_eik, k):
    """Eq. 6 with Eq. 7's weight, plus the eikonal term: returns (loss[3], g_f, g_grad) with
    loss = [L_recon + w_eik L_eik, L_recon, L_eik] and the upstream gradients (weight fixed)."""
    f = np.asarray(f, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n = f.shape[0]
    w = surface_weight(f, d, k)
    out, gf, gg = sdf_loss(f, grad, d, w_eik)  # the unweighted terms (C oracle)
    recon = float(np.sum(w * np.abs(f - d)) / n) if n else 0.0
    loss = np.array([recon + w_eik * out[2], recon, out[2]])
    return loss, w * gf, gg


def _axes_of(coeffs, dim):
    """Vertex axes of a [res_z, res_y, res_x, C] (or [res_y, res_x, C]) array: x, y (, z)."""
    return [dim - 1 - a for a in range(dim)]


def tv(coeffs, dim):
    """TV value and its gradient with respect to every coefficient."""
    C = np.asarray(coeffs, dtype=np.float64)
    nvert = int(np.prod(C.shape[:dim]))
    deltas = []
    for ax in _axes_of(C, dim):
        dl = np.zeros_like(C)
        sl_lo = [slice(None)] * C.ndim
        sl_hi = [slice(None)] * C.ndim
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        dl[tuple(sl_lo)] = C[tuple(sl_hi)] - C[tuple(sl_lo)]  # forward difference, 0 on the last layer
        deltas.append((ax, dl))
    s = np.sqrt(sum(dl * dl for _, dl in deltas))
    value = float(s.sum() / nvert)
    safe = np.where(s > 0.0, s, 1.0)
    grad = np.zeros_like(C)
    for ax, dl in deltas:
        q = np.where(s > 0.0, dl / safe, 0.0)  # d s(v) / d Delta_a(v)
        # Delta_a(v) = C(v + e_a) - C(v): -q at v, +q at v + e_a
        grad -= q
        sl_lo = [slice(None)] * C.ndim
        sl_hi = [slice(None)] * C.ndim
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        grad[tuple(sl_hi)] += q[tuple(sl_lo)]
    return value, grad / nvert


def upsample(geom_coarse: Geometry, coeffs_coarse, geom_fine: Geometry):
    """Fine-grid coefficients [.., C_fine] from the coarse field's value, gradient and
    Hessian at the fine vertices, in the stored order (value; gradient x, y(, z); Hessian
    xx, xy(, xz), yy(, yz, zz)), truncated to the fine order."""
    dim = geom_fine.dim
    axes = [np.linspace(geom_fine.lo[a], geom_fine.hi[a], geom_fine.res[a]) for a in range(dim)]
    mesh = np.meshgrid(*axes, indexing="ij")  # mesh[a][i_x, i_y(, i_z)]
    pts = np.stack([m.transpose(tuple(reversed(range(dim)))).reshape(-1) for m in mesh], axis=1)
    f, g, h = forward(geom_coarse, coeffs_coarse, pts, want_grad=True, want_hess=True)
    cols = [f]
    if geom_fine.order >= 1:
        cols += [g[:, a] for a in range(dim)]
    if geom_fine.order >= 2:
        cols += [h[:, a, b] for a in range(dim) for b in range(a, dim)]
    return np.stack(cols, axis=1).reshape(geom_fine.coeff_shape)
