"""NumPy brute force of the TaylorGrid field for tiny grids (TEST INFRASTRUCTURE ONLY).

A second, independent implementation used to cross-check the C oracle.  It is written in
the matrix form of Eq. 1 (Sec. 3.1): T(x - v) = f0 + g.(x - v) + 1/2 (x - v)^T H (x - v),
with H the full symmetric Hessian assembled from the stored entries, followed by the
multilinear interpolation of Eq. 4 over the corners of the cell of Eq. 2.  Only orders
0, 1 and 2 are supported.  The adjoint is obtained by its definition: probing the forward
map with every unit coefficient vector gives the Jacobian, whose transpose is applied to
the upstream gradients.
"""
from __future__ import annotations

import itertools

import numpy as np


def _hessian_from_entries(entries, dim):
    """Stored second derivatives (graded-lex: xx, xy, xz, yy, yz, zz) -> symmetric matrix."""
    H = np.zeros((dim, dim))
    k = 0
    for a in range(dim):
        for c in range(a, dim):
            H[a, c] = H[c, a] = entries[k]
            k += 1
    return H


def _taylor(block, d, order, dim):
    """Value and gradient (in x) of one vertex's polynomial at world offset d."""
    val = block[0]
    grad = np.zeros(dim)
    if order >= 1:
        g = np.asarray(block[1 : 1 + dim])
        val = val + g @ d
        grad = grad + g
    if order >= 2:
        H = _hessian_from_entries(block[1 + dim :], dim)
        val = val + 0.5 * d @ H @ d
        grad = grad + H @ d
    return val, grad


def forward(dim, res, order, lo, hi, coeffs, q):
    """Field value and spatial gradient for each query (Python loops; tiny inputs only)."""
    res = np.asarray(res[:dim], dtype=np.int64)
    lo = np.asarray(lo[:dim], dtype=np.float64)
    hi = np.asarray(hi[:dim], dtype=np.float64)
    C = np.asarray(coeffs, dtype=np.float64).reshape(int(np.prod(res)), -1)
    h = (hi - lo) / (res - 1)
    q = np.asarray(q, dtype=np.float64).reshape(-1, dim)
    f = np.zeros(len(q))
    G = np.zeros((len(q), dim))
    for n, qq in enumerate(q):
        x = np.clip(qq, lo, hi)
        clamped = x != qq
        s = (x - lo) / h
        cell = np.minimum(np.floor(s).astype(np.int64), res - 2)
        t = s - cell
        for b in itertools.product((0, 1), repeat=dim):
            b = np.asarray(b)
            vid = cell + b
            flat = 0
            for a in reversed(range(dim)):
                flat = flat * res[a] + vid[a]
            v = lo + vid * h
            d = x - v
            val, grad = _taylor(C[flat], d, order, dim)
            fac = np.where(b == 1, t, 1.0 - t)
            w = np.prod(fac)
            dw = np.array([(1.0 if b[a] else -1.0) / h[a] * np.prod(np.delete(fac, a)) for a in range(dim)])
            f[n] += w * val
            G[n] += dw * val + w * grad
        G[n][clamped] = 0.0
    return f, G


def backward(dim, res, order, lo, hi, num_coeffs, q, gf, gg):
    """dC = J^T [gf; gg], J built column by column from unit coefficient vectors."""
    nvert = int(np.prod(res[:dim]))
    total = nvert * num_coeffs
    q = np.asarray(q, dtype=np.float64).reshape(-1, dim)
    gf = np.asarray(gf, dtype=np.float64).reshape(-1)
    gg = np.asarray(gg, dtype=np.float64).reshape(-1, dim)
    dC = np.zeros(total)
    for k in range(total):
        e = np.zeros(total)
        e[k] = 1.0
        f, G = forward(dim, res, order, lo, hi, e, q)
        dC[k] = gf @ f + np.sum(gg * G)
    return dC
