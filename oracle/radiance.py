"""FP64 CPU oracle of radiance-field compositing: the Max optical model along a ray (Sec. 3.3,
Eq. 10) with a ReLU density, and the photometric loss (Sec. 3.3, Eq. 11).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU-baseline leg use
it; the GPU library never imports, links or calls it, and it shares nothing with the GPU path.

Per ray r with samples i = 0..N-1 (positions along the ray in order):
  sigma_i = max(f_i, 0)              f: the density grid's value at the sample
  a_i     = sigma_i * delta_i         delta_i: the distance to the next sample
  T_i     = exp(-sum_{j<i} a_j)       transmittance up to the sample
  alpha_i = 1 - exp(-a_i)
  C(r)    = sum_i T_i alpha_i c_i     c_i: the three colour channels at the sample
  L       = (1/R) sum_r |C(r) - target_r|^2
The adjoint, written out from those definitions (the paper prints none):
  dL/dC(r)       = 2 (C(r) - target_r) / R
  dL/dc_i        = dL/dC . (T_i alpha_i)                         per channel
  dC/dsigma_i    = delta_i (T_i exp(-a_i) c_i - sum_{j>i} T_j alpha_j c_j)
  dL/df_i        = [f_i > 0] dL/dC . dC/dsigma_i

Parity status: pinned by ``tests/test_oracle_radiance.py`` (closed forms for one sample and for
a homogeneous ray, the product form of the transmittance, the telescoping sum of the weights,
central finite differences of both gradients); none is unpinned.
"""
from __future__ import annotations

import numpy as np


def composite(f, c, delta):
    """Eq. 10 with sigma = relu(f).  f, delta: [R, N]; c: [R, N, 3].
    Returns (rgb [R, 3], T [R, N], alpha [R, N])."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    sigma = np.maximum(f, 0.0)
    a = sigma * delta
    R, N = a.shape
    T = np.empty((R, N))
    run = np.zeros(R)
    for i in range(N):  # sum over the samples before i
        T[:, i] = np.exp(-run)
        run = run + a[:, i]
    alpha = 1.0 - np.exp(-a)
    rgb = np.einsum("rn,rnk->rk", T * alpha, c)
    return rgb, T, alpha


def photometric_loss(rgb, target):
    """Eq. 11: the mean over the rays of the squared colour error."""
    d = np.asarray(rgb, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.sum(d * d) / d.shape[0])


def composite_backward(f, c, delta, target):
    """Loss and gradients of Eq. 11 through Eq. 10: returns (loss, rgb, g_f [R, N], g_c [R, N, 3])."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    rgb, T, alpha = composite(f, c, delta)
    R, N = f.shape
    loss = photometric_loss(rgb, target)
    g_rgb = 2.0 * (rgb - np.asarray(target, dtype=np.float64)) / R  # [R, 3]
    w = T * alpha
    g_c = w[:, :, None] * g_rgb[:, None, :]
    wc = w[:, :, None] * c                                # each sample's contribution to C
    after = np.zeros((R, N, 3))                           # sum_{j>i} T_j alpha_j c_j
    acc = np.zeros((R, 3))
    for i in range(N - 1, -1, -1):
        after[:, i] = acc
        acc = acc + wc[:, i]
    a = np.maximum(f, 0.0) * delta
    dC_dsigma = delta[:, :, None] * (T[:, :, None] * np.exp(-a)[:, :, None] * c - after)
    g_sigma = np.einsum("rnk,rk->rn", dC_dsigma, g_rgb)
    g_f = np.where(f > 0.0, g_sigma, 0.0)
    return loss, rgb, g_f, g_c
