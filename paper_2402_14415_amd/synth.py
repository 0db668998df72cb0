"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input generation only: random coefficient grids, query sets, and the
analytic target fields that stand in for the paper's datasets (which are not available).
It contains none of the TaylorGrid arithmetic and imports neither the GPU library nor the
oracle.

Workloads (shapes follow the paper's SDF-fitting task, Sec. 3.2 and Sec. 4.1):
  * disc2d   : 2D grid on [0,1]^2; queries uniform in the square; target = signed distance
               to the circle of radius 0.3 centred at (0.5, 0.5).
  * scene3d  : 3D grid on [-1,1]^3; a seeded union of 8 spheres (centres U[-0.5,0.5]^3,
               radii U(0.1,0.4)) and one torus (centre U[-0.3,0.3]^3, R=0.3, r=0.08, random
               axis); target = min of the primitives' signed distances.  A batch is half
               uniform points in the box and half points on the union's surface (uniform on
               a uniformly chosen primitive, kept only when no other primitive contains it),
               jittered by N(0, 0.01) per coordinate.
  * radiance : rays of 400 x 400-pixel pinhole cameras (40 degree field of view) placed on a
               sphere of radius 4 around the box and looking at its centre (100 Fibonacci-
               sphere positions); a batch draws random pixels among those whose ray crosses
               the box, clips each ray to the box and places stratified samples on the inside
               segment.  The reference volume is a
               seeded sum of 32 anisotropic Gaussian blobs, each with a density and an RGB
               colour (density- and colour-weighted mixture); it stands in for the
               Synthetic-NeRF scenes.
Random draws use numpy's PCG64 (``default_rng``) in FP64; callers cast to FP32 for the GPU
and give the oracle the same FP32-rounded values.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------- coefficients
def normal_coeffs(shape, std=0.05, seed=0):
    """i.i.d. N(0, std) coefficients (FP64), drawn first from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=shape), rng


# ----------------------------------------------------------------------------- 2D disc
DISC_CENTRE = np.array([0.5, 0.5])
DISC_RADIUS = 0.3


def disc_sdf(q):
    q = np.asarray(q, dtype=np.float64)
    return np.linalg.norm(q - DISC_CENTRE, axis=-1) - DISC_RADIUS


def disc2d_inputs(res=64, order=2, n=65536, seed=0, std=0.05):
    """Coefficients [res, res, C] ~ N(0, std), then n uniform queries in [0,1]^2 and the
    disc SDF at the FP32-rounded queries.  Returns FP64 arrays (q already FP32-exact)."""
    C = (order + 1) * (order + 2) // 2
    coeffs, rng = normal_coeffs((res, res, C), std=std, seed=seed)
    q = rng.uniform(0.0, 1.0, size=(n, 2)).astype(np.float32).astype(np.float64)
    return coeffs, q, disc_sdf(q)


# ----------------------------------------------------------------------------- 3D scene
class Scene:
    """Union of 8 spheres and one torus, seeded."""

    TORUS_R = 0.3
    TORUS_r = 0.08

    def __init__(self, seed=0):
        rng = np.random.default_rng(seed)
        self.centres = rng.uniform(-0.5, 0.5, size=(8, 3))
        self.radii = rng.uniform(0.1, 0.4, size=8)
        self.torus_c = rng.uniform(-0.3, 0.3, size=3)
        axis = rng.normal(size=3)
        self.torus_n = axis / np.linalg.norm(axis)
        # orthonormal frame (e1, e2, n)
        helper = np.array([1.0, 0.0, 0.0]) if abs(self.torus_n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(self.torus_n, helper)
        self.e1 = e1 / np.linalg.norm(e1)
        self.e2 = np.cross(self.torus_n, self.e1)

    # signed distances of each primitive: [..., 9]
    def primitive_sdf(self, p):
        p = np.asarray(p, dtype=np.float64)
        sph = np.linalg.norm(p[..., None, :] - self.centres, axis=-1) - self.radii
        rel = p - self.torus_c
        along = rel @ self.torus_n
        radial = np.linalg.norm(rel - along[..., None] * self.torus_n, axis=-1)
        tor = np.sqrt((radial - self.TORUS_R) ** 2 + along ** 2) - self.TORUS_r
        return np.concatenate([sph, tor[..., None]], axis=-1)

    def sdf(self, p):
        return self.primitive_sdf(p).min(axis=-1)

    def _surface_candidates(self, rng, k):
        prim = rng.integers(0, 9, size=k)
        out = np.empty((k, 3))
        is_s = prim < 8
        ns = int(is_s.sum())
        u = rng.normal(size=(ns, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        out[is_s] = self.centres[prim[is_s]] + self.radii[prim[is_s], None] * u
        nt = k - ns
        if nt:
            R, r = self.TORUS_R, self.TORUS_r
            # area element of the torus is proportional to R + r cos(theta): rejection sample
            theta = np.empty(0)
            while theta.size < nt:
                th = rng.uniform(0, 2 * np.pi, size=2 * nt)
                keep = rng.uniform(0, R + r, size=2 * nt) < R + r * np.cos(th)
                theta = np.concatenate([theta, th[keep]])
            theta = theta[:nt]
            phi = rng.uniform(0, 2 * np.pi, size=nt)
            radial = np.cos(phi)[:, None] * self.e1 + np.sin(phi)[:, None] * self.e2
            out[~is_s] = (self.torus_c + (R + r * np.cos(theta))[:, None] * radial
                          + (r * np.sin(theta))[:, None] * self.torus_n)
        return prim, out

    def surface_points(self, rng, k):
        """k points uniform on a uniformly chosen primitive, not inside any other one."""
        pts = []
        have = 0
        while have < k:
            prim, cand = self._surface_candidates(rng, int(1.3 * (k - have)) + 64)
            d = self.primitive_sdf(cand)
            d[np.arange(len(prim)), prim] = np.inf
            keep = d.min(axis=1) >= 0.0
            pts.append(cand[keep])
            have += int(keep.sum())
        return np.concatenate(pts)[:k]


def scene_batch(scene: Scene, n, seed=0, step=0, lo=-1.0, hi=1.0, jitter=0.01):
    """One training batch: n/2 uniform points in the box, n - n/2 jittered surface points.
    Draws from ``default_rng([seed, step])``.  Returns (q, d) as FP64 arrays whose q values
    are exactly representable in FP32; d is the scene SDF at those points."""
    rng = np.random.default_rng([seed, step])
    nu = n // 2
    qu = rng.uniform(lo, hi, size=(nu, 3))
    qs = scene.surface_points(rng, n - nu) + rng.normal(0.0, jitter, size=(n - nu, 3))
    q = np.concatenate([qu, qs]).astype(np.float32).astype(np.float64)
    return q, scene.sdf(q)


def scene3d_inputs(res=128, order=2, n=1 << 20, seed=0, std=0.05):
    """Coefficients ~ N(0, std) (drawn first), then one scene batch (seed, step 0)."""
    C = (order + 1) * (order + 2) * (order + 3) // 6
    coeffs, _ = normal_coeffs((res, res, res, C), std=std, seed=seed)
    scene = Scene(seed)
    q, d = scene_batch(scene, n, seed=seed, step=0)
    return coeffs, q, d, scene


def uniform_queries(n, dim=3, lo=-1.0, hi=1.0, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, dim)).astype(np.float32)


# ----------------------------------------------------------------------------- fitted grids
def scene_taylor_grid(scene: Scene, res, order, lo=-1.0, hi=1.0, device="cpu", eps=1e-4):
    """Coefficients of a grid 'fitted' to the scene by Taylor projection: at each vertex the
    scene SDF's value, gradient and Hessian (central differences in FP64, step eps), laid out
    [res_z, res_y, res_x, C] in graded-lex order.  Stands in for a trained grid where only
    the grid's size and contents' scale matter (serving).  Returns an FP32 torch tensor."""
    import torch

    c = torch.as_tensor(scene.centres, dtype=torch.float64, device=device)
    rad = torch.as_tensor(scene.radii, dtype=torch.float64, device=device)
    tc = torch.as_tensor(scene.torus_c, dtype=torch.float64, device=device)
    tn = torch.as_tensor(scene.torus_n, dtype=torch.float64, device=device)

    def sdf(p):
        sph = torch.linalg.norm(p[..., None, :] - c, dim=-1) - rad
        rel = p - tc
        along = rel @ tn
        radial = torch.linalg.norm(rel - along[..., None] * tn, dim=-1)
        tor = torch.sqrt((radial - scene.TORUS_R) ** 2 + along ** 2) - scene.TORUS_r
        return torch.minimum(sph.min(dim=-1).values, tor)

    nc = (order + 1) * (order + 2) * (order + 3) // 6
    out = torch.empty((res, res, res, nc), dtype=torch.float32, device=device)
    ax = torch.linspace(lo, hi, res, dtype=torch.float64, device=device)
    E = torch.eye(3, dtype=torch.float64, device=device) * eps
    for z in range(res):
        zz = torch.full((res, res), float(ax[z]), dtype=torch.float64, device=device)
        yy, xx = torch.meshgrid(ax, ax, indexing="ij")
        p = torch.stack([xx, yy, zz], dim=-1)
        f0 = sdf(p)
        cols = [f0]
        if order >= 1:
            fp = [sdf(p + E[a]) for a in range(3)]
            fm = [sdf(p - E[a]) for a in range(3)]
            cols += [(fp[a] - fm[a]) / (2 * eps) for a in range(3)]
        if order >= 2:
            for a in range(3):
                for b in range(a, 3):
                    if a == b:
                        cols.append((fp[a] - 2 * f0 + fm[a]) / eps ** 2)
                    else:
                        cols.append((sdf(p + E[a] + E[b]) - sdf(p + E[a] - E[b])
                                     - sdf(p - E[a] + E[b]) + sdf(p - E[a] - E[b])) / (4 * eps ** 2))
        out[z] = torch.stack(cols, dim=-1).to(torch.float32)
    return out


# ----------------------------------------------------------------------------- radiance rays
def camera_centres(n_cams=100, radius=4.0):
    """n_cams points spread over the sphere of the given radius (Fibonacci lattice)."""
    i = np.arange(n_cams) + 0.5
    z = 1.0 - 2.0 * i / n_cams
    phi = np.pi * (1.0 + 5.0 ** 0.5) * i
    rxy = np.sqrt(1.0 - z * z)
    return radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def box_segment(o, d, lo=-1.0, hi=1.0):
    """Entry and exit parameters (t_in <= t_out) of the rays o + t d (t >= 0) through the box
    [lo, hi]^3 (slab test); t_in == t_out for a ray that misses it."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    t_in = np.maximum(tmin, 0.0)
    return t_in, np.maximum(tmax, t_in)


def camera_rays(n_rays, seed=0, step=0, n_cams=100, radius=4.0, width=400, fov_deg=40.0, lo=-1.0, hi=1.0):
    """Origins [n_rays, 3] and unit directions [n_rays, 3] of random pixel rays of pinhole
    cameras on a sphere looking at the origin, drawn among the pixels whose ray crosses the
    box [lo, hi]^3 (a ray that misses it carries no samples).  Draws from
    ``default_rng([seed, step, 7])``."""
    rng = np.random.default_rng([seed, step, 7])
    out_o, out_d, have = [], [], 0
    while have < n_rays:
        o, d = _pixel_rays(rng, 2 * (n_rays - have) + 16, n_cams, radius, width, fov_deg)
        t_in, t_out = box_segment(o, d, lo, hi)
        hit = t_out > t_in
        out_o.append(o[hit])
        out_d.append(d[hit])
        have += int(hit.sum())
    return np.concatenate(out_o)[:n_rays], np.concatenate(out_d)[:n_rays]


def _pixel_rays(rng, n_rays, n_cams, radius, width, fov_deg):
    cams = camera_centres(n_cams, radius)
    cam = rng.integers(0, n_cams, size=n_rays)
    px = rng.integers(0, width, size=(n_rays, 2)) + 0.5
    o = cams[cam]
    fwd = -o / np.linalg.norm(o, axis=1, keepdims=True)
    up = np.where(np.abs(fwd[:, 2:3]) < 0.99, np.array([[0.0, 0.0, 1.0]]), np.array([[0.0, 1.0, 0.0]]))
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right, axis=1, keepdims=True)
    up = np.cross(right, fwd)
    half = np.tan(np.radians(fov_deg) / 2.0)
    u = (px[:, 0:1] / width * 2.0 - 1.0) * half
    v = (px[:, 1:2] / width * 2.0 - 1.0) * half
    d = fwd + u * right + v * up
    return o, d / np.linalg.norm(d, axis=1, keepdims=True)


def stratified_samples(o, d, n_samples, seed=0, step=0, lo=-1.0, hi=1.0):
    """Sample positions and spacings along rays (o + t d) inside the box [lo, hi]^3.

    The inside segment [t_in, t_out] comes from the slab test (empty for a ray that misses,
    which then gets zero spacings); it is cut into n_samples equal strata with one uniform
    position in each.  delta_i = t_{i+1} - t_i, and the last sample's runs to t_out.
    Returns q [n_rays * n_samples, 3] and delta [n_rays * n_samples], both exactly
    representable in FP32 (q ray-major, sample-minor)."""
    rng = np.random.default_rng([seed, step, 11])
    t_in, t_out = box_segment(o, d, lo, hi)  # a miss gives an empty segment
    n = o.shape[0]
    width = (t_out - t_in) / n_samples
    t = t_in[:, None] + (np.arange(n_samples)[None, :] + rng.uniform(size=(n, n_samples))) * width[:, None]
    t = t.astype(np.float32).astype(np.float64)
    nxt = np.concatenate([t[:, 1:], t_out[:, None]], axis=1)
    delta = np.maximum(nxt - t, 0.0).astype(np.float32).astype(np.float64)
    q = o[:, None, :] + t[:, :, None] * d[:, None, :]
    q = np.clip(q, lo, hi).astype(np.float32).astype(np.float64)
    return q.reshape(-1, 3), delta.reshape(-1)


class BlobVolume:
    """A seeded sum of anisotropic Gaussian blobs: density(x) = sum_k a_k exp(-|A_k (x - m_k)|^2 / 2)
    and colour(x) = the density-weighted mean of the blobs' RGB colours."""

    def __init__(self, seed=0, n_blobs=32):
        rng = np.random.default_rng([seed, 13])
        self.m = rng.uniform(-0.6, 0.6, size=(n_blobs, 3))
        scales = rng.uniform(4.0, 12.0, size=(n_blobs, 3))
        rot = np.linalg.qr(rng.normal(size=(n_blobs, 3, 3)))[0]
        self.A = scales[:, :, None] * np.transpose(rot, (0, 2, 1))
        self.a = rng.uniform(5.0, 30.0, size=n_blobs)
        self.rgb = rng.uniform(0.05, 0.95, size=(n_blobs, 3))

    def density_and_colour(self, x):
        x = np.asarray(x, dtype=np.float64)
        g = np.zeros((x.shape[0], len(self.a)))
        for k in range(len(self.a)):
            y = (x - self.m[k]) @ self.A[k].T
            g[:, k] = self.a[k] * np.exp(-0.5 * np.sum(y * y, axis=1))
        dens = g.sum(axis=1)
        col = (g @ self.rgb) / np.maximum(dens, 1e-12)[:, None]
        return dens, col

    def density_and_colour_torch(self, x):
        """The same density [n] and colour [n, 3] for a torch tensor x [n, 3] on its device,
        in FP64 (a faster generator of targets for long runs; the same values as the NumPy
        form up to rounding)."""
        import torch

        dev = x.device
        x = x.double()
        m = torch.tensor(self.m, dtype=torch.float64, device=dev)
        A = torch.tensor(self.A, dtype=torch.float64, device=dev)
        a = torch.tensor(self.a, dtype=torch.float64, device=dev)
        rgb = torch.tensor(self.rgb, dtype=torch.float64, device=dev)
        g = torch.empty((x.shape[0], len(self.a)), dtype=torch.float64, device=dev)
        for k in range(len(self.a)):
            y = (x - m[k]) @ A[k].T
            g[:, k] = a[k] * torch.exp(-0.5 * (y * y).sum(dim=1))
        dens = g.sum(dim=1)
        col = (g @ rgb) / dens.clamp_min(1e-12)[:, None]
        return dens, col
