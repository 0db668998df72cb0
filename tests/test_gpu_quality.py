"""SDF quality measures on the GPU against the FP64 oracle (oracle/quality.py): exact IoU
counts, the marching-cubes mesh triangle for triangle in the documented order (ragged
lattices, exact zeros, every corner sign pattern, every cell crossing, a 128^3 scene
lattice, a short output buffer, an empty level set), a grid's field on a lattice finer than the grid, the mesh of a
grid's field, the Chamfer distance in both norms, and the measures of fitted grids of every
order against the analytic scene."""
import numpy as np
import pytest
import torch

import oracle
from oracle import quality as qo
from paper_2402_14415_amd import quality, synth
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_VALUE, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


@pytest.mark.parametrize("n", [1_000_003, 1, 0])
def test_iou_counts_are_exact(n):
    rng = np.random.default_rng(n)
    f = rng.normal(size=n).astype(np.float32)
    d = (f + rng.normal(0, 0.5, size=n)).astype(np.float32)
    if n > 10:
        f[::97] = 0.0  # zero is outside
        d[::89] = -0.0
    got = quality.iou(_t(f), _t(d))
    inter, union = qo.iou_counts(f, d)
    assert got[1:] == (inter, union)
    assert got[0] == qo.iou(f, d)


def _lattice(fun, n, lo, hi):
    axes = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.transpose(fun(X, Y, Z), (2, 1, 0)).astype(np.float32)  # [z, y, x]


def _wavy(x, y, z):
    return np.sqrt(x * x + y * y + z * z) - 0.55 + 0.08 * np.sin(5 * x) * np.cos(4 * y) + 0.05 * np.sin(7 * z)


def _check_mesh(values, lo, hi, max_tris=None):
    tri, total = quality.mesh(_t(values), lo, hi, max_tris=max_tris)
    ref = qo.marching_cubes(values.astype(np.float64), lo, hi)
    torch.cuda.synchronize()
    assert total == len(ref)
    got = to_np(tri)
    k = len(got)
    assert k == (total if max_tris is None else min(total, max_tris))
    if k:
        scale = max(np.max(np.abs(hi)), np.max(np.abs(lo)))
        assert np.max(np.abs(got - ref[:k])) <= 2e-6 * scale
    return got


def test_mesh_matches_oracle_ragged_lattice():
    lo, hi = (-1.0, -0.9, -1.1), (1.0, 0.8, 1.2)
    V = _lattice(_wavy, (31, 37, 29), lo, hi)
    V[5, 6, :] = 0.0  # exact zeros (outside)
    _check_mesh(V, lo, hi)


def test_mesh_every_sign_pattern():
    """Random values padded with outside ones: all 256 corner patterns occur (ambiguous faces
    included); triangle for triangle against the oracle (whose meshes of such lattices are
    pinned closed and consistently oriented)."""
    rng = np.random.default_rng(8)
    V = np.ones((26, 25, 24), dtype=np.float32)
    V[1:-1, 1:-1, 1:-1] = (rng.normal(size=(24, 23, 22)) + 0.1).astype(np.float32)
    ins = V < 0
    pat = np.zeros((25, 24, 23), dtype=np.int64)
    for c in range(8):
        pat |= ins[(c >> 2) & 1: 25 + ((c >> 2) & 1), (c >> 1) & 1: 24 + ((c >> 1) & 1), c & 1: 23 + (c & 1)].astype(
            np.int64) << c
    assert len(np.unique(pat)) == 256
    lo, hi = (0.0, 0.0, 0.0), (23.0, 24.0, 25.0)
    _check_mesh(V, lo, hi)


def test_mesh_every_cell_crossing():
    """A sign checkerboard: every cell crosses the level set, so each block's list of crossing
    cells is full (and the last block's ragged); four triangles in every cell."""
    n = (45, 38, 41)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    V = np.where((i + j + k) % 2 == 0, 1.0, -1.0).astype(np.float32)
    V *= (1.0 + 0.25 * np.sin(0.7 * i + 0.3 * j - 0.5 * k)).astype(np.float32)
    lo, hi = (-1.0, -0.5, 0.0), (1.0, 1.5, 1.0)
    got = _check_mesh(V, lo, hi)
    assert len(got) == 4 * (n[0] - 1) * (n[1] - 1) * (n[2] - 1)


def test_mesh_full_size_scene_lattice():
    """The scene SDF on a 128^3 lattice over [-1, 1]^3."""
    scene = synth.Scene(0)
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    axes = np.linspace(-1, 1, 128)
    Z, Y, X = np.meshgrid(axes, axes, axes, indexing="ij")
    V = scene.sdf(np.stack([X, Y, Z], -1).reshape(-1, 3)).reshape(128, 128, 128).astype(np.float32)
    _check_mesh(V, lo, hi)


def test_mesh_short_buffer_and_empty_level_set():
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    V = _lattice(_wavy, (20, 21, 22), lo, hi)
    full = _check_mesh(V, lo, hi)
    part = _check_mesh(V, lo, hi, max_tris=len(full) // 3)
    assert np.array_equal(part, full[: len(part)])
    tri, total = quality.mesh(_t(np.ones((5, 6, 7))), lo, hi)
    assert total == 0 and tri.shape[0] == 0


@pytest.mark.parametrize("order,storage,s", [(2, "f32", 2), (1, "bf16", 3), (0, "f32", 1), (2, "f16", 4),
                                             (2, "f32", 6)])
def test_field_lattice_matches_oracle(order, storage, s):
    """The grid's field on the lattice s times finer than a ragged grid, against the C
    oracle's field at the same lattice (FP64 positions) on the storage-rounded coefficients
    (s <= 4: a thread per cell; s = 6: a thread per cell row pair and lattice layer)."""
    rng = np.random.default_rng(10 + order)
    res = (13, 11, 9)
    lo, hi = (-1.0, -0.5, 0.0), (1.0, 1.5, 0.75)
    nc = [1, 4, 10][order]
    C32 = rng.normal(0, 0.1, size=(9, 11, 13, nc)).astype(np.float32)
    g = TaylorGrid(3, res, order, lo, hi, storage=storage, coeffs=torch.from_numpy(C32), device=DEV)
    vals = quality.field_lattice(g, s)
    torch.cuda.synchronize()
    Cr = g.coeffs.float().cpu().double().numpy()  # the storage rounding (checked against NumPy elsewhere)
    n, pts = qo.field_lattice(geometry(g), Cr, s)
    assert vals.shape == (n[2], n[1], n[0])
    ref = oracle.forward(geometry(g), Cr, pts, want_grad=False)
    assert nerr(to_np(vals).reshape(-1), ref) <= TOL_VALUE
    # every s-th point is a grid vertex: the stored value
    np.testing.assert_allclose(to_np(vals)[::s, ::s, ::s], Cr[..., 0], rtol=0, atol=1e-6)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_mesh_of_a_grid_field_matches_oracle(order):
    """The mesh of a grid's field (tg_field_lattice then tg_mesh, s = 2) against the oracle's
    (FP64 field on the same lattice, inside decided in FP32): triangle for triangle in every
    cell whose corner signs both sides decide alike; the lattice points where they differ
    (|f| at rounding level) are counted and must be rare."""
    scene = synth.Scene(0)
    res = 24
    C32 = synth.scene_taylor_grid(scene, res, order).numpy()
    g = TaylorGrid(3, (res,) * 3, order, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    vals = quality.field_lattice(g, 2)
    tri, total = quality.mesh(vals, (-1.0,) * 3, (1.0,) * 3)
    torch.cuda.synchronize()
    geom = geometry(g)
    C = C32.astype(np.float64)
    n, pts = qo.field_lattice(geom, C, 2)
    f64 = oracle.forward(geom, C, pts, want_grad=False).reshape(n[2], n[1], n[0])
    ref, cells = qo.mesh_field(geom, C, 2, with_cells=True)
    gv = to_np(vals)
    differ = (gv < 0) != (f64.astype(np.float32) < 0)
    print(f"order {order}: {total} triangles, {int(differ.sum())} lattice points decided differently")
    assert differ.sum() <= 10
    # cells touching a differing point
    bad = np.zeros((n[2] - 1, n[1] - 1, n[0] - 1), dtype=bool)
    for z, y, x in np.argwhere(differ):
        bad[max(z - 1, 0): z + 1, max(y - 1, 0): y + 1, max(x - 1, 0): x + 1] = True
    bad_ids = np.nonzero(bad.reshape(-1))[0]
    got = to_np(tri)
    h = 2.0 / (n[0] - 1)
    gcell = np.floor((got.mean(axis=1) + 1.0) / h).astype(np.int64).clip(0, n[0] - 2)
    gid = gcell[:, 0] + (n[0] - 1) * (gcell[:, 1] + (n[1] - 1) * gcell[:, 2])
    keep_g = ~np.isin(gid, bad_ids)
    keep_r = ~np.isin(cells, bad_ids)
    assert keep_g.sum() == keep_r.sum()
    assert np.max(np.abs(got[keep_g] - ref[keep_r])) <= 1e-4 * h
    if not differ.any():
        assert total == len(ref)


@pytest.mark.parametrize("norm", [1, 2])
def test_chamfer_matches_oracle(norm):
    rng = np.random.default_rng(4)
    a = rng.normal(0, 0.3, size=(20_000, 3)).astype(np.float32)
    b = (rng.normal(0, 0.3, size=(15_000, 3)) + 0.02).astype(np.float32)
    got = quality.chamfer(_t(a), _t(b), norm=norm)
    ref = qo.chamfer(a.astype(np.float64), b.astype(np.float64), norm)
    assert abs(got[0] - ref) <= 1e-5 * ref
    assert abs(got[1] + got[2] - got[0]) <= 1e-12 * got[0]


@pytest.mark.parametrize("na,nb", [(3001, 200_003), (1, 70_000), (5, 1)])
def test_chamfer_lopsided_sets(na, nb):
    """A small source set against a large destination set, single points (a one-cell grid),
    and the arguments swapped."""
    rng = np.random.default_rng(na)
    a = rng.uniform(-1, 1, size=(na, 3)).astype(np.float32)
    b = rng.normal(0, 0.5, size=(nb, 3)).astype(np.float32)
    got = quality.chamfer(_t(a), _t(b))
    ref_ab = qo.chamfer(a.astype(np.float64), b.astype(np.float64), 1)
    assert abs(got[0] - ref_ab) <= 1e-5 * ref_ab
    swapped = quality.chamfer(_t(b), _t(a))
    assert abs(swapped[1] - got[2]) <= 1e-12 * got[2] and abs(swapped[2] - got[1]) <= 1e-12 * got[1]


@pytest.mark.parametrize("layout", ["far", "flat", "duplicates"])
def test_chamfer_bucket_grid_layouts(layout):
    """Layouts that test the bucket search's stopping bound: sets far apart (every search runs
    out of the other set's grid), a destination set of zero extent along z, and many copies of
    a few points (one crowded cell per copy), in both norms."""
    rng = np.random.default_rng(12)
    a = rng.normal(0, 0.4, size=(4000, 3))
    if layout == "far":
        b = rng.normal(0, 0.3, size=(6000, 3)) + np.array([6.0, -2.0, 1.0])
    elif layout == "flat":
        b = np.c_[rng.uniform(-1, 1, size=(6000, 2)), np.full(6000, 0.25)]
    else:
        b = np.repeat(rng.normal(0, 0.5, size=(3, 3)), 2000, axis=0)
    a, b = a.astype(np.float32), b.astype(np.float32)
    for norm in (1, 2):
        got = quality.chamfer(_t(a), _t(b), norm=norm)
        ref = qo.chamfer(a.astype(np.float64), b.astype(np.float64), norm)
        assert abs(got[0] - ref) <= 1e-5 * ref, (norm, got, ref)


def test_quality_of_fitted_grids_by_order():
    """Fit 48^3 grids of order 0, 1 and 2 to the scene for 150 steps each; IoU on 100k uniform
    points, and the Chamfer-L1 distance between the vertices of the mesh of each grid's field
    (s = 2) and 50k analytic surface points.  The fitted grids are the GPU's own results, so
    these are checked as properties: good fits (IoU > 0.85, Chamfer under 2 cells), meshes in
    the box with every triangle inside one lattice cell, and orders that differ."""
    scene = synth.Scene(0)
    res = 48
    h = 2.0 / (res - 1)
    rng = np.random.default_rng(6)
    pts = rng.uniform(-1, 1, size=(100_000, 3)).astype(np.float32)
    d = _t(scene.sdf(pts.astype(np.float64)).astype(np.float32))
    surf = _t(scene.surface_points(np.random.default_rng(7), 50_000).astype(np.float32))
    n = 1 << 17
    out = []
    for order in (0, 1, 2):
        g = TaylorGrid(3, (res,) * 3, order, (-1.0,) * 3, (1.0,) * 3, device=DEV)
        ws = g.workspace(n)
        for st in range(150):
            q, dd = synth.scene_batch(scene, n, seed=5, step=st)
            g.train_step(_t(q), _t(dd), ws, eik_weight=0.1, lr=1e-2)
        wq = g.workspace(len(pts))
        qt = _t(pts)
        g.sort(qt, wq)
        f, _ = g.forward(qt, wq, want_grad=False)
        iou = quality.iou(f, d)
        assert 0 < iou[1] <= iou[2] <= len(pts)
        vals = quality.field_lattice(g, 2)
        tri, total = quality.mesh(vals, (-1.0,) * 3, (1.0,) * 3)
        ch = quality.chamfer(tri.reshape(-1, 3).contiguous(), surf)
        print(f"order {order}: IoU {iou[0]:.4f}, triangles {total}, CD-L1 {ch[0]:.5f}")
        assert iou[0] > 0.85 and ch[0] < 2 * 3 * h and abs(ch[1] + ch[2] - ch[0]) <= 1e-12 * ch[0]
        p = to_np(tri)
        assert np.all(np.abs(p) <= 1.0 + 1e-6)
        span = np.max(np.linalg.norm(p[:, [0, 1, 2]] - p[:, [1, 2, 0]], axis=2))
        assert span <= np.sqrt(3) * h / 2 * (1 + 1e-5)
        out.append((iou[0], ch[0]))
    assert len({c for _, c in out}) == 3  # the three orders give three different meshes
