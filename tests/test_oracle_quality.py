"""Pins of the FP64 quality oracle (oracle/quality.py) against facts other than itself: IoU by
brute force and in closed cases; marching cubes over all 256 corner sign cases against a
brute-force count of the crossing edges, lone corners cut off facing out, closed and
consistently oriented meshes of random padded lattices (every ambiguous face included), the
mesh of a linear field (exact: every vertex on the plane, the area of the plane's section of
the box) and of a sphere's SDF (every vertex within O(h^2) of the sphere, closed, the enclosed
volume of the ball by the divergence theorem, outward orientation); the field lattice of a
grid (vertex property) and the mesh of a grid holding a sphere's Taylor series; Chamfer
distance in both norms by brute force and in closed cases."""
import math

import numpy as np
import pytest

from oracle import quality as qo


def test_iou_brute_force_and_closed_cases():
    rng = np.random.default_rng(0)
    f, d = rng.normal(size=500), rng.normal(size=500)
    inter = sum(1 for a, b in zip(f, d) if a < 0 and b < 0)
    union = sum(1 for a, b in zip(f, d) if a < 0 or b < 0)
    assert qo.iou_counts(f, d) == (inter, union)
    assert qo.iou(f, f) == 1.0
    assert qo.iou(np.abs(f), -np.abs(f) - 1) == 0.0
    assert qo.iou(np.ones(7), np.ones(7)) == 1.0  # both empty
    assert qo.iou_counts(np.zeros(3), -np.ones(3)) == (0, 3)  # 0 is not inside


def _lattice(fun, n, lo, hi):
    axes = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.transpose(fun(X, Y, Z), (2, 1, 0))  # -> [z, y, x]


def _area(tris):
    return 0.5 * np.linalg.norm(np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]), axis=1)


def _topological_mesh(V):
    """The oracle's triangles of a lattice as triples of global edge identities (axis, lower
    lattice point), in the mesh's order: the connectivity, free of geometric coincidences
    (a fan's diagonal may lie in a cube face, where a neighbour's diagonal can lie too)."""
    nz, ny, nx = V.shape
    tris = []
    for k in range(nz - 1):
        for j in range(ny - 1):
            for i in range(nx - 1):
                cv = [V[k + ((c >> 2) & 1), j + ((c >> 1) & 1), i + (c & 1)] for c in range(8)]
                for t in qo.cube_triangles([v < 0 for v in cv]):
                    ids = []
                    for e in t:
                        a, _ = qo.EDGES[e]
                        ids.append((e // 4, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1)))
                    tris.append(tuple(ids))
    return tris


def _closed_and_oriented(tris):
    """Every edge of the connectivity is used by exactly two triangles, in opposite
    directions."""
    from collections import Counter

    d = Counter((t[i], t[(i + 1) % 3]) for t in tris for i in range(3))
    return all(c == 1 for c in d.values()) and all(d[(b, a)] == 1 for (a, b) in d)


def test_every_sign_case_uses_exactly_the_crossing_edges():
    """All 256 inside/outside patterns of a cube's corners: the triangles use exactly the
    edges whose ends differ (counted by brute force), each crossing edge by at least one
    triangle; no triangle repeats an edge; there are (crossing edges - 2 x loops)
    triangles; a cube with every corner on one side has none."""
    pairs = [(a, b) for a in range(8) for b in range(a + 1, 8) if bin(a ^ b).count("1") == 1]
    assert sorted(pairs) == sorted(qo.EDGES)
    most = 0
    for case in range(256):
        inside = [(case >> c) & 1 == 1 for c in range(8)]
        crossing = {qo.EDGE_OF[(a, b)] for a, b in pairs if inside[a] != inside[b]}
        tris = qo.cube_triangles(inside)
        used = {e for t in tris for e in t}
        assert used == crossing, case
        assert all(len(set(t)) == 3 for t in tris)
        loops = qo.cube_loops(inside)
        assert sum(len(l) for l in loops) == len(crossing)
        assert len(tris) == len(crossing) - 2 * len(loops)
        most = max(most, len(tris))
    assert qo.cube_triangles([False] * 8) == () and qo.cube_triangles([True] * 8) == ()
    assert most <= 5


def test_one_inside_corner_is_cut_off_facing_out():
    """A lone inside corner gets one triangle across its three edges, its normal pointing
    away from the corner (from inside to outside), for each of the 8 corners and for the
    complement (a lone outside corner: the normal points towards it)."""
    for c in range(8):
        for lone_inside in (True, False):
            inside = [(k == c) == lone_inside for k in range(8)]
            V = np.where(np.array(inside), -1.0, 1.0)
            tris = qo.marching_cubes(V.reshape(2, 2, 2), (0, 0, 0), (1, 1, 1))
            assert tris.shape == (1, 3, 3)
            n = np.cross(tris[0, 1] - tris[0, 0], tris[0, 2] - tris[0, 0])
            corner = qo._corner_offset(c)
            away = tris[0].mean(axis=0) - corner
            assert np.dot(n, away) * (1 if lone_inside else -1) > 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_lattices_give_closed_consistently_oriented_meshes(seed):
    """Random corner values (every sign pattern, ambiguous faces included) inside a lattice
    padded with outside values: the inside set is enclosed, so the mesh must be closed and
    consistently oriented (every edge in exactly two triangles, in opposite directions), and
    its enclosed volume (divergence theorem) positive."""
    rng = np.random.default_rng(seed)
    V = np.ones((12, 11, 10))
    V[1:-1, 1:-1, 1:-1] = rng.normal(size=(10, 9, 8)) + 0.2
    tris = qo.marching_cubes(V, (0.0, 0.0, 0.0), (9.0, 10.0, 11.0))
    assert len(tris) > 100
    topo = _topological_mesh(V)
    assert len(topo) == len(tris) and _closed_and_oriented(topo)
    vol = np.sum(np.einsum("ij,ij->i", tris[:, 0], np.cross(tris[:, 1], tris[:, 2]))) / 6.0
    assert vol > 0
    # every vertex on a lattice edge, between its ends
    frac = tris.reshape(-1, 3) % 1.0
    on_edge = (np.sum((frac > 0) & (frac < 1), axis=1) <= 1)
    assert on_edge.all()


def test_mesh_of_a_plane_is_exact():
    """Linear interpolation along edges is exact for a linear field: every vertex lies on the
    plane z = 0.3 + 0.2 x, and the section of the unit box has area sqrt(1 + 0.2^2)."""
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    V = _lattice(lambda x, y, z: z - 0.3 - 0.2 * x, (5, 6, 7), lo, hi)
    tris = qo.marching_cubes(V, lo, hi)
    p = tris.reshape(-1, 3)
    assert np.max(np.abs(p[:, 2] - 0.3 - 0.2 * p[:, 0])) < 1e-14
    assert abs(_area(tris).sum() - math.sqrt(1 + 0.04)) < 1e-12
    # oriented from inside (below the plane) to outside: normals point up
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    assert np.all(n[_area(tris) > 1e-12][:, 2] > 0)


@pytest.mark.parametrize("n", [17, 33])
def test_mesh_of_a_sphere(n):
    r = 0.6
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    V = _lattice(lambda x, y, z: np.sqrt(x * x + y * y + z * z) - r, (n, n, n), lo, hi)
    tris = qo.marching_cubes(V, lo, hi)
    h = 2.0 / (n - 1)
    p = tris.reshape(-1, 3)
    # interpolating |x| - r linearly along an edge of length h errs by at most about
    # h^2 / (8 r) (the distance's curvature across the edge is at most 1 / r)
    assert np.max(np.abs(np.linalg.norm(p, axis=1) - r)) < 1.25 * h * h / (8 * r)
    assert _closed_and_oriented(_topological_mesh(V))
    # enclosed volume by the divergence theorem (positive: normals point outward)
    vol = np.sum(np.einsum("ij,ij->i", tris[:, 0], np.cross(tris[:, 1], tris[:, 2]))) / 6.0
    exact = 4.0 / 3.0 * math.pi * r ** 3
    assert 0 < vol and abs(vol - exact) < 3.0 * h * h * exact


def test_field_lattice_and_mesh_of_a_grid():
    """The lattice s times finer than a grid holds the grid's vertices at every s-th point,
    where the sampled field equals the stored values (vertex property of Eq. 1-4); a grid
    storing the Taylor series of a sphere's SDF (|x| - r: value, gradient, Hessian) meshes to
    a closed surface near the sphere, closer with the order."""
    import oracle

    res, r = 10, 0.55  # no vertex at the centre, where the distance has no gradient
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    errs = []
    for order in (0, 1, 2):
        geom = oracle.Geometry(3, (res,) * 3, order, lo, hi)
        ax = np.linspace(-1, 1, res)
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        P = np.stack([X, Y, Z], -1)
        rho = np.linalg.norm(P, axis=-1)
        g = P / rho[..., None]
        cols = [rho - r]
        if order >= 1:
            cols += [g[..., 0], g[..., 1], g[..., 2]]
        if order >= 2:
            for a in range(3):
                for b in range(a, 3):
                    cols.append(((a == b) - g[..., a] * g[..., b]) / rho)
        C = np.stack(cols, -1)
        n, pts = qo.field_lattice(geom, C, 2)
        assert n == [2 * res - 1] * 3
        f = oracle.forward(geom, C, pts, want_grad=False).reshape(n[2], n[1], n[0])
        np.testing.assert_allclose(f[::2, ::2, ::2], C[..., 0], rtol=0, atol=1e-14)
        tris = qo.mesh_field(geom, C, 2)
        assert _closed_and_oriented(_topological_mesh(f.astype(np.float32)))
        errs.append(np.max(np.abs(np.linalg.norm(tris.reshape(-1, 3), axis=1) - r)))
    assert errs[2] < errs[1] < errs[0]


def test_chamfer_brute_force_and_closed_form():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(60, 3)), rng.normal(size=(45, 3))
    for norm, dist in ((2, np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)),
                       (1, np.abs(a[:, None, :] - b[None, :, :]).sum(axis=2))):
        assert abs(qo.chamfer(a, b, norm) - (dist.min(axis=1).mean() + dist.min(axis=0).mean())) < 1e-12
    # two copies of a point set offset by delta (smaller than half the spacing): 2 delta in
    # either norm along an axis; 2 (|dx| + |dy|) in L1 along a diagonal
    g = np.stack(np.meshgrid(np.arange(4.0), np.arange(4.0), np.arange(4.0), indexing="ij"), -1).reshape(-1, 3)
    assert abs(qo.chamfer(g, g + np.array([0.0, 0.0, 0.3]), 1) - 0.6) < 1e-12
    assert abs(qo.chamfer(g, g + np.array([0.0, 0.0, 0.3]), 2) - 0.6) < 1e-12
    assert abs(qo.chamfer(g, g + np.array([0.1, 0.2, 0.0]), 1) - 0.6) < 1e-12
    assert abs(qo.chamfer(g, g + np.array([0.3, 0.4, 0.0]), 2) - 1.0) < 1e-12
    assert qo.chamfer(g, g) == 0.0


def test_planted_mistakes_in_marching_cubes_are_caught(monkeypatch):
    """Mistakes planted in the marching cubes oracle fail its pins: walking the faces the
    wrong way round turns the normals inward (negative enclosed volume); joining each entering
    crossing to the last leaving one instead of the next breaks the mesh's closure on
    ambiguous faces."""
    rng = np.random.default_rng(5)
    V = np.ones((9, 9, 9))
    V[1:-1, 1:-1, 1:-1] = rng.normal(size=(7, 7, 7)) + 0.2

    def volume(tris):
        return np.sum(np.einsum("ij,ij->i", tris[:, 0], np.cross(tris[:, 1], tris[:, 2]))) / 6.0

    good = qo.marching_cubes(V, (0.0,) * 3, (8.0,) * 3)
    assert volume(good) > 0 and _closed_and_oriented(_topological_mesh(V))
    try:
        monkeypatch.setattr(qo, "FACE_WALKS", tuple(tuple(reversed(w)) for w in qo.FACE_WALKS))
        qo._case_triangles.cache_clear()
        assert volume(qo.marching_cubes(V, (0.0,) * 3, (8.0,) * 3)) < 0
        monkeypatch.undo()

        def loops_far(inside):
            succ = {}
            for walk in qo.FACE_WALKS:
                enter, leave = [], []
                for k in range(4):
                    a, b = walk[k], walk[(k + 1) % 4]
                    if inside[a] != inside[b]:
                        e = qo.EDGE_OF[(min(a, b), max(a, b))]
                        (leave if inside[a] else enter).append((k, e))
                for k, e in enter:
                    succ[e] = max(leave, key=lambda kl: (kl[0] - k) % 4)[1]  # planted: the last
            loops, seen = [], set()
            for e0 in sorted(succ):
                if e0 not in seen:
                    loop, e = [], e0
                    while e not in seen:
                        seen.add(e)
                        loop.append(e)
                        e = succ[e]
                    loops.append(loop)
            return loops

        monkeypatch.setattr(qo, "cube_loops", loops_far)
        qo._case_triangles.cache_clear()
        assert not _closed_and_oriented(_topological_mesh(V))
    finally:
        monkeypatch.undo()
        qo._case_triangles.cache_clear()
