"""Pins of the FP64 quality oracle (oracle/quality.py) against facts other than itself: IoU by
brute force and in closed cases; the zero-level-set mesh of a linear field (exact: every
vertex on the plane, the area of the plane's section of the box) and of a sphere's SDF (every
vertex within O(h^2) of the sphere, watertight, the enclosed volume of the ball by the
divergence theorem, outward orientation); Chamfer distance by brute force and in a closed
case."""
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


def test_mesh_of_a_plane_is_exact():
    """Linear interpolation along edges is exact for a linear field: every vertex lies on the
    plane z = 0.3 + 0.2 x, and the section of the unit box has area sqrt(1 + 0.2^2)."""
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    V = _lattice(lambda x, y, z: z - 0.3 - 0.2 * x, (5, 6, 7), lo, hi)
    tris = qo.marching_tetrahedra(V, lo, hi)
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
    tris = qo.marching_tetrahedra(V, lo, hi)
    h = 2.0 / (n - 1)
    p = tris.reshape(-1, 3)
    # interpolating |x| - r linearly along an edge of length L <= sqrt(3) h errs by at most
    # about L^2 / (8 r) (the distance's curvature across the edge is at most 1 / r)
    assert np.max(np.abs(np.linalg.norm(p, axis=1) - r)) < 1.25 * 3 * h * h / (8 * r)
    # watertight: every edge of the mesh is shared by exactly two triangles
    key = lambda a: tuple(np.round(a / h * 1e6).astype(np.int64))
    count = {}
    for t in tris:
        for i in range(3):
            e = tuple(sorted((key(t[i]), key(t[(i + 1) % 3]))))
            if e[0] != e[1]:
                count[e] = count.get(e, 0) + 1
    assert set(count.values()) == {2}
    # enclosed volume by the divergence theorem (positive: normals point outward)
    vol = np.sum(np.einsum("ij,ij->i", tris[:, 0], np.cross(tris[:, 1], tris[:, 2]))) / 6.0
    exact = 4.0 / 3.0 * math.pi * r ** 3
    assert 0 < vol and abs(vol - exact) < 3.0 * h * h * exact


def test_chamfer_brute_force_and_closed_form():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(60, 3)), rng.normal(size=(45, 3))
    dist = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
    assert abs(qo.chamfer(a, b) - (dist.min(axis=1).mean() + dist.min(axis=0).mean())) < 1e-12
    # two copies of a point set offset by delta (smaller than half the spacing): 2 delta
    g = np.stack(np.meshgrid(np.arange(4.0), np.arange(4.0), np.arange(4.0), indexing="ij"), -1).reshape(-1, 3)
    assert abs(qo.chamfer(g, g + np.array([0.0, 0.0, 0.3])) - 0.6) < 1e-12
    assert qo.chamfer(g, g) == 0.0
