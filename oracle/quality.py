"""FP64 CPU oracle of the SDF quality measures that stand in for the paper's evaluation
(Sec. 4.1 reports IoU and Chamfer distance of reconstructed shapes): IoU of the inside sets
on sample points, a zero-level-set mesh of a sampled field, and the Chamfer distance between
two point sets.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU-baseline leg use
it; the GPU library never imports, links or calls it, and it shares nothing with the GPU path.

* Inside: a point is inside a shape when its signed distance is < 0.
  IoU = |inside(f) and inside(d)| / |inside(f) or inside(d)| over the sample points (1 when
  both sets are empty).
* Zero-level-set mesh (marching tetrahedra): the lattice cell with corner (i, j, k) is split
  into 6 tetrahedra around its main diagonal, corner 0 = (0,0,0) to corner 7 = (1,1,1) (corner
  index bx + 2 by + 4 bz), tetrahedron t being (0, P_t[0], P_t[1], 7) with the corner pairs
  P = ((1,3), (3,2), (2,6), (6,4), (4,5), (5,1)).  In a tetrahedron with corner values v, the
  corners with v < 0 are inside; with one corner apart from the other three (inside or
  outside) the surface is one triangle across the 3 edges leaving it, with two on each side a
  quadrilateral across the 4 edges between the sides, split into two triangles.  A surface
  point on edge (a, b) is a + v_a / (v_a - v_b) (b - a).  Triangles are listed cell by cell (x
  fastest), tetrahedron by tetrahedron; a lone corner's triangle has its edges in the order of
  the other corners, a quadrilateral with inside corners i0 < i1 and outside o0 < o1 is
  (i0 o0, i0 o1, i1 o1, i1 o0), split along its first diagonal; each triangle is oriented so
  that its normal (p1 - p0) x (p2 - p0) points from the inside corners to the outside ones.
* Chamfer distance between point sets A and B: mean over A of the distance to the nearest
  point of B, plus the same from B to A.

Parity status: pinned by ``tests/test_oracle_quality.py`` (IoU by brute force and closed
cases; the mesh of a plane and of a sphere's SDF against their exact surfaces, watertightness,
the enclosed volume, orientation; Chamfer by brute force and closed forms); none is unpinned.
"""
from __future__ import annotations

import numpy as np

# tetrahedra of a cell: corner 0, a pair, corner 7
TET_PAIRS = ((1, 3), (3, 2), (2, 6), (6, 4), (4, 5), (5, 1))


def iou_counts(f, d):
    """(|A and B|, |A or B|) of the inside sets A = {f < 0}, B = {d < 0}."""
    a = np.asarray(f) < 0
    b = np.asarray(d) < 0
    return int(np.sum(a & b)), int(np.sum(a | b))


def iou(f, d):
    inter, union = iou_counts(f, d)
    return 1.0 if union == 0 else inter / union


def _corner_offset(c):
    return np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1], dtype=np.float64)


def _edge_point(pa, pb, va, vb):
    return pa + (va / (va - vb)) * (pb - pa)


def tet_triangles(p, v, pc):
    """Triangles of the zero level set in one tetrahedron: p [4, 3] corner positions, v [4]
    values, pc [4, 3] the corners' offsets in the cell (0 or 1).  Returns a list of (3, 3)
    arrays.  Orientation is decided on the triangle through the edge midpoints, in the cell's
    own coordinates (exact), and is the same for the true triangle: moving the points along
    their edges never flips it."""
    inside = [i for i in range(4) if v[i] < 0]
    outside = [i for i in range(4) if not v[i] < 0]
    edges = []  # each triangle as three (a, b) corner pairs
    if len(inside) in (1, 3):
        lone = inside[0] if len(inside) == 1 else outside[0]
        others = [i for i in range(4) if i != lone]
        edges.append([(lone, o) for o in others])
    elif len(inside) == 2:
        i0, i1 = inside
        o0, o1 = outside
        quad = [(i0, o0), (i0, o1), (i1, o1), (i1, o0)]  # cyclic around the quadrilateral
        edges.append([quad[0], quad[1], quad[2]])
        edges.append([quad[0], quad[2], quad[3]])
    tris = []
    if edges:
        pc = np.asarray(pc, dtype=np.float64)
        cin = np.mean([pc[i] for i in inside], axis=0)
        cout = np.mean([pc[i] for i in outside], axis=0)
        for tri in edges:
            m = [0.5 * (pc[a] + pc[b]) for a, b in tri]
            n = np.cross(m[1] - m[0], m[2] - m[0])
            if not np.dot(n, cout - cin) > 0:
                tri = [tri[0], tri[2], tri[1]]
            tris.append(np.array([_edge_point(p[a], p[b], v[a], v[b]) for a, b in tri]))
    return tris


def marching_tetrahedra(values, lo, hi):
    """Zero-level-set triangles of a field sampled on a lattice: values [nz, ny, nx] at
    lo + i (hi - lo) / (n - 1).  Returns an array [T, 3, 3] (triangle, vertex, xyz)."""
    V = np.asarray(values, dtype=np.float64)
    nz, ny, nx = V.shape
    lo = np.asarray(lo, dtype=np.float64)
    h = (np.asarray(hi, dtype=np.float64) - lo) / (np.array([nx, ny, nz]) - 1)
    # corner values of every cell [nz-1, ny-1, nx-1, 8]; only cells with corners on both
    # sides produce triangles, visited in cell order (x fastest)
    corners = np.stack([V[(c >> 2) & 1: nz - 1 + ((c >> 2) & 1), (c >> 1) & 1: ny - 1 + ((c >> 1) & 1),
                          c & 1: nx - 1 + (c & 1)] for c in range(8)], axis=-1)
    inside = corners < 0
    mixed = np.argwhere(inside.any(axis=-1) & ~inside.all(axis=-1))  # rows (k, j, i), C order
    out = []
    for k, j, i in mixed:
        cv = corners[k, j, i]
        base = np.array([i, j, k], dtype=np.float64)
        cp = np.array([lo + (base + _corner_offset(c)) * h for c in range(8)])
        for a, b in TET_PAIRS:
            idx = [0, a, b, 7]
            out.extend(tet_triangles(cp[idx], cv[idx], [_corner_offset(c) for c in idx]))
    return np.array(out).reshape(-1, 3, 3)


def chamfer(a, b):
    """Symmetric Chamfer distance (mean nearest distance A -> B plus B -> A)."""
    from scipy.spatial import cKDTree

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    da, _ = cKDTree(b).query(a)
    db, _ = cKDTree(a).query(b)
    return float(da.mean() + db.mean())
