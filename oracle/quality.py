"""FP64 CPU oracle of the SDF quality measures that stand in for the paper's evaluation
(Sec. 4.1 reports IoU on uniform sample points and the Chamfer-L1 distance of the mesh that
marching cubes extracts from the learned field): IoU of the inside sets on sample points, the
zero-level-set mesh of a field sampled on a lattice by marching cubes, the lattice sampling of
a TaylorGrid's field, and the Chamfer distance between two point sets.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU-baseline leg use
it; the GPU library never imports, links or calls it, and it shares nothing with the GPU path.

* Inside: a point is inside a shape when its signed distance is < 0.
  IoU = |inside(f) and inside(d)| / |inside(f) or inside(d)| over the sample points (1 when
  both sets are empty).
* Zero-level-set mesh (marching cubes; the paper extracts its meshes with marching cubes and
  prints no variant).  A lattice cell has corners c = bx + 2 by + 4 bz; a corner is inside
  when its value is < 0.  Its 12 edges are numbered axis by axis (x, y, z), each axis's four
  in increasing order of their lower corner.  An edge whose ends differ in inside-ness carries
  one surface vertex, p_a + v_a / (v_a - v_b) (p_b - p_a) with a the lower end.  The polygons
  are built face by face, computed here directly for every cell (no case table):
    - every face of the cube is walked counterclockwise as seen from outside the cube, and
      each crossing where the walk enters the inside set is joined by a segment to the next
      crossing where it leaves it, directed from the entering to the leaving one (a face
      with two inside corners on a diagonal thus separates those corners: the ambiguity rule);
    - every crossing edge starts exactly one segment and ends exactly one, so the segments
      form closed loops; a loop starts at its smallest edge number, loops are taken in
      increasing order of that number, and a loop (e0, e1, ..., e_k-1) becomes the fan
      (e0, e_i, e_i+1), i = 1 .. k-2.
  The segment direction makes every triangle's normal (p1 - p0) x (p2 - p0) point from the
  inside to the outside, and neighbouring cells, which see a shared face's four corners
  alike, put the same segments on it: the mesh is closed wherever the inside set is.
  Triangles are listed cell by cell (x fastest), then in loop and fan order.
* The field of a grid is meshed on a lattice s times finer than the grid (vertices at
  lo + i (hi - lo) / (s (res - 1)), i = 0 .. s (res - 1)), sampled with the C oracle; the
  inside test takes the sampled values rounded to FP32 (the kernels' precision), positions
  use the FP64 values.
* Chamfer distance between point sets A and B (Sec. 4.1's CD-L1, computed with PyTorch3D's
  code in the paper): mean over A of the distance to the nearest point of B, plus the same
  from B to A, with the L1 norm |dx| + |dy| + |dz| (norm=1), or the Euclidean norm (norm=2).

Parity status: pinned by ``tests/test_oracle_quality.py`` (IoU by brute force and closed
cases; every one of the 256 corner sign cases against a brute-force count of crossing edges;
consistently oriented closed meshes of random lattices; the mesh of a plane exactly and of a
sphere's SDF against its surface, watertightness, enclosed volume and orientation; the lattice
sampling against the C oracle's values at the vertices; Chamfer by brute force and closed
forms); none is unpinned.
"""
from __future__ import annotations

import functools

import numpy as np


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


# the 12 cube edges: axis by axis, each axis's four in increasing order of the lower corner
EDGES = tuple((u, u | (1 << a)) for a in range(3) for u in range(8) if not (u >> a) & 1)
EDGE_OF = {e: k for k, e in enumerate(EDGES)}


def _face_walks():
    """The six faces' corners in counterclockwise order as seen from outside the cube."""
    walks = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3  # e_b x e_c = e_a
        for side in (0, 1):
            square = [(0, 0), (1, 0), (1, 1), (0, 1)]  # counterclockwise about +e_a
            if side == 0:  # the outward normal is -e_a: walk the other way round
                square = [square[0], square[3], square[2], square[1]]
            walks.append([(side << a) | (u << b) | (v << c) for u, v in square])
    return walks


FACE_WALKS = tuple(tuple(w) for w in _face_walks())


def cube_loops(inside):
    """Surface loops of one cube: inside [8] booleans.  Returns a list of loops, each a list
    of edge numbers, in the order the mesh uses them."""
    succ = {}
    for walk in FACE_WALKS:
        enter, leave = [], []  # crossings along the walk: (position, edge)
        for k in range(4):
            a, b = walk[k], walk[(k + 1) % 4]
            if inside[a] != inside[b]:
                e = EDGE_OF[(min(a, b), max(a, b))]
                (leave if inside[a] else enter).append((k, e))
        for k, e in enter:
            # the next crossing after position k (cyclically) where the walk leaves
            nxt = min(leave, key=lambda kl: (kl[0] - k) % 4)
            assert e not in succ
            succ[e] = nxt[1]
    loops, seen = [], set()
    for e0 in sorted(succ):
        if e0 in seen:
            continue
        loop, e = [], e0
        while e not in seen:
            seen.add(e)
            loop.append(e)
            e = succ[e]
        assert e == e0
        loops.append(loop)
    return loops


def cube_triangles(inside):
    """Triangles of one cube as triples of edge numbers (fan of every loop)."""
    return _case_triangles(sum(1 << c for c in range(8) if inside[c]))


@functools.lru_cache(maxsize=256)
def _case_triangles(case):
    tris = []
    for loop in cube_loops([(case >> c) & 1 == 1 for c in range(8)]):
        for i in range(1, len(loop) - 1):
            tris.append((loop[0], loop[i], loop[i + 1]))
    return tuple(tris)


def marching_cubes(values, lo, hi, decide=None, with_cells=False):
    """Zero-level-set triangles of a field sampled on a lattice: values [nz, ny, nx] at
    lo + i (hi - lo) / (n - 1).  The inside test reads ``decide`` (same shape; default the
    values themselves), positions the values.  Returns an array [T, 3, 3] (triangle, vertex,
    xyz), and with ``with_cells`` also each triangle's cell (linear index, x fastest)."""
    V = np.asarray(values, dtype=np.float64)
    D = V if decide is None else np.asarray(decide)
    nz, ny, nx = V.shape
    lo = np.asarray(lo, dtype=np.float64)
    h = (np.asarray(hi, dtype=np.float64) - lo) / (np.array([nx, ny, nz]) - 1)

    def corners(A):
        return np.stack([A[(c >> 2) & 1: nz - 1 + ((c >> 2) & 1), (c >> 1) & 1: ny - 1 + ((c >> 1) & 1),
                           c & 1: nx - 1 + (c & 1)] for c in range(8)], axis=-1)

    cv_all = corners(V)
    inside = corners(D) < 0
    mixed = np.argwhere(inside.any(axis=-1) & ~inside.all(axis=-1))  # rows (k, j, i), C order
    out, cells = [], []
    for k, j, i in mixed:
        cv = cv_all[k, j, i]
        base = np.array([i, j, k], dtype=np.float64)
        cp = [lo + (base + _corner_offset(c)) * h for c in range(8)]
        for tri in cube_triangles(inside[k, j, i]):
            pts = []
            for e in tri:
                a, b = EDGES[e]
                pts.append(cp[a] + (cv[a] / (cv[a] - cv[b])) * (cp[b] - cp[a]))
            out.append(np.array(pts))
            cells.append(i + (nx - 1) * (j + (ny - 1) * k))
    tris = np.array(out).reshape(-1, 3, 3)
    return (tris, np.array(cells, dtype=np.int64)) if with_cells else tris


def field_lattice(geom, coeffs, s):
    """The lattice s times finer than the grid: (n [3] points per axis, points [N, 3] in
    x-fastest order, FP64)."""
    n = [s * (r - 1) + 1 for r in geom.res]
    axes = [geom.lo[a] + np.arange(n[a]) * ((geom.hi[a] - geom.lo[a]) / (n[a] - 1)) for a in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return n, np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def mesh_field(geom, coeffs, s, with_cells=False):
    """Marching cubes of a TaylorGrid's field (the C oracle's FP64 forward) on the lattice s
    times finer than the grid; the inside test takes the values rounded to FP32."""
    import oracle

    n, pts = field_lattice(geom, coeffs, s)
    f = oracle.forward(geom, coeffs, pts, want_grad=False).reshape(n[2], n[1], n[0])
    return marching_cubes(f, geom.lo, geom.hi, decide=f.astype(np.float32), with_cells=with_cells)


def chamfer(a, b, norm=1):
    """Symmetric Chamfer distance: mean nearest distance A -> B plus B -> A, with the L1
    norm (norm=1) or the Euclidean norm (norm=2)."""
    from scipy.spatial import cKDTree

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    da, _ = cKDTree(b).query(a, p=norm)
    db, _ = cKDTree(a).query(b, p=norm)
    return float(da.mean() + db.mean())
