"""GPU edge cases: empty and single-query inputs, single-cell grids, queries exactly on
vertices and faces, non-finite queries, brick-boundary cells (a query feeding 8 vertex
bricks) and the maximal sort fan-out."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, nerr_cols, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _grid(dim, res, order, lo, hi, rng, storage="f32"):
    nc = [1, 4, 10][order] if dim == 3 else [1, 3, 6][order]
    C32 = rng.normal(0, 0.1, size=tuple(reversed(res)) + (nc,)).astype(np.float32)
    return TaylorGrid(dim, res, order, lo, hi, storage=storage, coeffs=torch.from_numpy(C32), device=DEV), \
        C32.astype(np.float64)


def _fwd_bwd(grid, q64, gf64, gg64):
    q = torch.tensor(q64, dtype=torch.float32, device=DEV).reshape(-1, grid.dim)
    ws = grid.workspace(q.shape[0])
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    gf = torch.tensor(gf64, dtype=torch.float32, device=DEV)
    gg = torch.tensor(gg64, dtype=torch.float32, device=DEV).reshape(-1, grid.dim)
    dq = grid.backward(q, ws, gf, gg, want_dq=True)
    torch.cuda.synchronize()
    return to_np(f), to_np(g), to_np(grid.grad), to_np(dq)


def _compare(grid, C, q64, gf, gg, res_f, res_g, res_dC, res_dq, strict=False):
    """Against the oracle; under the rule for faces unless strict (the same cell on both
    sides for every query).  Returns the number of queries on a face."""
    ref_f, ref_g = oracle.forward(geometry(grid), C, q64)
    ref_dC, ref_dq = oracle.backward(geometry(grid), C, q64, gf, gg, want_dq=True)
    assert nerr(res_f, ref_f) <= TOL_VALUE
    if strict:
        assert nerr_cols(res_g, ref_g) <= TOL_GRAD
        assert nerr(res_dC.reshape(-1), ref_dC.reshape(-1)) <= TOL_GRAD
        assert nerr_cols(res_dq, ref_dq) <= TOL_GRAD
        return 0
    rule = FaceRule(geometry(grid), C, q64)
    assert rule.grad_err(res_g, ref_g) <= TOL_GRAD
    assert rule.dC_err(res_dC, ref_dC, gf, gg) <= TOL_GRAD
    assert rule.dq_err(res_dq, ref_dq, gf, gg) <= TOL_GRAD
    return rule.count


def test_empty_queries():
    rng = np.random.default_rng(0)
    grid, _ = _grid(3, (20, 20, 20), 2, (-1,) * 3, (1,) * 3, rng)
    grid.grad.fill_(7.0)
    q = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    ws = grid.workspace(0)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    grid.backward(q, ws, torch.empty(0, device=DEV), torch.empty((0, 3), device=DEV), accumulate=True)
    torch.cuda.synchronize()
    assert f.numel() == 0 and torch.all(grid.grad == 7.0)
    grid.backward(q, ws, torch.empty(0, device=DEV), torch.empty((0, 3), device=DEV))  # overwrite: zeros
    torch.cuda.synchronize()
    assert torch.count_nonzero(grid.grad) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_single_query_and_single_cell_grid(dim):
    rng = np.random.default_rng(1)
    res = (2,) * dim
    grid, C = _grid(dim, res, 2, (-1,) * dim, (1,) * dim, rng)
    for n in (1, 7, 1000):
        q64 = rng.uniform(-1.3, 1.3, size=(n, dim)).astype(np.float32).astype(np.float64)
        gf = rng.normal(size=n).astype(np.float32).astype(np.float64)
        gg = rng.normal(size=(n, dim)).astype(np.float32).astype(np.float64)
        _compare(grid, C, q64, gf, gg, *_fwd_bwd(grid, q64, gf, gg))


@pytest.mark.parametrize("dim", [2, 3])
def test_queries_on_vertices_faces_and_corners(dim):
    """On a grid with spacing 1/4 every vertex coordinate is exact in FP32 and FP64, so both
    sides pick the same cell (the high face uses the last cell)."""
    rng = np.random.default_rng(2)
    res = (5,) * dim
    grid, C = _grid(dim, res, 2, (0.0,) * dim, (1.0,) * dim, rng)
    ticks = np.linspace(0, 1, 5)
    pts = np.stack(np.meshgrid(*[ticks] * dim, indexing="ij"), -1).reshape(-1, dim)
    faces = rng.uniform(0, 1, size=(400, dim))
    faces[np.arange(400), rng.integers(0, dim, 400)] = rng.choice(ticks, 400)
    q64 = np.concatenate([pts, faces, np.ones((3, dim)), np.zeros((3, dim))]).astype(np.float32).astype(np.float64)
    n = len(q64)
    gf = rng.normal(size=n).astype(np.float32).astype(np.float64)
    gg = rng.normal(size=(n, dim)).astype(np.float32).astype(np.float64)
    res_f, res_g, res_dC, res_dq = _fwd_bwd(grid, q64, gf, gg)
    _compare(grid, C, q64, gf, gg, res_f, res_g, res_dC, res_dq, strict=True)
    # vertex property: f equals the stored value at every vertex
    flat = C.reshape(-1, grid.C)
    idx = np.rint(pts * 4).astype(int)
    lin = idx[:, 0] + 5 * idx[:, 1] + (25 * idx[:, 2] if dim == 3 else 0)
    np.testing.assert_allclose(res_f[: len(pts)], flat[lin, 0], rtol=0, atol=1e-6)


def test_queries_on_faces_take_either_cell():
    """The rule for faces: the gradient of the field jumps across an interior face, so a
    query on one may take either adjacent cell.  Queries are put exactly on interior vertex
    planes (exact in FP32 on this grid), one float step to either side, and 1e-30 to either
    side of the plane through 0, where the FP32 two-float location and the FP64 oracle can
    pick different cells (1 + 1e-30 rounds to 1 in FP64).  They are counted, f is compared
    directly (it is continuous), and grad f, dq and dC under the rule."""
    rng = np.random.default_rng(6)
    res = (33, 17, 65)  # h = 1/16, 1/8, 1/32 on [-1, 1]: every vertex plane is exact
    grid, C = _grid(3, res, 2, (-1.0,) * 3, (1.0,) * 3, rng)
    n = 2000
    q = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
    axis = rng.integers(0, 3, n)
    for a in range(3):
        sel = axis == a
        h = np.float32(2.0 / (res[a] - 1))
        plane = (np.float32(-1) + rng.integers(1, res[a] - 1, sel.sum()).astype(np.float32) * h).astype(np.float32)
        kind = rng.integers(0, 5, sel.sum())
        v = plane.copy()
        v[kind == 1] = np.nextafter(plane[kind == 1], np.float32(np.inf))
        v[kind == 2] = np.nextafter(plane[kind == 2], np.float32(-np.inf))
        v[kind == 3] = np.float32(1e-30)
        v[kind == 4] = np.float32(-1e-30)
        q[sel, a] = v
    q64 = q.astype(np.float64)
    gf = rng.normal(size=n).astype(np.float32).astype(np.float64) / n
    gg = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64) / n
    count = _compare(grid, C, q64, gf, gg, *_fwd_bwd(grid, q64, gf, gg))
    print(f"{count} of {n} queries on a face")
    assert count >= n // 2


def test_brick_boundary_cells_fan_out():
    """Queries in cells on the high layer of a brick along every axis feed eight vertex
    bricks; put every query there (the sort's worst case)."""
    rng = np.random.default_rng(3)
    res = (33, 33, 33)  # cells 0..31: bricks of 8 cells, boundary cells 7, 15, 23, 31
    grid, C = _grid(3, res, 2, (0.0,) * 3, (32.0,) * 3, rng)
    n = 20000
    cells = rng.choice([7, 15, 23], size=(n, 3))
    q64 = (cells + rng.uniform(0.01, 0.99, size=(n, 3))).astype(np.float32).astype(np.float64)
    gf = rng.normal(size=n).astype(np.float32).astype(np.float64)
    gg = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    _compare(grid, C, q64, gf, gg, *_fwd_bwd(grid, q64, gf, gg))


def test_nonfinite_queries_do_not_disturb_others():
    rng = np.random.default_rng(4)
    grid, C = _grid(3, (16, 16, 16), 2, (-1,) * 3, (1,) * 3, rng)
    n = 4000
    q64 = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32).astype(np.float64)
    bad = q64.copy()
    bad[::97, 0] = np.nan
    bad[1::97, 1] = np.inf
    bad[2::97, 2] = -np.inf
    q = torch.tensor(bad, dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    torch.cuda.synchronize()
    good = np.all(np.isfinite(bad), axis=1)
    ref_f, ref_g = oracle.forward(geometry(grid), C, q64[good])
    assert nerr(to_np(f)[good], ref_f) <= TOL_VALUE
    assert nerr_cols(to_np(g)[good], ref_g) <= TOL_GRAD


def test_many_queries_in_one_cell():
    rng = np.random.default_rng(5)
    grid, C = _grid(3, (24, 24, 24), 2, (-1,) * 3, (1,) * 3, rng)
    n = 30000
    q64 = (0.1 + rng.uniform(0, 0.05, size=(n, 3))).astype(np.float32).astype(np.float64)
    gf = rng.normal(size=n).astype(np.float32).astype(np.float64) / n
    gg = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64) / n
    _compare(grid, C, q64, gf, gg, *_fwd_bwd(grid, q64, gf, gg))


def test_sort_table_forgets_old_workspaces():
    """The library remembers the sort generation of the 1024 most recently sorted workspaces;
    a workspace that drops out reads as holding no sort (TG_ERR_STATE), never as current."""
    from paper_2402_14415_amd._lib import TaylorGridError

    rng = np.random.default_rng(7)
    grid, _ = _grid(3, (9, 9, 9), 1, (-1,) * 3, (1,) * 3, rng)
    other, _ = _grid(3, (9, 9, 9), 1, (-1,) * 3, (1,) * 3, rng)
    q = torch.zeros((1, 3), dtype=torch.float32, device=DEV)
    wss = [grid.workspace(1) for _ in range(1030)]
    grid.sort(q, wss[0])
    grid.forward(q, wss[0])  # current
    for w in wss[1:]:
        other.sort(q, w)
    with pytest.raises(TaylorGridError) as e:
        grid.forward(q, wss[0])
    assert e.value.status == 5
    grid.sort(q, wss[0])  # sorting again makes it current
    grid.forward(q, wss[0])
    torch.cuda.synchronize()
