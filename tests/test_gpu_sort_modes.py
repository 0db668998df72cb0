"""The three bucketing paths, each against the oracle through a forward and an adjoint.

The sort keeps one counter per bucket key (2 per vertex brick) in LDS: 32-bit counters up to
40704 keys, packed 16-bit counters up to 81920 keys, and global atomic counters beyond.  The
grids below fall in each range (bricks of 8^3 cells in 3D, 16^2 in 2D):
  200^3 -> 25^3 bricks -> 31250 keys (32-bit),  264^3 -> 33^3 -> 71874 keys (16-bit),
  4000^2 -> 250^2 bricks -> 125000 keys (atomic)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("dim,res,order,keys", [
    (3, (200, 200, 200), 1, 31250),
    (3, (264, 264, 264), 0, 71874),
    (2, (4000, 4000), 1, 125000),
])
def test_sort_paths_against_oracle(dim, res, order, keys):
    bricks = int(np.prod([-(-r // (8 if dim == 3 else 16)) for r in res]))
    assert 2 * bricks == keys
    rng = np.random.default_rng(keys)
    lo, hi = (-1.0,) * dim, (1.0,) * dim
    nc = [[1, 3, 6], [1, 4, 10]][dim - 2][order]
    C32 = rng.normal(0, 0.05, size=tuple(reversed(res)) + (nc,)).astype(np.float32)
    C = C32.astype(np.float64)
    grid = TaylorGrid(dim, res, order, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    n = 300000
    q64 = rng.uniform(-1.02, 1.02, size=(n, dim))
    q64[: n // 10] = 0.3 + 0.01 * rng.uniform(size=(n // 10, dim))  # a crowded brick
    q64 = q64.astype(np.float32).astype(np.float64)
    gf = (rng.normal(size=n) / n).astype(np.float32).astype(np.float64)
    gg = (rng.normal(size=(n, dim)) / n).astype(np.float32).astype(np.float64)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    print(f"dim {dim} res {res} keys {keys}", flush=True)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    grid.backward(q, ws, torch.tensor(gf, dtype=torch.float32, device=DEV),
                  torch.tensor(gg, dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    geom = geometry(grid)
    ref_f, ref_g = oracle.forward(geom, C, q64)
    rule = FaceRule(geom, C, q64)
    assert nerr(to_np(f), ref_f) <= TOL_VALUE
    assert rule.grad_err(to_np(g), ref_g) <= TOL_GRAD
    ref_dC, _ = oracle.backward(geom, C, q64, gf, gg)
    e = rule.dC_err(to_np(grid.grad), ref_dC, gf, gg)
    print(f"  dC err {e:.2e} ({rule.count} queries on a face)", flush=True)
    assert e <= TOL_GRAD
