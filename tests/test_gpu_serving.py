"""Serving form on the GPU: tg_query against the FP64 oracle, and the continuous-batching
server (a request's result is the same alone and in any mix, the footprint budget holds)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd.grid import TaylorGrid, query
from paper_2402_14415_amd.serving import Server, run_trace
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _grid(dim, res, order, storage, seed, lo=-1.0, hi=1.0):
    g = TaylorGrid(dim, res, order, (lo,) * dim, (hi,) * dim, storage=storage, device=DEV, optimizer=False)
    rng = np.random.default_rng(seed)
    g.master.copy_(torch.tensor(rng.normal(0, 0.05, size=g.shape), dtype=torch.float32))
    g.sync_storage()
    return g


def _points(dim, n, seed, lo=-1.0, hi=1.0, outside=0.1):
    rng = np.random.default_rng(seed)
    q = rng.uniform(lo, hi, size=(n, dim))
    k = int(n * outside)
    if k:
        q[:k] = rng.uniform(lo - 0.3, hi + 0.3, size=(k, dim))
    return q.astype(np.float32).astype(np.float64)


def _oracle_sdf_normal(grid, q64):
    C64 = grid.coeffs.float().cpu().double().numpy()
    f, g = oracle.forward(geometry(grid), C64, q64)
    nrm = np.linalg.norm(g, axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        normal = np.where(nrm > 0, g / nrm, 0.0)
    return f, normal, nrm[:, 0]


@pytest.mark.parametrize("dim,order,storage", [(3, 2, "f32"), (3, 2, "bf16"), (3, 2, "f16"), (3, 1, "bf16"),
                                               (3, 0, "f32"), (2, 2, "f32"), (2, 1, "f16")])
def test_query_matches_oracle(dim, order, storage):
    res_list = [(9, 12, 7)[:dim], (17,) * dim, (5, 33, 6)[:dim]]
    grids = [_grid(dim, r, order, storage, seed=10 + k) for k, r in enumerate(res_list)]
    sizes = [0, 1, 255, 257, 3000, 777]
    reqs, refs = [], []
    for k, n in enumerate(sizes):
        gi = k % len(grids)
        q64 = _points(dim, n, 100 + k)
        q = torch.tensor(q64, dtype=torch.float32, device=DEV).reshape(n, dim)
        sdf = torch.full((n,), float("nan"), device=DEV)
        normal = torch.full((n, dim), float("nan"), device=DEV)
        reqs.append((gi, q, sdf, normal))
        refs.append((gi, q64.reshape(n, dim)))
    query(grids, reqs)
    torch.cuda.synchronize()
    for (gi, q, sdf, normal), (_, q64) in zip(reqs, refs):
        if q64.shape[0] == 0:
            continue
        f_ref, n_ref, gnorm = _oracle_sdf_normal(grids[gi], q64)
        ef = nerr(to_np(sdf), f_ref)
        ok = gnorm > 1e-3 * gnorm.max()  # the normal is ill-conditioned where the gradient vanishes
        ok[FaceRule(geometry(grids[gi]), None, q64).idx] = False  # either side's normal on a face
        en = float(np.max(np.abs(to_np(normal)[ok] - n_ref[ok]))) if ok.any() else 0.0
        print(f"grid {gi} n={q64.shape[0]}: f err {ef:.2e}, normal err {en:.2e}")
        assert ef <= TOL_VALUE
        assert en <= TOL_GRAD


def test_query_zero_gradient_gives_zero_normal():
    g = _grid(3, (6, 6, 6), 2, "f32", seed=0)
    g.master.zero_()  # zero field: value and gradient are exactly zero in any precision
    q = torch.tensor(_points(3, 500, 1), dtype=torch.float32, device=DEV)
    sdf = torch.full((500,), float("nan"), device=DEV)
    normal = torch.full((500, 3), float("nan"), device=DEV)
    query([g], [(0, q, sdf, normal)])
    torch.cuda.synchronize()
    assert torch.all(sdf == 0)
    assert torch.all(normal == 0)  # not NaN


def _serving_setup(seed=0):
    grids = [_grid(3, (17, 23, 19), 2, "bf16", seed), _grid(3, (33,) * 3, 1, "bf16", seed + 1),
             _grid(3, (12,) * 3, 2, "f32", seed + 2), _grid(3, (40, 9, 21), 2, "f16", seed + 3)]
    rng = np.random.default_rng(seed)
    sizes = [1, 5000, 20000, 3, 4096, 4097, 70000, 12, 999, 30000, 2, 15000]
    reqs = []
    for k, n in enumerate(sizes):
        q = torch.tensor(_points(3, n, 200 + k), dtype=torch.float32, device=DEV)
        reqs.append((int(rng.integers(0, len(grids))), q))
    return grids, reqs


def _alone(grids, gi, q):
    sdf = torch.empty(q.shape[0], device=DEV)
    normal = torch.empty((q.shape[0], 3), device=DEV)
    query(grids, [(gi, q, sdf, normal)])
    torch.cuda.synchronize()
    return sdf, normal


def test_serving_results_same_alone_and_in_mix():
    grids, reqs = _serving_setup()
    alone = [_alone(grids, gi, q) for gi, q in reqs]
    srv = Server(grids, budget_bytes=1 << 30, streams=2, depth=3, chunk_points=4096, max_reqs=5)
    handles = [srv.submit(gi, q) for gi, q in reqs]
    srv.drain()
    torch.cuda.synchronize()
    assert srv.launches > len(reqs) // 5
    for h, (s, nm) in zip(handles, alone):
        assert h.done
        assert torch.equal(h.sdf, s) and torch.equal(h.normal, nm), f"request {h.rid} differs in the mix"


def test_serving_budget_and_poisson_trace():
    grids, reqs = _serving_setup(seed=1)
    alone = [_alone(grids, gi, q) for gi, q in reqs]
    budget = 28 * 80000  # room for a few requests at a time
    srv = Server(grids, budget_bytes=budget, streams=2, depth=4, chunk_points=16384)
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(2e-4, size=len(reqs)))
    out = run_trace(srv, [(float(t), gi, q) for t, (gi, q) in zip(arrivals, reqs)])
    torch.cuda.synchronize()
    print(out)
    assert out["requests"] == len(reqs)
    assert out["peak_inflight_bytes"] <= budget
    assert srv.used_bytes == 0
    by_rid = {r.rid: r for r in srv.completed}
    for k, (s, nm) in enumerate(alone):
        r = by_rid[k]
        assert torch.equal(r.sdf, s) and torch.equal(r.normal, nm)


def test_query_splits_beyond_launch_limits():
    """More requests and grids than one launch holds: the call splits them, results equal
    the single-request calls."""
    grids = [_grid(3, (6 + k, 7, 8), 1 + k % 2, "bf16", seed=k) for k in range(18)]
    reqs, alone = [], []
    for k in range(40):
        gi = (k * 7) % len(grids)
        q = torch.tensor(_points(3, 50 + 13 * k, 300 + k), dtype=torch.float32, device=DEV)
        alone.append(_alone(grids, gi, q))
        reqs.append((gi, q, torch.empty(q.shape[0], device=DEV), torch.empty((q.shape[0], 3), device=DEV)))
    query(grids, reqs)
    torch.cuda.synchronize()
    for (gi, q, s, nm), (s0, n0) in zip(reqs, alone):
        assert torch.equal(s, s0) and torch.equal(nm, n0)
