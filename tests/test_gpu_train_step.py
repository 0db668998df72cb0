"""The production training step (tg_train_step: sort, forward with the loss in its epilogue,
adjoint with Adam in the same pass, crowded bricks taken whole or merged) against the FP64 oracle's forward,
loss, adjoint and Adam, at the full SDF-fitting size and on crowded bricks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _step_against_oracle(g, C, m0, v0, q, d, step, eik=0.1, lr=1e-2):
    """One tg_train_step on the grid (whose master, moments hold C, m0, v0) and the oracle's
    step on the same FP32-rounded inputs; checks loss, master, moments and sum(dC^2).
    Targets d must keep |f - d| clear of rounding level (the sign of the residual decides
    the L1 gradient)."""
    n = len(q)
    ws = g.workspace(n)
    gn = torch.zeros(1, dtype=torch.float64, device=DEV)
    loss = g.train_step(torch.tensor(q, dtype=torch.float32, device=DEV),
                        torch.tensor(d, dtype=torch.float32, device=DEV), ws, eik_weight=eik, lr=lr, step=step,
                        grad_norm_sq=gn)
    torch.cuda.synchronize()
    geom = geometry(g)
    f, grad = oracle.forward(geom, C, q)
    ref, gf, gg = oracle.sdf_loss(f, grad, d, eik)
    dC = oracle.backward(geom, C, q, gf, gg)[0]
    th, mm, vv, ss = oracle.adam(C.reshape(-1), m0.reshape(-1), v0.reshape(-1), dC.reshape(-1), lr, step=step)
    rule = FaceRule(geom, C, q)
    e = {"loss": nerr(to_np(loss), ref), "master": nerr(to_np(g.master).reshape(-1), th),
         "m": nerr(to_np(g.adam_m).reshape(-1), mm), "v": nerr(to_np(g.adam_v).reshape(-1), vv),
         "grad_norm": abs(gn.item() - ss) / ss}
    print({k: f"{x:.2e}" for k, x in e.items()}, f"({rule.count} queries on a face)")
    assert rule.count == 0  # a query on a face would need the face rule's slack on dC
    assert e["loss"] <= TOL_VALUE and e["master"] <= TOL_VALUE
    # the moments carry the adjoint's FP32 error: m linearly, v through g^2 (twice the relative error)
    assert e["m"] <= TOL_GRAD and e["v"] <= 2 * TOL_GRAD and e["grad_norm"] <= 2 * TOL_GRAD


def _away_from_residual_zero(geom, C, q, d, gap=1e-4):
    """Targets moved so that |f - d| >= gap for the oracle's f (inputs built from the oracle
    alone)."""
    f = oracle.forward(geom, C, q, want_grad=False)
    r = f - d
    near = np.abs(r) < gap
    d = d.copy()
    d[near] = f[near] - np.where(r[near] >= 0, 2 * gap, -2 * gap)
    return d.astype(np.float32).astype(np.float64)


def test_train_step_full_size_against_oracle():
    """128^3 vertices, K=2, 2^20 scene queries (half on the surfaces: crowded bricks above one
    adjoint work item, staged whole by their first item), L1 + 0.1 eikonal, Adam with established moments at
    step 5, every one of the 21 M coefficients compared."""
    C64, q, d, _ = synth.scene3d_inputs(res=128, order=2, n=1 << 20, seed=0)
    C32 = C64.astype(np.float32)
    del C64
    C = C32.astype(np.float64)
    rng = np.random.default_rng(55)
    m0 = rng.normal(0, 1e-5, size=C.shape).astype(np.float32)
    v0 = rng.uniform(1e-10, 1e-9, size=C.shape).astype(np.float32)
    g = TaylorGrid(3, (128,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    g.adam_m.copy_(torch.from_numpy(m0))
    g.adam_v.copy_(torch.from_numpy(v0))
    d = _away_from_residual_zero(geometry(g), C, q, d)
    _step_against_oracle(g, C, m0.astype(np.float64), v0.astype(np.float64), q, d, step=5)


@pytest.mark.parametrize("order,crowd", [(1, 48_000), (2, 48_000), (2, 5_000)])
def test_train_step_split_bricks_against_oracle(order, crowd):
    """`crowd` queries packed into a few cells of one brick: its records exceed one adjoint
    work item several times over.  With 48,000 the brick is above the size the adjoint with
    Adam stages in one workgroup, so its items store partial sums and the one that finishes
    last adds them and applies Adam; with 5,000 the brick's first item stages all of its
    records."""
    rng = np.random.default_rng(56 + order + crowd)
    res = (24, 20, 22)
    nc = [1, 4, 10][order]
    C32 = rng.normal(0, 0.05, size=(22, 20, 24, nc)).astype(np.float32)
    C = C32.astype(np.float64)
    n = 80_000
    q = rng.uniform(-1, 1, size=(n, 3))
    k = crowd
    q[:k] = -0.3 + rng.uniform(0, 0.15, size=(k, 3))  # about 2 cells per axis of one brick
    q = q.astype(np.float32).astype(np.float64)
    m0 = rng.normal(0, 1e-4, size=C.shape).astype(np.float32)
    v0 = rng.uniform(1e-9, 1e-8, size=C.shape).astype(np.float32)
    g = TaylorGrid(3, res, order, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    g.adam_m.copy_(torch.from_numpy(m0))
    g.adam_v.copy_(torch.from_numpy(v0))
    d = _away_from_residual_zero(geometry(g), C, q, rng.normal(0, 0.1, size=n).astype(np.float32).astype(np.float64))
    _step_against_oracle(g, C, m0.astype(np.float64), v0.astype(np.float64), q, d, step=3)


@pytest.mark.parametrize("crowd", [5_000, 30_000])
def test_train_step_split_bricks_2d_against_oracle(crowd):
    """The same in 2D (bricks of 16 x 16 cells): a brick of about `crowd` records is staged whole
    by its first item (5,000) or merged by its last item (30,000)."""
    rng = np.random.default_rng(60 + crowd)
    res = (50, 40)
    C32 = rng.normal(0, 0.05, size=(40, 50, 6)).astype(np.float32)
    C = C32.astype(np.float64)
    n = 60_000
    q = rng.uniform(-1, 1, size=(n, 2))
    q[:crowd] = 0.2 + rng.uniform(0, 0.05, size=(crowd, 2))
    q = q.astype(np.float32).astype(np.float64)
    m0 = rng.normal(0, 1e-4, size=C.shape).astype(np.float32)
    v0 = rng.uniform(1e-9, 1e-8, size=C.shape).astype(np.float32)
    g = TaylorGrid(2, res, 2, (-1.0,) * 2, (1.0,) * 2, coeffs=torch.from_numpy(C32), device=DEV)
    g.adam_m.copy_(torch.from_numpy(m0))
    g.adam_v.copy_(torch.from_numpy(v0))
    d = _away_from_residual_zero(geometry(g), C, q, rng.normal(0, 0.1, size=n).astype(np.float32).astype(np.float64))
    _step_against_oracle(g, C, m0.astype(np.float64), v0.astype(np.float64), q, d, step=4)


def test_presorted_step_and_pipelined_loop_match_the_plain_step():
    """tg_train_step_sorted on a sort written beforehand gives tg_train_step's result, and a
    loop that sorts the next batch on a second stream (a twin handle, a second workspace)
    while the current step runs ends where the plain loop ends.  Without a sort of the batch
    in the workspace the presorted step refuses (TG_ERR_STATE)."""
    from paper_2402_14415_amd._lib import TaylorGridError

    rng = np.random.default_rng(57)
    res = (40, 36, 33)
    C32 = rng.normal(0, 0.05, size=(33, 36, 40, 10)).astype(np.float32)
    scene = synth.Scene(0)
    batches = []
    for b in range(5):
        q, d = synth.scene_batch(scene, 1 << 16, seed=7, step=b)
        batches.append((torch.tensor(q, dtype=torch.float32, device=DEV), torch.tensor(d, dtype=torch.float32, device=DEV)))
    a = TaylorGrid(3, res, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    b = TaylorGrid(3, res, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    # established moments: from zero moments Adam's first steps move every coefficient by about
    # lr whatever the size of its gradient, which turns rounding-level differences of tiny
    # gradients into visible ones
    m0 = torch.from_numpy(rng.normal(0, 1e-5, size=C32.shape).astype(np.float32))
    v0 = torch.from_numpy(rng.uniform(1e-9, 1e-8, size=C32.shape).astype(np.float32))
    for g_ in (a, b):
        g_.adam_m.copy_(m0)
        g_.adam_v.copy_(v0)
    wa = a.workspace(1 << 16)
    with pytest.raises(TaylorGridError) as e:
        a.train_step(*batches[0], wa, step=10, presorted=True)
    assert e.value.status == 5
    for k, (q, d) in enumerate(batches):
        a.train_step(q, d, wa, step=k + 10)
    # the pipelined loop on b
    twin = b.twin()
    hs, wss = (b, twin), (b.workspace(1 << 16), b.workspace(1 << 16))
    side = torch.cuda.Stream(DEV)
    main = torch.cuda.current_stream(DEV)
    sorted_ev = [torch.cuda.Event(), torch.cuda.Event()]
    done_ev = [torch.cuda.Event(), torch.cuda.Event()]
    hs[0].sort(batches[0][0], wss[0])
    sorted_ev[0].record(main)
    for k in range(len(batches)):
        h, h1 = k % 2, (k + 1) % 2
        if k + 1 < len(batches):
            with torch.cuda.stream(side):
                if k > 0:
                    side.wait_event(done_ev[h1])
                hs[h1].sort(batches[k + 1][0], wss[h1])
                sorted_ev[h1].record(side)
        main.wait_event(sorted_ev[h])
        hs[h].train_step(*batches[k], wss[h], step=k + 10, presorted=True)
        done_ev[h].record(main)
    torch.cuda.synchronize()
    # the same arithmetic; two sorts of one batch may order a bucket's records differently,
    # so the FP32 sums agree to rounding: the tolerances of the comparisons with the oracle
    for name, tol in (("master", TOL_VALUE), ("adam_m", TOL_GRAD), ("adam_v", 2 * TOL_GRAD)):
        e = nerr(to_np(getattr(b, name)).reshape(-1), to_np(getattr(a, name)).reshape(-1))
        print(name, f"{e:.2e}")
        assert e <= tol
