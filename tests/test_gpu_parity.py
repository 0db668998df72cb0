"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs.  See parity_util for the comparison rule and tolerances."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, nerr_cols, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(grid, q64, gf64=None, gg64=None, want_dq=False, accumulate=False):
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(q.shape[0])
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    out = {"f": f, "g": g, "q": q, "ws": ws}
    if gf64 is not None or gg64 is not None:
        gf = None if gf64 is None else torch.tensor(gf64, dtype=torch.float32, device=DEV)
        gg = None if gg64 is None else torch.tensor(gg64, dtype=torch.float32, device=DEV)
        out["dq"] = grid.backward(q, ws, gf, gg, want_dq=want_dq, accumulate=accumulate)
    torch.cuda.synchronize()
    return out


def _check_forward(grid, C64, q64, out, tol_f=TOL_VALUE, tol_g=TOL_GRAD):
    ref_f, ref_g = oracle.forward(geometry(grid), C64, q64)
    rule = FaceRule(geometry(grid), C64, q64)
    ef = nerr(to_np(out["f"]), ref_f)  # f is continuous across faces: no exemption
    eg = rule.grad_err(to_np(out["g"]), ref_g)
    print(f"forward err f={ef:.2e} grad={eg:.2e} ({rule.count} queries on a face)")
    assert ef <= tol_f and eg <= tol_g
    return ref_f, ref_g


def _mixed_queries(dim, lo, hi, n, rng):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    k_out = n // 10
    k_hot = n // 10
    qu = rng.uniform(lo, hi, size=(n - k_out - k_hot, dim))
    qo = rng.uniform(lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo), size=(k_out, dim))  # many outside: clamped
    centre = lo + (hi - lo) * 0.37
    qh = centre + rng.uniform(0, 1e-3, size=(k_hot, dim)) * (hi - lo)  # one hot cell: contention
    return np.concatenate([qu, qo, qh])


# ----------------------------------------------------------------------------- config 0
def test_config0_disc2d_forward_l1_backward():
    """2D, 64x64 vertices, K=2 (6 coefficients), N(0,0.05) init, 65,536 uniform queries,
    disc SDF target, one forward + L1 backward (seed 0)."""
    C64, q64, d64 = synth.disc2d_inputs(res=64, order=2, n=65536, seed=0)
    C32 = C64.astype(np.float32)
    C = C32.astype(np.float64)
    grid = TaylorGrid(2, (64, 64), 2, (0.0, 0.0), (1.0, 1.0), coeffs=torch.from_numpy(C32), device=DEV)
    out = _run(grid, q64)
    ref_f, _ = _check_forward(grid, C, q64, out)

    d = torch.tensor(d64, dtype=torch.float32, device=DEV)
    loss, gf, _ = sdf_loss(out["f"], None, d, 0.0, out["ws"])
    ref_loss, ref_gf, _ = oracle.sdf_loss(ref_f, None, d.double().cpu().numpy(), 0.0)
    assert abs(float(loss[0]) - ref_loss[0]) <= TOL_VALUE * abs(ref_loss[0])
    # sign(f - d) may differ only where the residual is at FP32 rounding level
    r = ref_f - d.double().cpu().numpy()
    mism = to_np(gf) != ref_gf
    assert np.all(np.abs(r[mism]) < 1e-5)

    # the adjoint: both sides take the oracle's upstream gradient (rounded to FP32) as input
    gf32 = ref_gf.astype(np.float32)
    grid.backward(out["q"], out["ws"], torch.tensor(gf32, device=DEV), None)
    ref_dC, _ = oracle.backward(geometry(grid), C, q64, gf32.astype(np.float64), None)
    e = FaceRule(geometry(grid), C, q64).dC_err(to_np(grid.grad), ref_dC, gf32, None)
    print(f"dC err {e:.2e}")
    assert e <= TOL_GRAD


# ----------------------------------------------------------------------------- 3D, all orders
@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("res", [(37, 37, 37), (17, 30, 9)])
def test_forward_backward_3d(order, res):
    """Several bricks with ragged edges, clamped queries outside the box, and one hot cell."""
    rng = np.random.default_rng(100 + order)
    lo, hi = (-1.0, -0.5, 0.25), (1.0, 1.5, 0.75)
    nc = tg_nc = (order + 1) * (order + 2) * (order + 3) // 6
    C32 = rng.normal(0, 0.05, size=(res[2], res[1], res[0], nc)).astype(np.float32)
    C = C32.astype(np.float64)
    grid = TaylorGrid(3, res, order, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    n = 60000
    q64 = _mixed_queries(3, lo, hi, n, rng).astype(np.float32).astype(np.float64)
    gf = rng.normal(size=n) / n
    gg = rng.normal(size=(n, 3)) / n
    out = _run(grid, q64, gf.astype(np.float32).astype(np.float64), gg.astype(np.float32).astype(np.float64),
               want_dq=True)
    _check_forward(grid, C, q64, out)
    gf32 = gf.astype(np.float32).astype(np.float64)
    gg32 = gg.astype(np.float32).astype(np.float64)
    ref_dC, ref_dq = oracle.backward(geometry(grid), C, q64, gf32, gg32, want_dq=True)
    rule = FaceRule(geometry(grid), C, q64)
    e_dc = rule.dC_err(to_np(grid.grad), ref_dC, gf32, gg32)
    e_dq = rule.dq_err(to_np(out["dq"]), ref_dq, gf32, gg32)
    print(f"order {order} res {res}: dC err {e_dc:.2e} dq err {e_dq:.2e}")
    assert e_dc <= TOL_GRAD and e_dq <= TOL_GRAD
    assert tg_nc == grid.C


@pytest.mark.parametrize("order", [0, 1, 2])
def test_forward_backward_2d(order):
    rng = np.random.default_rng(200 + order)
    res, lo, hi = (45, 38), (-2.0, 0.0), (2.0, 3.0)
    nc = (order + 1) * (order + 2) // 2
    C32 = rng.normal(0, 0.05, size=(res[1], res[0], nc)).astype(np.float32)
    C = C32.astype(np.float64)
    grid = TaylorGrid(2, res, order, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    n = 50000
    q64 = _mixed_queries(2, lo, hi, n, rng).astype(np.float32).astype(np.float64)
    gf = (rng.normal(size=n) / n).astype(np.float32).astype(np.float64)
    gg = (rng.normal(size=(n, 2)) / n).astype(np.float32).astype(np.float64)
    out = _run(grid, q64, gf, gg, want_dq=True)
    _check_forward(grid, C, q64, out)
    ref_dC, ref_dq = oracle.backward(geometry(grid), C, q64, gf, gg, want_dq=True)
    rule = FaceRule(geometry(grid), C, q64)
    assert rule.dC_err(to_np(grid.grad), ref_dC, gf, gg) <= TOL_GRAD
    assert rule.dq_err(to_np(out["dq"]), ref_dq, gf, gg) <= TOL_GRAD


def test_backward_accumulates():
    rng = np.random.default_rng(7)
    res = (20, 20, 20)
    C32 = rng.normal(0, 0.05, size=(20, 20, 20, 10)).astype(np.float32)
    grid = TaylorGrid(3, res, 2, (-1,) * 3, (1,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    n = 5000
    q64 = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32).astype(np.float64)
    gf = (rng.normal(size=n) / n).astype(np.float32).astype(np.float64)
    out = _run(grid, q64, gf, None)
    first = grid.grad.clone()
    grid.backward(out["q"], out["ws"], torch.tensor(gf, dtype=torch.float32, device=DEV), None, accumulate=True)
    torch.cuda.synchronize()
    assert nerr(to_np(grid.grad), 2 * to_np(first)) <= 1e-6
    # overwrite mode resets it (the in-brick merge order may differ, so compare to rounding)
    grid.backward(out["q"], out["ws"], torch.tensor(gf, dtype=torch.float32, device=DEV), None)
    torch.cuda.synchronize()
    assert nerr(to_np(grid.grad), to_np(first)) <= 1e-6


# ----------------------------------------------------------------------------- config 1 shape
def test_config1_full_size_forward_backward():
    """128^3 vertices, K=2, FP32, 2^20 queries (half uniform, half near the sphere/torus
    surface), L1 + 0.1 eikonal upstream gradients computed by the loss kernel."""
    C64, q64, d64, _ = synth.scene3d_inputs(res=128, order=2, n=1 << 20, seed=0)
    C32 = C64.astype(np.float32)
    del C64
    C = C32.astype(np.float64)
    grid = TaylorGrid(3, (128,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    out = _run(grid, q64)
    ref_f, ref_g = _check_forward(grid, C, q64, out)

    d = torch.tensor(d64, dtype=torch.float32, device=DEV)
    loss, gf, gg = sdf_loss(out["f"], out["g"], d, 0.1, out["ws"])
    # the loss kernel on the GPU's forward against the oracle's loss on the oracle's forward
    d32 = d64.astype(np.float32).astype(np.float64)
    ref_loss, ref_gf, ref_gg = oracle.sdf_loss(ref_f, ref_g, d32, 0.1)
    np.testing.assert_allclose(to_np(loss), ref_loss, rtol=TOL_VALUE)
    # sign(f - d) may differ only where the residual is at FP32 rounding level
    mism = to_np(gf) != ref_gf
    assert np.all(np.abs(ref_f - d32)[mism] < 1e-5)
    # g_grad follows grad f, which may take either side's value for a query on a face
    keep = np.ones(len(q64), dtype=bool)
    keep[FaceRule(geometry(grid), C, q64).idx] = False
    assert nerr_cols(to_np(gg)[keep], ref_gg[keep]) <= TOL_GRAD
    # the adjoint: both sides take the oracle's upstream gradients (rounded to FP32) as input
    gf32, gg32 = ref_gf.astype(np.float32), ref_gg.astype(np.float32)
    grid.backward(out["q"], out["ws"], torch.tensor(gf32, device=DEV), torch.tensor(gg32, device=DEV))
    torch.cuda.synchronize()
    ref_dC, _ = oracle.backward(geometry(grid), C, q64, gf32.astype(np.float64), gg32.astype(np.float64))
    e = FaceRule(geometry(grid), C, q64).dC_err(to_np(grid.grad), ref_dC, gf32, gg32)
    print(f"config1 dC err {e:.2e}")
    assert e <= TOL_GRAD


# ----------------------------------------------------------------------------- loss
def test_sdf_loss_kernel():
    rng = np.random.default_rng(3)
    n = 100003  # ragged
    f = rng.normal(size=n).astype(np.float32)
    d = f.copy()
    d[: n // 2] = rng.normal(size=n // 2).astype(np.float32)  # half have r == 0 exactly
    g = rng.normal(size=(n, 3)).astype(np.float32)
    g[:100] = 0.0  # zero-norm gradients
    ft, dt, gt = (torch.tensor(x, device=DEV) for x in (f, d, g))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    loss, gf, gg = sdf_loss(ft, gt, dt, 0.1, ws)
    ref_loss, ref_gf, ref_gg = oracle.sdf_loss(f.astype(np.float64), g.astype(np.float64), d.astype(np.float64), 0.1)
    np.testing.assert_allclose(to_np(loss), ref_loss, rtol=1e-6)
    np.testing.assert_array_equal(np.sign(to_np(gf)), np.sign(ref_gf))
    assert nerr(to_np(gf), ref_gf) <= 1e-6
    assert nerr_cols(to_np(gg), ref_gg) <= TOL_GRAD
    assert np.all(to_np(gg)[:100] == 0.0)
    # empty input
    e = torch.empty(0, device=DEV)
    loss0, _, _ = sdf_loss(e, torch.empty((0, 3), device=DEV), e, 0.1, ws)
    assert np.all(to_np(loss0) == 0.0)


# ----------------------------------------------------------------------------- Adam
@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_adam_step(storage):
    rng = np.random.default_rng(5)
    res = (13, 11, 7)  # 1001 vertices * 10 = 10010 coefficients: not a multiple of 4
    shape = (7, 11, 13, 10)
    th = rng.normal(0, 0.5, size=shape).astype(np.float32)
    grid = TaylorGrid(3, res, 2, (-1,) * 3, (1,) * 3, storage=storage, coeffs=torch.from_numpy(th), device=DEV)
    m = rng.normal(0, 0.01, size=shape).astype(np.float32)
    v = rng.uniform(0, 1e-3, size=shape).astype(np.float32)
    grid.adam_m.copy_(torch.from_numpy(m))
    grid.adam_v.copy_(torch.from_numpy(v))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    gns = torch.zeros(1, dtype=torch.float64, device=DEV)
    th64, m64, v64 = th.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in (1, 2, 3):
        g = (rng.normal(size=shape) * 10.0 ** rng.integers(-6, 1)).astype(np.float32)
        grid.grad.copy_(torch.from_numpy(g))
        grid.adam_step(ws, lr=1e-2, weight_decay=0.01 if step == 2 else 0.0, grad_norm_sq=gns, zero_grad=True)
        torch.cuda.synchronize()
        th64, m64, v64, ss = oracle.adam(th64, m64, v64, g.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8,
                                         0.01 if step == 2 else 0.0, step)
        assert nerr(to_np(grid.master), th64) <= TOL_VALUE
        assert nerr(to_np(grid.adam_m), m64) <= TOL_VALUE
        assert nerr(to_np(grid.adam_v), v64) <= TOL_VALUE
        assert abs(float(gns[0]) - ss) <= 1e-12 * ss
        assert torch.count_nonzero(grid.grad) == 0
        if storage != "f32":
            expect = grid.master.clamp(-65504, 65504).to(grid.coeffs.dtype) if storage == "f16" else \
                grid.master.to(torch.bfloat16)
            assert torch.equal(grid.coeffs.view(torch.int16), expect.view(torch.int16))
        # keep the oracle on the GPU's own state so errors do not compound
        th64 = to_np(grid.master)
        m64 = to_np(grid.adam_m)
        v64 = to_np(grid.adam_v)


def test_adam_step_full_size():
    """tg_adam_step at the training workload's size (128^3 vertices x 10 coefficients, FP32)
    against the oracle's Adam, every element, with established moments."""
    rng = np.random.default_rng(6)
    shape = (128, 128, 128, 10)
    th = rng.normal(0, 0.05, size=shape).astype(np.float32)
    grid = TaylorGrid(3, (128,) * 3, 2, (-1,) * 3, (1,) * 3, coeffs=torch.from_numpy(th), device=DEV)
    m = rng.normal(0, 1e-3, size=shape).astype(np.float32)
    v = rng.uniform(0, 1e-6, size=shape).astype(np.float32)
    g = (rng.normal(size=shape) * 1e-3).astype(np.float32)
    grid.adam_m.copy_(torch.from_numpy(m))
    grid.adam_v.copy_(torch.from_numpy(v))
    grid.grad.copy_(torch.from_numpy(g))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    gns = torch.zeros(1, dtype=torch.float64, device=DEV)
    grid.adam_step(ws, lr=1e-2, grad_norm_sq=gns, zero_grad=True, step=7)
    torch.cuda.synchronize()
    th64, m64, v64, ss = oracle.adam(th.astype(np.float64).reshape(-1), m.astype(np.float64).reshape(-1),
                                     v.astype(np.float64).reshape(-1), g.astype(np.float64).reshape(-1), 1e-2,
                                     0.9, 0.999, 1e-8, 0.0, 7)
    assert nerr(to_np(grid.master).reshape(-1), th64) <= TOL_VALUE
    assert nerr(to_np(grid.adam_m).reshape(-1), m64) <= TOL_VALUE
    assert nerr(to_np(grid.adam_v).reshape(-1), v64) <= TOL_VALUE
    # FP64 sums of the same 21M exact squares in two orders: n * 2^-53 bounds the difference
    assert abs(float(gns[0]) - ss) <= 21e6 * 2.0 ** -53 * ss
    assert torch.count_nonzero(grid.grad) == 0
