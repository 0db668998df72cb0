"""GPU parity of the packed layout: tg_forward_packed writes (f, grad f) of a query in one
16-byte row, and tg_backward / tg_backward_adam with TG_BWD_PACKED read (g_f, g_grad) in the
same layout.  Each is compared with the FP64 oracle, and with the separate-array calls on
the same inputs, which evaluate the same arithmetic: the forward and dq bit for bit, the
coefficient adjoint to rounding (the order of a vertex's summands inside one cell follows
LDS atomics, so it may differ between two launches)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _queries(dim, lo, hi, n, rng):
    """Uniform queries, a tenth outside the box (clamped axes) and a tenth in one hot cell."""
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    k = n // 10
    qu = rng.uniform(lo, hi, size=(n - 2 * k, dim))
    qo = rng.uniform(lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo), size=(k, dim))
    qh = lo + (hi - lo) * 0.37 + rng.uniform(0, 1e-3, size=(k, dim)) * (hi - lo)
    return np.concatenate([qu, qo, qh]).astype(np.float32).astype(np.float64)


def _pack(gf32, gg32, dim, pad=0.0):
    """[n, 4] rows (g_f, g_grad, pad...)."""
    up = np.full((len(gf32), 4), pad, dtype=np.float32)
    up[:, 0] = gf32
    up[:, 1:1 + dim] = gg32
    return torch.tensor(up, device=DEV)


def _both(grid, q64, gf32, gg32, pad=0.0):
    """Separate-array and packed forward, adjoint and dq on the same sort."""
    dim = grid.dim
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(q.shape[0])
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    fg = grid.forward_packed(q, ws)
    dq = grid.backward(q, ws, torch.tensor(gf32, device=DEV), torch.tensor(gg32, device=DEV), want_dq=True)
    dC = grid.grad.clone()
    dq_p = grid.backward(q, ws, packed=_pack(gf32, gg32, dim, pad), want_dq=True)
    torch.cuda.synchronize()
    return {"f": f, "g": g, "fg": fg, "dq": dq, "dC": dC, "dq_p": dq_p, "dC_p": grid.grad.clone()}


def _check(grid, C64, q64, gf32, gg32, r):
    dim = grid.dim
    fg = r["fg"]
    # the packed rows hold exactly the separate outputs
    assert torch.equal(fg[:, 0], r["f"]) and torch.equal(fg[:, 1:1 + dim], r["g"])
    if dim == 2:
        assert torch.all(fg[:, 3] == 0)
    assert torch.equal(r["dq_p"], r["dq"])
    assert nerr(to_np(r["dC_p"]), to_np(r["dC"])) <= TOL_VALUE
    # and against the oracle
    geom = geometry(grid)
    rule = FaceRule(geom, C64, q64)
    ref_f, ref_g = oracle.forward(geom, C64, q64)
    assert nerr(to_np(fg[:, 0]), ref_f) <= TOL_VALUE
    assert rule.grad_err(to_np(fg[:, 1:1 + dim]), ref_g) <= TOL_GRAD
    gf, gg = gf32.astype(np.float64), gg32.astype(np.float64)
    ref_dC, ref_dq = oracle.backward(geom, C64, q64, gf, gg, want_dq=True)
    e_dc = rule.dC_err(to_np(r["dC_p"]), ref_dC, gf, gg)
    e_dq = rule.dq_err(to_np(r["dq_p"]), ref_dq, gf, gg)
    print(f"packed: dC err {e_dc:.2e} dq err {e_dq:.2e} ({rule.count} queries on a face)")
    assert e_dc <= TOL_GRAD and e_dq <= TOL_GRAD


@pytest.mark.parametrize("order", [0, 1, 2])
def test_packed_3d(order):
    """Ragged 3D grid (several bricks, partial edge bricks), clamped and crowded queries."""
    rng = np.random.default_rng(700 + order)
    res, lo, hi = (37, 30, 19), (-1.0, -0.5, 0.25), (1.0, 1.5, 0.75)
    nc = (order + 1) * (order + 2) * (order + 3) // 6
    C32 = rng.normal(0, 0.05, size=(res[2], res[1], res[0], nc)).astype(np.float32)
    grid = TaylorGrid(3, res, order, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    n = 50_000
    q64 = _queries(3, lo, hi, n, rng)
    gf32 = (rng.normal(size=n) / n).astype(np.float32)
    gg32 = (rng.normal(size=(n, 3)) / n).astype(np.float32)
    _check(grid, C32.astype(np.float64), q64, gf32, gg32, _both(grid, q64, gf32, gg32))


@pytest.mark.parametrize("order", [1, 2])
def test_packed_2d_ignores_the_fourth_word(order):
    """2D rows carry (g_f, g_grad_x, g_grad_y, unused): a NaN in the unused word must not reach
    any result, and the forward writes 0 there."""
    rng = np.random.default_rng(710 + order)
    res, lo, hi = (45, 38), (-2.0, 0.0), (2.0, 3.0)
    nc = (order + 1) * (order + 2) // 2
    C32 = rng.normal(0, 0.05, size=(res[1], res[0], nc)).astype(np.float32)
    grid = TaylorGrid(2, res, order, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    n = 40_000
    q64 = _queries(2, lo, hi, n, rng)
    gf32 = (rng.normal(size=n) / n).astype(np.float32)
    gg32 = (rng.normal(size=(n, 2)) / n).astype(np.float32)
    r = _both(grid, q64, gf32, gg32, pad=float("nan"))
    assert torch.isfinite(r["dC_p"]).all() and torch.isfinite(r["dq_p"]).all()
    _check(grid, C32.astype(np.float64), q64, gf32, gg32, r)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_packed_16bit_storage(storage):
    """BF16 / FP16 storage (coefficients widened when staged): the packed rows equal the
    separate-array outputs bit for bit, and the adjoint from packed upstream gradients equals
    the separate one to rounding."""
    rng = np.random.default_rng(725)
    res, lo, hi = (29, 22, 17), (-1.0,) * 3, (1.0,) * 3
    C32 = rng.normal(0, 0.05, size=(res[2], res[1], res[0], 10)).astype(np.float32)
    grid = TaylorGrid(3, res, 2, lo, hi, storage=storage, coeffs=torch.from_numpy(C32), device=DEV)
    n = 30_000
    q64 = _queries(3, lo, hi, n, rng)
    gf32 = (rng.normal(size=n) / n).astype(np.float32)
    gg32 = (rng.normal(size=(n, 3)) / n).astype(np.float32)
    r = _both(grid, q64, gf32, gg32)
    assert torch.equal(r["fg"][:, 0], r["f"]) and torch.equal(r["fg"][:, 1:], r["g"])
    assert torch.equal(r["dq_p"], r["dq"])
    assert nerr(to_np(r["dC_p"]), to_np(r["dC"])) <= TOL_VALUE


def test_packed_full_hessian_layout():
    """The 13-coefficient layout through the packed calls equals its separate-array calls."""
    rng = np.random.default_rng(720)
    res, lo, hi = (21, 18, 26), (-1.0,) * 3, (1.0,) * 3
    C32 = rng.normal(0, 0.05, size=(res[2], res[1], res[0], 13)).astype(np.float32)
    grid = TaylorGrid(3, res, 2, lo, hi, coeffs=torch.from_numpy(C32), device=DEV, hessian="full")
    n = 30_000
    q64 = _queries(3, lo, hi, n, rng)
    gf32 = (rng.normal(size=n) / n).astype(np.float32)
    gg32 = (rng.normal(size=(n, 3)) / n).astype(np.float32)
    r = _both(grid, q64, gf32, gg32)
    assert torch.equal(r["fg"][:, 0], r["f"]) and torch.equal(r["fg"][:, 1:], r["g"])
    assert torch.equal(r["dq_p"], r["dq"])
    assert nerr(to_np(r["dC_p"]), to_np(r["dC"])) <= TOL_VALUE


def test_packed_backward_adam_equals_separate():
    """tg_backward_adam with TG_BWD_PACKED: the same update as with separate arrays, over
    several steps (master, both moments and the gradient norm), to the rounding of the
    adjoint's sums."""
    rng = np.random.default_rng(730)
    res, lo, hi = (33, 33, 33), (-1.0,) * 3, (1.0,) * 3
    C32 = rng.normal(0, 0.05, size=(res[2], res[1], res[0], 10)).astype(np.float32)
    a = TaylorGrid(3, res, 2, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    b = TaylorGrid(3, res, 2, lo, hi, coeffs=torch.from_numpy(C32), device=DEV)
    # established moments: on a first step a gradient near zero would turn the rounding
    # difference of two summation orders into a step of up to lr
    m0 = torch.tensor(rng.normal(0, 1e-5, size=C32.shape), dtype=torch.float32)
    v0 = torch.tensor(rng.uniform(1e-9, 1e-8, size=C32.shape), dtype=torch.float32)
    for g_ in (a, b):
        g_.adam_m.copy_(m0)
        g_.adam_v.copy_(v0)
    n = 40_000
    q = torch.tensor(_queries(3, lo, hi, n, rng), dtype=torch.float32, device=DEV)
    ws = a.workspace(n)
    na = torch.empty(1, dtype=torch.float64, device=DEV)
    nb = torch.empty(1, dtype=torch.float64, device=DEV)
    for step in range(3):
        gf32 = (rng.normal(size=n) / n).astype(np.float32)
        gg32 = (rng.normal(size=(n, 3)) / n).astype(np.float32)
        a.sort(q, ws)
        a.backward_adam(q, ws, torch.tensor(gf32, device=DEV), torch.tensor(gg32, device=DEV), grad_norm_sq=na,
                        step=10 + step)
        b.sort(q, ws)
        b.backward_adam(q, ws, packed=_pack(gf32, gg32, 3), grad_norm_sq=nb, step=10 + step)
        torch.cuda.synchronize()
        np.testing.assert_allclose(nb.item(), na.item(), rtol=TOL_VALUE)  # FP32 gradients equal up to rounding
    for name, tol in (("master", 1e-6), ("adam_m", TOL_VALUE), ("adam_v", TOL_VALUE)):
        e = nerr(to_np(getattr(b, name)), to_np(getattr(a, name)))
        print(f"{name}: {e:.2e}")
        assert e <= tol


def test_packed_full_size_matches_separate():
    """128^3 vertices, K=2, 2^20 queries of the SDF-fitting batch (the size the benchmark's
    forward + backward runs at): the packed calls reproduce the separate-array calls (the
    forward bit for bit, the adjoint to rounding), and sampled queries agree with the
    oracle."""
    C64, q64, _, _ = synth.scene3d_inputs(res=128, order=2, n=1 << 20, seed=0)
    C32 = C64.astype(np.float32)
    del C64
    grid = TaylorGrid(3, (128,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    rng = np.random.default_rng(740)
    n = len(q64)
    gf32 = (rng.normal(size=n) / n).astype(np.float32)
    gg32 = (rng.normal(size=(n, 3)) / n).astype(np.float32)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    fg = grid.forward_packed(q, ws)
    grid.backward(q, ws, torch.tensor(gf32, device=DEV), torch.tensor(gg32, device=DEV))
    dC = grid.grad.clone()
    grid.backward(q, ws, packed=_pack(gf32, gg32, 3))
    torch.cuda.synchronize()
    assert torch.equal(fg[:, 0], f) and torch.equal(fg[:, 1:], g)
    assert nerr(to_np(grid.grad), to_np(dC)) <= TOL_VALUE
    # sampled forward rows against the oracle
    idx = rng.choice(n, 4096, replace=False)
    geom = geometry(grid)
    C = C32.astype(np.float64)
    ref_f, ref_g = oracle.forward(geom, C, q64[idx])
    rule = FaceRule(geom, C, q64[idx])
    assert nerr(to_np(fg[idx, 0]), ref_f) <= TOL_VALUE
    assert rule.grad_err(to_np(fg[idx, 1:]), ref_g) <= TOL_GRAD
