"""The paper's full SDF objective and the coarse-to-fine step on the GPU against the FP64
oracle (oracle/objective.py): Eq. 7's adaptive weight in the stand-alone loss, in the fused
forward + loss and in the training step; the TV term (value and gradient, overwrite and
accumulate, 2D and 3D, every coefficient count, ragged tiles, the 128^3 K=2 grid); the
training step with every term against the oracle's forward, loss, adjoint, TV and Adam; the
coarse-to-fine transfer (exact quadratics, random fields, coarse faces under fine vertices)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import objective as obj
from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss
from parity_util import TOL_GRAD, TOL_VALUE, geometry, nerr, nerr_cols, to_np
from test_oracle_pins import _random_poly, _taylor_coeffs_of

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _grid(dim, res, order, rng, lo=None, hi=None, storage="f32", std=0.05):
    lo = lo or (-1.0,) * dim
    hi = hi or (1.0,) * dim
    C = oracle.num_coeffs(dim, order)
    coeffs = _f32(rng.normal(0, std, size=tuple(reversed(res)) + (C,)))
    g = TaylorGrid(dim, res, order, lo, hi, storage=storage, coeffs=torch.from_numpy(coeffs.astype(np.float32)),
                   device=DEV)
    return g, coeffs


@pytest.mark.parametrize("k", [0.0, 9.0, 60.0])
def test_weighted_sdf_loss_kernel(k):
    rng = np.random.default_rng(int(k) + 1)
    n = 200_003
    f = _f32(rng.normal(0, 0.2, size=n))
    d = _f32(f + rng.normal(0, 0.1, size=n))
    gr = _f32(rng.normal(0, 1, size=(n, 3)))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    loss, g_f, g_grad = sdf_loss(T(f), T(gr), T(d), 0.1, ws, surface_k=k)
    ref, rgf, rgg = obj.weighted_sdf_loss(f, gr, d, 0.1, k)
    torch.cuda.synchronize()
    assert nerr(to_np(loss), ref) <= TOL_VALUE
    assert nerr(to_np(g_f), rgf) <= TOL_GRAD
    assert nerr_cols(to_np(g_grad), rgg) <= TOL_GRAD


def test_weighted_forward_sdf_loss():
    rng = np.random.default_rng(5)
    g, C = _grid(3, (37, 40, 29), 2, rng)
    n = 150_000
    q = _f32(rng.uniform(-1, 1, size=(n, 3)))
    d = _f32(rng.normal(0, 0.05, size=n))
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    ws = g.workspace(n)
    g.sort(qt, ws)
    loss, g_f, g_grad = g.forward_sdf_loss(qt, ws, torch.tensor(d, dtype=torch.float32, device=DEV), 0.1,
                                           surface_k=12.0)
    f, grad = oracle.forward(geometry(g), C, q)
    ref, rgf, rgg = obj.weighted_sdf_loss(f, grad, d, 0.1, 12.0)
    torch.cuda.synchronize()
    assert nerr(to_np(loss), ref) <= TOL_VALUE
    assert nerr(to_np(g_f), rgf) <= TOL_GRAD
    assert nerr_cols(to_np(g_grad), rgg) <= TOL_GRAD


@pytest.mark.parametrize("dim,res,order", [(3, (37, 40, 29), 2), (3, (9, 17, 8), 1), (3, (20, 3, 11), 0),
                                           (2, (70, 45), 2), (2, (33, 16), 1), (2, (2, 50), 0)])
def test_tv_matches_oracle(dim, res, order):
    """Tiles of 8^3 (16^2) vertices with ragged edges, and the accumulate flag."""
    rng = np.random.default_rng(sum(res) + order)
    g, C = _grid(dim, res, order, rng)
    ws = torch.empty(g.workspace_bytes(0), dtype=torch.uint8, device=DEV)
    weight = 0.75
    loss = g.tv_loss(weight, ws)
    torch.cuda.synchronize()
    ref, rgrad = obj.tv(C, dim)
    assert abs(float(loss[0]) - ref) <= TOL_VALUE * ref
    assert nerr(to_np(g.grad), weight * rgrad) <= TOL_GRAD
    base = _f32(rng.normal(0, 1e-3, size=C.shape))
    g.grad.copy_(torch.from_numpy(base.astype(np.float32)))
    g.tv_loss(weight, ws, accumulate=True)
    torch.cuda.synchronize()
    assert nerr(to_np(g.grad), base + weight * rgrad) <= TOL_GRAD


def test_tv_full_size_128():
    """The 128^3 K=2 grid (10 coefficients per vertex) of the SDF workload."""
    rng = np.random.default_rng(128)
    g, C = _grid(3, (128,) * 3, 2, rng)
    ws = torch.empty(g.workspace_bytes(0), dtype=torch.uint8, device=DEV)
    loss = g.tv_loss(2e-5, ws)
    torch.cuda.synchronize()
    ref, rgrad = obj.tv(C, 3)
    assert abs(float(loss[0]) - ref) <= TOL_VALUE * ref
    assert nerr(to_np(g.grad), 2e-5 * rgrad) <= TOL_GRAD


@pytest.mark.parametrize("tv_weight", [0.0, 2.0])
def test_train_step_full_objective(tv_weight):
    """One step of L = weighted L1 + 0.1 eikonal (+ TV) against the oracle: forward, Eq. 7
    weight, loss gradients, coefficient adjoint, TV gradient, Adam (established moments)."""
    rng = np.random.default_rng(77)
    g, C = _grid(3, (37, 40, 29), 2, rng)
    m0 = _f32(rng.normal(0, 1e-5, size=C.shape))
    v0 = _f32(rng.uniform(1e-9, 1e-8, size=C.shape))
    g.adam_m.copy_(torch.from_numpy(m0.astype(np.float32)))
    g.adam_v.copy_(torch.from_numpy(v0.astype(np.float32)))
    n = 100_000
    q = _f32(rng.uniform(-1, 1, size=(n, 3)))
    d = _f32(rng.normal(0, 0.05, size=n))
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    ws = g.workspace(n)
    gn = torch.zeros(1, dtype=torch.float64, device=DEV)
    loss = g.train_step(qt, torch.tensor(d, dtype=torch.float32, device=DEV), ws, eik_weight=0.1, lr=1e-2,
                        step=10, grad_norm_sq=gn, surface_k=12.0, tv_weight=tv_weight)
    torch.cuda.synchronize()

    geom = geometry(g)
    f, grad = oracle.forward(geom, C, q)
    ref, gf, gg = obj.weighted_sdf_loss(f, grad, d, 0.1, 12.0)
    dC = oracle.backward(geom, C, q, gf, gg)[0]
    ref = list(ref)
    if tv_weight:
        tv, tg = obj.tv(C, 3)
        dC = dC + tv_weight * tg
        ref[0] += tv_weight * tv
        ref.append(tv)
    assert nerr(to_np(loss), np.array(ref)) <= TOL_VALUE
    th, mm, vv, ss = oracle.adam(C.reshape(-1), m0.reshape(-1), v0.reshape(-1), dC.reshape(-1), 1e-2, step=10)
    assert nerr(to_np(g.master).reshape(-1), th) <= TOL_VALUE
    assert nerr(to_np(g.adam_m).reshape(-1), mm) <= TOL_GRAD
    assert abs(gn.item() - ss) <= 1e-4 * ss


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("fine_order", [0, 1, 2])
def test_upsample_reproduces_a_quadratic(dim, fine_order):
    rng = np.random.default_rng(40 + dim)
    p = _random_poly(dim, 2, rng)
    if dim == 3:
        lo, hi, rc, rf = (-1.0, 0.25, -3.0), (2.0, 1.5, -0.5), (4, 5, 3), (7, 9, 6)
    else:
        lo, hi, rc, rf = (-1.0, 0.25), (2.0, 1.5), (5, 4), (9, 10)
    gc = oracle.Geometry(dim, rc, 2, lo, hi)
    gf = oracle.Geometry(dim, rf, fine_order, lo, hi)
    coarse = TaylorGrid(dim, rc, 2, lo, hi, coeffs=torch.tensor(_taylor_coeffs_of(p, gc), dtype=torch.float32),
                        device=DEV)
    fine = TaylorGrid(dim, rf, fine_order, lo, hi, device=DEV)
    fine.adam_m.fill_(1.0)
    fine.upsample_from(coarse)
    torch.cuda.synchronize()
    exact = _taylor_coeffs_of(p, gf)
    assert nerr(to_np(fine.master), exact) <= TOL_VALUE
    assert not fine.adam_m.any()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_upsample_random_field(storage):
    """A random K=2 field, 33^3 -> 64^3 (gcd(32, 63) = 1: no fine vertex on a coarse face
    inside the box), against the oracle's value, gradient and Hessian."""
    rng = np.random.default_rng(9)
    coarse, Cc = _grid(3, (33,) * 3, 2, rng)
    fine = TaylorGrid(3, (64,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, storage=storage, device=DEV)
    fine.upsample_from(coarse)
    torch.cuda.synchronize()
    ref = obj.upsample(geometry(coarse), Cc, geometry(fine))
    got = to_np(fine.master)
    assert nerr(got[..., 0], ref[..., 0]) <= TOL_VALUE
    for k in range(1, 10):
        assert nerr(got[..., k], ref[..., k]) <= TOL_GRAD, k
    if storage == "bf16":
        expect = fine.master.to(torch.bfloat16)
        assert torch.equal(fine.coeffs, expect)


def test_upsample_fine_vertices_on_coarse_faces():
    """17^3 -> 33^3: every other fine vertex lies on a coarse face.  The value is continuous
    there and matches everywhere; the one-sided gradient and Hessian are compared where the
    fine vertex is inside a coarse cell on every axis."""
    rng = np.random.default_rng(11)
    coarse, Cc = _grid(3, (17,) * 3, 2, rng)
    fine = TaylorGrid(3, (33,) * 3, 1, (-1.0,) * 3, (1.0,) * 3, device=DEV)
    fine.upsample_from(coarse)
    torch.cuda.synchronize()
    ref = obj.upsample(geometry(coarse), Cc, geometry(fine))
    got = to_np(fine.master)
    assert nerr(got[..., 0], ref[..., 0]) <= TOL_VALUE
    odd = np.arange(33) % 2 == 1
    inside = odd[:, None, None] & odd[None, :, None] & odd[None, None, :]
    for k in range(1, 4):
        assert nerr(got[..., k][inside], ref[..., k][inside]) <= TOL_GRAD


def test_progressive_fit_continues_from_the_coarse_field():
    """32^3 -> 64^3 on the scene with the full objective: the fine level starts from the
    coarse field (its loss is far below the random start's, though above the coarse loss: the
    coarse field is only C0 across its cell faces, which the fine Taylor series smooth), and
    fitting at the fine level lowers the loss further."""
    import math

    from paper_2402_14415_amd import synth
    from paper_2402_14415_amd.progressive import ProgressiveFit

    scene = synth.Scene(3)
    k = math.log(3.0) / (2 * 2.0 / 63)
    fit = ProgressiveFit(3, [32, 64], 2, (-1.0,) * 3, (1.0,) * 3, device=DEV, eik_weight=0.1, surface_k=k,
                         tv_weight=1e-4, lr=1e-2)
    batches = []
    for s in range(4):
        q, d = synth.scene_batch(scene, 1 << 16, seed=3, step=s)
        batches.append((torch.tensor(q, dtype=torch.float32, device=DEV),
                        torch.tensor(d, dtype=torch.float32, device=DEV)))
    first = None
    for it in range(60):
        loss = fit.step(*batches[it % 4])
        if first is None:
            first = float(loss[0])
    lc = to_np(fit.step(*batches[0], lr=0.0))  # lr 0: the loss of the field as it is
    coarse_last = float(lc[0])
    fit.advance()
    assert fit.grid.res == (64, 64, 64) and fit.grid.step_count == 0
    lf = to_np(fit.step(*batches[0], lr=0.0))
    fine_first = float(lf[0])
    print("coarse [total, weighted L1, eikonal, TV]:", lc, " fine start:", lf)
    for it in range(60):
        loss = fit.step(*batches[it % 4])
    fine_last = float(fit.step(*batches[0], lr=0.0)[0])
    print(f"loss: start {first:.4f}, coarse {coarse_last:.4f}, fine start {fine_first:.4f}, fine {fine_last:.4f}")
    assert coarse_last < 0.5 * first
    assert fine_first < 0.5 * first
    assert fine_last < fine_first
    with pytest.raises(IndexError):
        fit.advance()


def test_full_objective_train_step_matches_separate_calls_full_size():
    """128^3 K=2, 2^20 scene queries (the headline shape) with every term of Eq. 8: the
    one-call step against sort + tg_tv_loss + tg_forward_sdf_loss + tg_backward_adam with the
    TV gradient added (TG_BWD_ADD_GRAD), over two steps."""
    import math

    from paper_2402_14415_amd import synth

    C64, q64, d64, scene = synth.scene3d_inputs(res=128, order=2, n=1 << 20, seed=0)
    C32 = torch.from_numpy(C64.astype(np.float32))
    del C64
    a = TaylorGrid(3, (128,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=C32, device=DEV)
    b = TaylorGrid(3, (128,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=C32, device=DEV)
    # established moments: a first Adam step from zero moments divides by |g| itself and so
    # amplifies the rounding of near-cancelling gradient sums (the two sorts order a bucket's
    # records differently)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(8)
    m0 = torch.randn(a.shape, generator=gen, device=DEV) * 1e-5
    v0 = torch.rand(a.shape, generator=gen, device=DEV) * 9e-9 + 1e-9
    for g_ in (a, b):
        g_.adam_m.copy_(m0)
        g_.adam_v.copy_(v0)
    k = math.log(3.0) / (2 * 2.0 / 127)
    n = 1 << 20
    wa, wb = a.workspace(n), b.workspace(n)
    for step in range(2):
        q64, d64 = synth.scene_batch(scene, n, seed=0, step=step)
        q = torch.tensor(q64, dtype=torch.float32, device=DEV)
        d = torch.tensor(d64, dtype=torch.float32, device=DEV)
        la = a.train_step(q, d, wa, eik_weight=0.1, lr=1e-2, surface_k=k, tv_weight=2e-5, step=step + 10)
        b.sort(q, wb)
        tv = b.tv_loss(2e-5, wb)
        lb, gf, gg = b.forward_sdf_loss(q, wb, d, 0.1, surface_k=k)
        b.backward_adam(q, wb, gf, gg, lr=1e-2, step=step + 10, add_grad=True)
        torch.cuda.synchronize()
        np.testing.assert_allclose(to_np(la)[:3] - [2e-5 * float(tv[0]), 0, 0], to_np(lb), rtol=1e-6)
        assert abs(float(la[3]) - float(tv[0])) <= 1e-12 * float(tv[0])
        for name, tol in (("master", 1e-6), ("adam_m", TOL_VALUE), ("adam_v", TOL_VALUE)):
            e = nerr(to_np(getattr(a, name)).reshape(-1), to_np(getattr(b, name)).reshape(-1))
            print(f"step {step} {name}: {e:.2e}")
            assert e <= tol


def test_train_step_without_queries_applies_tv_alone():
    """No queries: the step's loss is the TV term alone and every coefficient takes the Adam
    step of the TV gradient (tg_tv_loss then tg_adam_step)."""
    rng = np.random.default_rng(12)
    a, C = _grid(3, (20, 17, 23), 2, rng)
    b = TaylorGrid(3, (20, 17, 23), 2, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(C.astype(np.float32)),
                   device=DEV)
    q = torch.empty((0, 3), device=DEV)
    d = torch.empty(0, device=DEV)
    wa = a.workspace(0)
    loss = a.train_step(q, d, wa, eik_weight=0.1, lr=1e-2, tv_weight=0.5, step=1)
    wb = b.workspace(0)
    tv = b.tv_loss(0.5, wb)
    b.adam_step(wb, lr=1e-2, step=1)
    torch.cuda.synchronize()
    ref, _ = obj.tv(C, 3)
    assert to_np(loss)[1] == 0.0 and to_np(loss)[2] == 0.0
    assert abs(to_np(loss)[3] - ref) <= TOL_VALUE * ref and abs(to_np(loss)[0] - 0.5 * to_np(loss)[3]) <= 1e-15
    assert float(tv[0]) == to_np(loss)[3]
    assert nerr(to_np(a.master).reshape(-1), to_np(b.master).reshape(-1)) <= 1e-6
