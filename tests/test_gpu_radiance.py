"""Radiance-field form on the GPU against the FP64 oracle (oracle/radiance.py and the grid
oracle): the compositing kernel (Sec. 3.3 Eq. 10-11 and its adjoint) for every sample-count
shape it dispatches on, rendering at the full 160^3 size on sampled rays, and one whole
training step (grid evaluation, compositing, fused adjoint + Adam of the density and the
three-channel colour grid), the shared sort and the three-channel grid itself."""
import numpy as np
import pytest
import torch

import oracle
from oracle import radiance as orad
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.radiance import RadianceField, composite
from parity_util import TOL_GRAD, TOL_VALUE, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("n_rays,ns", [(1000, 256), (777, 37), (300, 100), (64, 1), (40, 1024), (0, 16),
                                         (200, 480), (50, 300)])
def test_composite_matches_oracle(n_rays, ns):
    rng = np.random.default_rng(ns)
    f = _f32(rng.normal(0.5, 2.0, size=(n_rays, ns)))  # a fifth or so non-positive: ReLU zeroes them
    c = _f32(rng.uniform(0, 1, size=(n_rays, ns, 3)))
    delta = _f32(rng.uniform(0.0, 3.0 / ns, size=(n_rays, ns)))
    target = _f32(rng.uniform(0, 1, size=(n_rays, 3)))
    ws = torch.empty(1 << 16, dtype=torch.uint8, device=DEV)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV).contiguous()
    print(f"rays {n_rays} samples {ns}", flush=True)
    rgb, loss, g_f, g_c = composite(t(f.reshape(-1)), t(np.moveaxis(c, 2, 0).reshape(3, -1)), t(delta.reshape(-1)),
                                    ns, ws, target=t(target))
    torch.cuda.synchronize()
    if n_rays == 0:
        assert float(loss[0]) == 0.0
        return
    ref_loss, ref_rgb, ref_gf, ref_gc = orad.composite_backward(f, c, delta, target)
    assert nerr(to_np(rgb), ref_rgb) <= TOL_VALUE
    assert abs(float(loss[0]) - ref_loss) <= TOL_VALUE * ref_loss
    assert nerr(to_np(g_f).reshape(n_rays, ns), ref_gf) <= TOL_GRAD
    assert nerr(to_np(g_c).reshape(3, n_rays, ns), np.moveaxis(ref_gc, 2, 0)) <= TOL_GRAD
    assert np.all(to_np(g_f).reshape(n_rays, ns)[f <= 0] == 0.0)
    # without a target: the colours only, the same values
    rgb2, loss2, _, _ = composite(t(f.reshape(-1)), t(np.moveaxis(c, 2, 0).reshape(3, -1)), t(delta.reshape(-1)),
                                  ns, ws)
    torch.cuda.synchronize()
    assert loss2 is None and torch.equal(rgb2, rgb)


def _field(res, seed):
    rng = np.random.default_rng(seed)
    dens = (0.5 + rng.normal(0, 0.3, size=tuple(reversed(res)) + (10,))).astype(np.float32)
    col = rng.uniform(0, 1, size=(3,) + tuple(reversed(res)) + (4,)).astype(np.float32)
    col[..., 1:] *= 0.1
    return dens, col


def _oracle_fields(res, dens, col, q):
    geom_d = oracle.Geometry(3, res, 2, (-1.0,) * 3, (1.0,) * 3)
    geom_c = oracle.Geometry(3, res, 1, (-1.0,) * 3, (1.0,) * 3)
    f = oracle.forward(geom_d, dens.astype(np.float64), q, want_grad=False)
    c = np.stack([oracle.forward(geom_c, col[k].astype(np.float64), q, want_grad=False) for k in range(3)], axis=-1)
    return geom_d, geom_c, f, c


def test_render_full_size_sampled_rays():
    """160^3 grids and a 4096-ray x 256-sample batch (the bench's shape); 64 rays checked."""
    res = (160, 160, 160)
    dens, col = _field(res, 1)
    field = RadianceField(res, coeffs=(torch.from_numpy(dens), [torch.from_numpy(col[k]) for k in range(3)]),
                          device=DEV)
    o, d = synth.camera_rays(4096, seed=1, step=0)
    q64, delta64 = synth.stratified_samples(o, d, 256, seed=1, step=0)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    delta = torch.tensor(delta64, dtype=torch.float32, device=DEV)
    ws = field.workspace(q.shape[0])
    rgb = to_np(field.render(q, delta, 256, ws))
    pick = np.random.default_rng(0).choice(4096, size=64, replace=False)
    qs = q64.reshape(4096, 256, 3)[pick].reshape(-1, 3)
    _, _, f, c = _oracle_fields(res, dens, col, qs)
    ref, _, _ = orad.composite(f.reshape(64, 256), c.reshape(64, 256, 3), delta64.reshape(4096, 256)[pick])
    assert nerr(rgb[pick], ref) <= TOL_VALUE


def test_training_step_matches_oracle():
    """One step on a 24^3 field: loss, and both grids' master and moments after the fused
    adjoint + Adam, against the oracle's forward, compositing adjoint, grid adjoint (per colour
    channel) and Adam.  Established moments (a first Adam step amplifies rounding where a
    gradient is near 0)."""
    res = (24, 24, 24)
    dens, col = _field(res, 2)
    field = RadianceField(res, coeffs=(torch.from_numpy(dens), [torch.from_numpy(col[k]) for k in range(3)]),
                          device=DEV)
    rng = np.random.default_rng(3)
    m0 = [rng.normal(0, 1e-4, size=g.master.shape).astype(np.float32) for g in field.grids]
    v0 = [rng.uniform(1e-9, 1e-8, size=g.master.shape).astype(np.float32) for g in field.grids]
    for g, m, v in zip(field.grids, m0, v0):
        g.adam_m.copy_(torch.from_numpy(m))
        g.adam_v.copy_(torch.from_numpy(v))
    n_rays, ns = 300, 64
    o, d = synth.camera_rays(n_rays, seed=2, step=0)
    q64, delta64 = synth.stratified_samples(o, d, ns, seed=2, step=0)
    target = _f32(rng.uniform(0, 1, size=(n_rays, 3)))
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = field.workspace(q.shape[0])
    loss = field.train_step(q, torch.tensor(delta64, dtype=torch.float32, device=DEV), ns,
                            torch.tensor(target, dtype=torch.float32, device=DEV), ws, lr=1e-2, step=10)
    torch.cuda.synchronize()

    geom_d, geom_c, f, c = _oracle_fields(res, dens, col, q64)
    ref_loss, _, g_f, g_c = orad.composite_backward(f.reshape(n_rays, ns), c.reshape(n_rays, ns, 3),
                                                    delta64.reshape(n_rays, ns), target)
    assert abs(float(loss[0]) - ref_loss) <= 1e-5 * ref_loss
    grads = [oracle.backward(geom_d, dens.astype(np.float64), q64, g_f.reshape(-1), None)[0]]
    # the colour grid stores the three channels' series per vertex, one after the other
    grads += [np.concatenate([oracle.backward(geom_c, col[k].astype(np.float64), q64, g_c[:, :, k].reshape(-1),
                                              None)[0] for k in range(3)], axis=-1)]
    inits = [dens, np.concatenate([col[k] for k in range(3)], axis=-1)]
    for g, th0, m, v, gr in zip(field.grids, inits, m0, v0, grads):
        th, mm, vv, _ = oracle.adam(th0.astype(np.float64).reshape(-1), m.astype(np.float64).reshape(-1),
                                    v.astype(np.float64).reshape(-1), gr.reshape(-1), 1e-2, step=10)
        e_th = nerr(to_np(g.master).reshape(-1), th)
        e_m = nerr(to_np(g.adam_m).reshape(-1), mm)
        print(f"order {g.order}: master {e_th:.2e} m {e_m:.2e}", flush=True)
        assert e_th <= TOL_VALUE and e_m <= TOL_GRAD


def test_shared_sort():
    """A K=1 grid reusing a K=2 grid's sort of the same samples (tg_share_sort): forward
    bitwise equal to its own sort's, adjoint against the oracle with crowded bricks split
    over several items (their partial sums sit behind the shared sections of the workspace),
    and a later sort into the workspace supersedes the shared one."""
    from paper_2402_14415_amd._lib import TaylorGridError
    from paper_2402_14415_amd.grid import TaylorGrid

    res = (40, 40, 40)
    rng = np.random.default_rng(7)
    n = 60000
    q64 = np.concatenate([rng.uniform(-1, 1, size=(n // 2, 3)),
                          np.clip(rng.normal(0.3, 0.03, size=(n - n // 2, 3)), -1, 1)])
    q64 = _f32(q64)
    cd = _f32(rng.normal(0, 0.05, size=res + (10,)))
    cc = _f32(rng.normal(0, 0.05, size=res + (4,)))
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    dens = TaylorGrid(3, res, 2, lo, hi, coeffs=torch.from_numpy(cd.astype(np.float32)), device=DEV)
    col = TaylorGrid(3, res, 1, lo, hi, coeffs=torch.from_numpy(cc.astype(np.float32)), device=DEV)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = dens.workspace(n)
    dens.sort(q, ws)
    col.share_sort(dens, q, ws)
    f_sh, g_sh = col.forward(q, ws)
    ws_own = col.workspace(n)
    col.sort(q, ws_own)
    f_own, g_own = col.forward(q, ws_own)
    assert torch.equal(f_sh, f_own) and torch.equal(g_sh, g_own)
    geom = oracle.Geometry(3, res, 1, lo, hi)
    f_ref, g_ref = oracle.forward(geom, cc, q64)
    assert nerr(to_np(f_sh), f_ref) <= TOL_VALUE and nerr(to_np(g_sh), g_ref) <= TOL_GRAD

    gf = _f32(rng.normal(0, 1, size=n))
    col.share_sort(dens, q, ws)
    col.backward(q, ws, torch.tensor(gf, dtype=torch.float32, device=DEV))
    dc_ref = oracle.backward(geom, cc, q64, gf, None)[0]
    assert nerr(to_np(col.grad).reshape(dc_ref.shape), dc_ref) <= TOL_GRAD

    # the density grid sorts other samples into ws: the colour grid's shared sort is stale
    q2 = q.flip(0).contiguous()
    dens.sort(q2, ws)
    with pytest.raises(TaylorGridError) as err:
        col.forward(q, ws)
    assert err.value.status == 5
    col.ensure_sorted(q, ws)  # the binding sees the same generation rule and sorts again
    f_again, _ = col.forward(q, ws)
    assert torch.equal(f_again, f_own)


def test_three_channel_grid():
    """The three-channel order-1 grid against the oracle channel by channel: forward (f [3, n]),
    adjoint from g_f [3, n], and the fused adjoint + Adam, with crowded bricks split over
    several items; the SDF calls refuse it."""
    from paper_2402_14415_amd._lib import TaylorGridError
    from paper_2402_14415_amd.grid import TaylorGrid

    res = (29, 33, 26)
    rng = np.random.default_rng(31)
    n = 70000
    q64 = _f32(np.concatenate([rng.uniform(-1.05, 1.05, size=(n // 2, 3)),
                               np.clip(rng.normal(-0.2, 0.03, size=(n - n // 2, 3)), -1, 1)]))
    cc = _f32(rng.normal(0, 0.05, size=res[::-1] + (12,)))
    g = TaylorGrid(3, res, 1, (-1.0,) * 3, (1.0,) * 3, coeffs=torch.from_numpy(cc.astype(np.float32)), device=DEV,
                   channels=3)
    assert g.C == 12
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = g.workspace(n)
    g.sort(q, ws)
    f, grad = g.forward(q, ws)
    assert grad is None and f.shape == (3, n)
    gf = _f32(rng.normal(0, 1, size=(3, n)))
    g.backward(q, ws, torch.tensor(gf, dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    geom = oracle.Geometry(3, res, 1, (-1.0,) * 3, (1.0,) * 3)
    dC = []
    for k in range(3):
        ck = cc[..., 4 * k: 4 * k + 4]
        assert nerr(to_np(f)[k], oracle.forward(geom, ck, q64, want_grad=False)) <= TOL_VALUE
        dC.append(oracle.backward(geom, ck, q64, gf[k], None)[0])
        assert nerr(to_np(g.grad)[..., 4 * k: 4 * k + 4], dC[k]) <= TOL_GRAD
    dC = np.concatenate(dC, axis=-1)
    m0 = _f32(rng.normal(0, 1e-5, size=cc.shape))
    v0 = _f32(rng.uniform(1e-9, 1e-8, size=cc.shape))
    g.adam_m.copy_(torch.from_numpy(m0.astype(np.float32)))
    g.adam_v.copy_(torch.from_numpy(v0.astype(np.float32)))
    g.backward_adam(q, ws, torch.tensor(gf, dtype=torch.float32, device=DEV), None, lr=1e-2, step=10)
    torch.cuda.synchronize()
    th, mm, _, _ = oracle.adam(cc.reshape(-1), m0.reshape(-1), v0.reshape(-1), dC.reshape(-1), 1e-2, step=10)
    assert nerr(to_np(g.master).reshape(-1), th) <= TOL_VALUE
    assert nerr(to_np(g.adam_m).reshape(-1), mm) <= TOL_GRAD
    d = torch.zeros(n, device=DEV)
    with pytest.raises(TaylorGridError) as err:
        g.train_step(q, d, ws)
    assert err.value.status == 2
    with pytest.raises(TaylorGridError):
        g.backward(q, ws, torch.zeros((3, n), device=DEV), torch.zeros((n, 3), device=DEV))
