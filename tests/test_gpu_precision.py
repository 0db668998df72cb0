"""Precision form: BF16 / FP16 coefficient storage with an FP32 master, FP32 accumulation.

Two errors per result, both against the FP64 oracle:
  * arithmetic error: oracle run on the *rounded* storage coefficients the kernels read;
    it must meet the FP32 tolerance (the kernels widen to FP32 and accumulate in FP32);
  * deployment error: oracle run on the FP32 master; it is the storage rounding itself,
    reported (and bounded by the rounding unit times the coefficient mass of a query).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.grid import TaylorGrid
from parity_util import TOL_GRAD, TOL_VALUE, FaceRule, geometry, nerr, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}  # half an ulp at 1, relative


def _rounded(C32, storage):
    """Round-to-nearest-even of FP32 coefficients to the storage format, computed here (FP16
    by NumPy's conversion, BF16 by rounding the FP32 bit pattern to its top 16 bits)."""
    if storage == "f16":
        return C32.astype(np.float16).astype(np.float64)
    u = C32.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _report(tag, grid, q64, f_gpu, master64):
    ref_m, _ = oracle.forward(geometry(grid), master64, q64)
    err = to_np(f_gpu) - ref_m
    print(f"{tag}: deployment SDF error vs oracle on the FP32 master: max {np.max(np.abs(err)):.3e} "
          f"rms {np.sqrt(np.mean(err ** 2)):.3e}")
    return err


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_precision_forward_backward_parity(storage):
    """A 40^3 K=2 grid holding the scene's Taylor projection plus noise (realistic scale:
    values O(1), gradients O(1), Hessians up to O(1/r))."""
    scene = synth.Scene(0)
    res = 40
    C32 = synth.scene_taylor_grid(scene, res, 2).numpy()
    rng = np.random.default_rng(21)
    C32 = (C32 + rng.normal(0, 0.05, size=C32.shape)).astype(np.float32)
    grid = TaylorGrid(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, storage=storage,
                      coeffs=torch.from_numpy(C32), device=DEV)
    Cr = _rounded(C32, storage)
    assert not np.array_equal(Cr, C32.astype(np.float64))  # storage really is rounded
    assert np.array_equal(grid.coeffs.float().cpu().double().numpy(), Cr)  # the device copy is that rounding
    q64, _ = synth.scene_batch(scene, 60000, seed=21, step=0)
    n = len(q64)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    gf64 = (rng.normal(size=n) / n).astype(np.float32).astype(np.float64)
    gg64 = (rng.normal(size=(n, 3)) / n).astype(np.float32).astype(np.float64)
    dq = grid.backward(q, ws, torch.tensor(gf64, dtype=torch.float32, device=DEV),
                       torch.tensor(gg64, dtype=torch.float32, device=DEV), want_dq=True)
    torch.cuda.synchronize()

    ref_f, ref_g = oracle.forward(geometry(grid), Cr, q64)
    rule = FaceRule(geometry(grid), Cr, q64)
    ef, eg = nerr(to_np(f), ref_f), rule.grad_err(to_np(g), ref_g)
    ref_dC, ref_dq = oracle.backward(geometry(grid), Cr, q64, gf64, gg64, want_dq=True)
    edc = rule.dC_err(to_np(grid.grad), ref_dC, gf64, gg64)
    edq = rule.dq_err(to_np(dq), ref_dq, gf64, gg64)
    print(f"{storage}: arithmetic error f {ef:.2e} grad {eg:.2e} dC {edc:.2e} dq {edq:.2e}")
    assert ef <= TOL_VALUE and eg <= TOL_GRAD and edc <= TOL_GRAD and edq <= TOL_GRAD

    err = _report(storage, grid, q64, f, C32.astype(np.float64))
    # |f(rounded) - f(master)| <= sum over the 8 corners of w_b * sum_a |m_a(d_b)| * |dC_a|,
    # and |dC_a| <= unit * |C_a|: bound by the rounding unit times the largest corner mass.
    h = 2.0 / (res - 1)
    mono = np.array([1, h, h, h, h * h / 2, h * h, h * h, h * h / 2, h * h, h * h / 2])
    mass = np.max(np.abs(C32).reshape(-1, 10) @ mono)
    assert np.max(np.abs(err)) <= UNIT[storage] * mass * 1.01


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_config2_full_size_sampled(storage):
    """256^3 vertices, K=2, 2^22 scene queries in the launch configuration of the training
    step.  The forward is checked on 2^16 sampled queries; the adjoint runs over all 2^22
    queries with upstream gradients that are zero except on 4096 sampled ones, so the
    oracle's adjoint of those 4096 alone is the exact expected gradient grid."""
    res, n = 256, 1 << 22
    rng = np.random.default_rng(22)
    C32 = (rng.standard_normal(size=(res, res, res, 10), dtype=np.float32) * np.float32(0.05))
    grid = TaylorGrid(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, storage=storage,
                      coeffs=torch.from_numpy(C32), device=DEV)
    scene = synth.Scene(0)
    q64, _ = synth.scene_batch(scene, n, seed=22, step=0)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    grid.sort(q, ws)
    f, g = grid.forward(q, ws)
    pick = np.sort(rng.choice(n, size=1 << 16, replace=False))
    sub = pick[:4096]
    gf64 = np.zeros(n)
    gg64 = np.zeros((n, 3))
    gf64[sub] = (rng.normal(size=len(sub)) * 1e-3).astype(np.float32)
    gg64[sub] = (rng.normal(size=(len(sub), 3)) * 1e-3).astype(np.float32)
    grid.backward(q, ws, torch.tensor(gf64, dtype=torch.float32, device=DEV),
                  torch.tensor(gg64, dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    Cr = _rounded(C32, storage)
    ref_f, ref_g = oracle.forward(geometry(grid), Cr, q64[pick])
    ef = nerr(to_np(f)[pick], ref_f)
    eg = FaceRule(geometry(grid), Cr, q64[pick]).grad_err(to_np(g)[pick], ref_g)
    ref_dC, _ = oracle.backward(geometry(grid), Cr, q64[sub], gf64[sub], gg64[sub])
    edc = FaceRule(geometry(grid), Cr, q64[sub]).dC_err(to_np(grid.grad), ref_dC, gf64[sub], gg64[sub])
    print(f"{storage} 256^3: arithmetic error f {ef:.2e} grad {eg:.2e} dC {edc:.2e}")
    assert ef <= TOL_VALUE and eg <= TOL_GRAD and edc <= TOL_GRAD
    _report(f"{storage} 256^3", grid, q64[pick], f[torch.from_numpy(pick).to(DEV)], C32.astype(np.float64))


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_storage_copy_made_by_the_library(storage):
    """The constructor's storage copy comes from tg_sync_storage: round to nearest even, FP16
    saturating at +-65504 (as after every Adam step), checked against the rounding computed
    here in NumPy.  The grid copies the caller's coefficients: a training step leaves the
    caller's tensor unchanged."""
    rng = np.random.default_rng(23)
    C32 = rng.normal(0, 0.05, size=(9, 10, 11, 10)).astype(np.float32)
    C32[0, 0, 0, :4] = [1e5, -7e4, 65519.0, 65520.0]  # beyond FP16's range, and the rounding edge
    C_dev = torch.from_numpy(C32).to(DEV)
    keep = C_dev.clone()
    grid = TaylorGrid(3, (11, 10, 9), 2, (-1.0,) * 3, (1.0,) * 3, storage=storage, coeffs=C_dev, device=DEV)
    torch.cuda.synchronize()
    expect = _rounded(np.clip(C32, -65504, 65504) if storage == "f16" else C32, storage)
    assert np.array_equal(grid.coeffs.float().cpu().double().numpy(), expect)
    assert grid.master.data_ptr() != C_dev.data_ptr()
    n = 4096
    q = torch.tensor(rng.uniform(-1, 1, size=(n, 3)), dtype=torch.float32, device=DEV)
    d = torch.tensor(rng.normal(size=n), dtype=torch.float32, device=DEV)
    ws = grid.workspace(n)
    grid.train_step(q, d, ws)
    torch.cuda.synchronize()
    assert torch.equal(C_dev, keep)
    assert not torch.equal(grid.master, keep)  # the step did update the grid's own copy
