"""Differentiation form: torch.autograd through the HIP forward/adjoint, checked against
the oracle's adjoints and against finite differences of the GPU forward itself."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_14415_amd import synth
from paper_2402_14415_amd.autograd import taylor_grid
from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss
from parity_util import TOL_GRAD, FaceRule, geometry, nerr, nerr_cols, to_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_autograd_matches_oracle_adjoints():
    rng = np.random.default_rng(0)
    res = (21, 18, 25)
    C32 = rng.normal(0, 0.05, size=(25, 18, 21, 10)).astype(np.float32)
    grid = TaylorGrid(3, res, 2, (-1,) * 3, (1,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    grid.master.requires_grad_(True)
    n = 20000
    q64 = rng.uniform(-1.1, 1.1, size=(n, 3)).astype(np.float32).astype(np.float64)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV, requires_grad=True)
    a64 = rng.normal(size=n).astype(np.float32).astype(np.float64)  # seeded upstream weights
    b64 = rng.normal(size=(n, 3)).astype(np.float32).astype(np.float64)
    a = torch.tensor(a64, dtype=torch.float32, device=DEV)
    b = torch.tensor(b64, dtype=torch.float32, device=DEV)
    f, g = taylor_grid(grid, q)
    ((f * a).sum() + (g * b).sum()).backward()
    torch.cuda.synchronize()
    ref_dC, ref_dq = oracle.backward(geometry(grid), C32.astype(np.float64), q64, a64, b64, want_dq=True)
    rule = FaceRule(geometry(grid), C32.astype(np.float64), q64)
    assert rule.dC_err(to_np(grid.master.grad), ref_dC, a64, b64) <= TOL_GRAD
    assert rule.dq_err(to_np(q.grad), ref_dq, a64, b64) <= TOL_GRAD


def test_autograd_finite_differences_in_coefficients():
    """f and grad f are linear in C, so a central difference along a random direction
    equals the directional derivative up to FP32 rounding."""
    rng = np.random.default_rng(1)
    C32 = rng.normal(0, 0.05, size=(12, 12, 12, 10)).astype(np.float32)
    grid = TaylorGrid(3, (12, 12, 12), 2, (-1,) * 3, (1,) * 3, coeffs=torch.from_numpy(C32), device=DEV)
    grid.master.requires_grad_(True)
    n = 3000
    q = torch.tensor(rng.uniform(-1, 1, size=(n, 3)), dtype=torch.float32, device=DEV)
    w_f = torch.randn(n, device=DEV)
    w_g = torch.randn(n, 3, device=DEV)
    f, g = taylor_grid(grid, q)
    ((f * w_f).sum() + (g * w_g).sum()).backward()
    grad = grid.master.grad.detach().clone()
    direction = torch.randn_like(grid.master)
    ws = grid.workspace(n)

    def obj():
        grid.sort(q, ws)
        ff, gg = grid.forward(q, ws)
        return float(((ff * w_f).double().sum() + (gg * w_g).double().sum()).item())

    base = grid.master.detach().clone()
    with torch.no_grad():
        grid.master.copy_(base + direction)
        up = obj()
        grid.master.copy_(base - direction)
        dn = obj()
        grid.master.copy_(base)
    fd = (up - dn) / 2.0
    an = float((grad.double() * direction.double()).sum())
    assert abs(fd - an) <= 1e-4 * max(1.0, abs(an))


def test_sdf_training_reduces_loss_2d():
    """A few Adam steps on the disc target: the L1 + eikonal objective goes down."""
    C64, q64, d64 = synth.disc2d_inputs(res=64, order=2, n=65536, seed=0)
    grid = TaylorGrid(2, (64, 64), 2, (0, 0), (1, 1), coeffs=torch.from_numpy(C64.astype(np.float32)), device=DEV)
    q = torch.tensor(q64, dtype=torch.float32, device=DEV)
    d = torch.tensor(d64, dtype=torch.float32, device=DEV)
    ws = grid.workspace(q.shape[0])
    losses = []
    for _ in range(60):
        grid.sort(q, ws)
        f, g = grid.forward(q, ws)
        loss, gf, gg = sdf_loss(f, g, d, 0.1, ws)
        grid.backward(q, ws, gf, gg)
        grid.adam_step(ws, lr=1e-2)
        losses.append(float(loss[0]))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
