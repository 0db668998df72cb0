"""The allocation-free loss entry point (tg_sdf_loss_noalloc) against tg_sdf_loss, through
the C ABI: the same inputs give the same loss and upstream gradients, on two calls in a row,
the second with a smaller input (the static scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2402_14415_amd import _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=n).astype(np.float32)
    d = f.copy()
    d[: n // 3] = rng.normal(size=n // 3).astype(np.float32)
    g = rng.normal(size=(n, 3)).astype(np.float32)
    g[:50] = 0.0
    return (torch.tensor(x, device=DEV) for x in (f, d, g))


def _call(fn, n, f, g, d, eik, k, ws=None):
    gf = torch.full((n,), float("nan"), device=DEV)
    gg = torch.full((n, 3), float("nan"), device=DEV)
    loss = torch.full((3,), float("nan"), dtype=torch.float64, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    if ws is None:
        _lib.call(fn, 3, n, _p(f), _p(g), _p(d), eik, k, _p(gf), _p(gg), _p(loss), stream)
    else:
        _lib.call(fn, 3, n, _p(f), _p(g), _p(d), eik, k, _p(gf), _p(gg), _p(loss), _p(ws), ws.numel(), stream)
    return loss, gf, gg


def test_noalloc_loss_matches_workspace_loss():
    ws = torch.empty(_lib.lib().tg_reduce_workspace_bytes(), dtype=torch.uint8, device=DEV)
    for n, seed, eik, k in ((1_000_003, 1, 0.1, 0.0), (70_001, 2, 0.3, 40.0)):
        f, d, g = _inputs(n, seed)
        a = _call("tg_sdf_loss_noalloc", n, f, g, d, eik, k)
        b = _call("tg_sdf_loss", n, f, g, d, eik, k, ws)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)  # same kernels, same block sums: bit for bit
        assert np.isfinite(a[0].cpu().numpy()).all()


def test_noalloc_loss_refuses_oversize_and_empty_is_zero():
    f = torch.zeros(1, device=DEV)
    loss = torch.full((3,), 7.0, dtype=torch.float64, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    st = _lib.lib().tg_sdf_loss_noalloc(3, (1 << 28) + 1, _p(f), None, _p(f), 0.0, 0.0, _p(f), None, _p(loss), stream)
    assert st == 4 and b"maximum" in _lib.lib().tg_last_error()
    _lib.call("tg_sdf_loss_noalloc", 3, 0, None, None, None, 0.0, 0.0, None, None, _p(loss), stream)
    torch.cuda.synchronize()
    assert torch.all(loss == 0.0)
