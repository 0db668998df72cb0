"""Host-side contract of the C ABI (no GPU needed: every call here fails validation before
anything is enqueued, or is a pure host function)."""
import ctypes
import os

import pytest

from paper_2402_14415_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libtaylorgrid.so not built")


def L():
    return _lib.lib()


def _desc(dim=3, res=(16, 16, 16), order=2, lo=(-1, -1, -1), hi=(1, 1, 1), storage=0):
    d = _lib.GridDesc()
    d.dim = dim
    d.order = order
    d.storage = storage
    for a in range(3):
        d.res[a] = res[a] if a < len(res) else 1
        d.lo[a] = lo[a] if a < len(lo) else 0
        d.hi[a] = hi[a] if a < len(hi) else 1
    return d


def _create(desc, bufs=None):
    h = ctypes.c_void_p()
    st = L().tg_create(ctypes.byref(desc), ctypes.byref(bufs) if bufs else None, ctypes.byref(h))
    return st, h


def test_exports_every_declared_symbol():
    names = _lib.declared_functions()
    assert "tg_forward" in names and "tg_backward" in names and "tg_query" in names
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


def test_coeffs_per_vertex():
    assert [L().tg_coeffs_per_vertex(3, k) for k in range(3)] == [1, 4, 10]
    assert [L().tg_coeffs_per_vertex(2, k) for k in range(3)] == [1, 3, 6]
    assert L().tg_coeffs_per_vertex(4, 1) == -1
    assert L().tg_coeffs_per_vertex(3, 3) == -1


def test_status_strings():
    for s in range(6):
        assert L().tg_status_string(s)
    assert L().tg_status_string(99) == b"unknown status"


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("order", 3), ("order", -1), ("storage", 7)])
def test_create_rejects_bad_descriptor(field, value):
    d = _desc()
    setattr(d, field, value)
    st, h = _create(d)
    assert st == 1 and not h.value
    assert L().tg_last_error()


def test_create_rejects_bad_geometry():
    d = _desc(res=(1, 16, 16))
    assert _create(d)[0] == 1
    d = _desc(lo=(0, 0, 0), hi=(0, 1, 1))
    assert _create(d)[0] == 1
    d = _desc(lo=(float("nan"), 0, 0))
    assert _create(d)[0] == 1
    assert L().tg_create(None, None, None) == 1


def test_create_rejects_inconsistent_buffers():
    b = _lib.GridBuffers()
    b.coeffs = 0x1000
    b.master = 0x2000
    assert _create(_desc(storage=0), b)[0] == 1  # f32: coeffs must equal master
    b.master = 0x1000
    assert _create(_desc(storage=1), b)[0] == 1  # bf16: must differ
    b.coeffs = 0x1004
    assert _create(_desc(storage=1), b)[0] == 1  # misaligned


def test_workspace_sizes_and_state_errors():
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    st, h = _create(_desc(res=(128, 128, 128)), b)
    assert st == 0
    try:
        n = 1 << 20
        ws = L().tg_workspace_bytes(h, n)
        # worst case: every query emits 8 bucket records of 16 bytes
        assert ws >= n * 8 * 16 + L().tg_reduce_workspace_bytes()
        assert L().tg_workspace_bytes(h, -1) == 0
        assert L().tg_workspace_bytes(None, 10) == 0
        fake = ctypes.c_void_p(0x100000)
        # a workspace that is too small is refused before any launch
        assert L().tg_sort_queries(h, fake, n, fake, ws - 1, None) == 4
        # forward without a sort of these queries is refused
        assert L().tg_forward(h, fake, n, fake, ws, fake, None, None) == 5
        # backward without grad buffer is refused
        assert L().tg_backward(h, fake, n, fake, ws, None, None, None, 0, None) == 1
        # misaligned workspace, negative n, NULL q
        assert L().tg_sort_queries(h, fake, n, ctypes.c_void_p(0x100010), ws, None) == 1
        assert L().tg_sort_queries(h, fake, -5, fake, ws, None) == 1
        assert L().tg_sort_queries(h, None, 10, fake, ws, None) == 1
        assert L().tg_sort_queries(h, fake, 1 << 29, fake, 1 << 40, None) == 4
        # adam needs all four buffers, and a valid step
        p = _lib.AdamParams(1e-2, 0.9, 0.999, 1e-8, 0.0, 1)
        assert L().tg_adam_step(h, ctypes.byref(p), None, fake, 1 << 20, 0, None) == 1
        # unknown flags
        assert L().tg_backward(h, fake, n, fake, ws, None, None, None, 4, None) == 1
    finally:
        assert L().tg_destroy(h) == 0


def test_share_sort_validation():
    """Each call departs from a valid set (same lattice, ws large enough for the receiving
    grid) in one argument; with no sort written anywhere every call is refused."""
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    fake = ctypes.c_void_p(0x100000)
    n = 4096
    hs = []
    try:
        for desc in (_desc(order=2), _desc(order=1), _desc(order=1, hi=(1, 1, 1.5)), _desc(order=1, res=(16, 16, 17))):
            st, h = _create(desc, b)
            assert st == 0
            hs.append(h)
        dens, col, other_box, other_res = hs
        ws_d, ws_c = L().tg_workspace_bytes(dens, n), L().tg_workspace_bytes(col, n)
        # the partial sums of split bricks grow with the coefficient count
        assert ws_d > ws_c
        # the sort-independent part of the layout is the same: the K=2 grid's workspace covers K=1
        assert L().tg_share_sort(col, dens, fake, n, fake, ws_d) == 5       # nothing sorted yet
        assert L().tg_share_sort(None, dens, fake, n, fake, ws_d) == 1
        assert L().tg_share_sort(col, None, fake, n, fake, ws_d) == 1
        assert L().tg_share_sort(other_box, dens, fake, n, fake, ws_d) == 1  # different hi
        assert L().tg_share_sort(other_res, dens, fake, n, fake, ws_d) == 1  # different res
        assert L().tg_share_sort(col, dens, fake, n, fake, ws_c - 1) == 4   # short workspace
        assert L().tg_share_sort(col, dens, fake, n, ctypes.c_void_p(0x100010), ws_d) == 1
        assert L().tg_share_sort(col, dens, None, n, fake, ws_d) == 1
        assert L().tg_share_sort(col, dens, fake, -1, fake, ws_d) == 1
        # a state error leaves the receiver unsorted
        assert L().tg_forward(col, fake, n, fake, ws_d, fake, None, None) == 5
    finally:
        for h in hs:
            assert L().tg_destroy(h) == 0


def test_adam_parameter_validation():
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    b.grad = 0x2000
    b.adam_m = 0x3000
    b.adam_v = 0x4000
    st, h = _create(_desc(), b)
    assert st == 0
    try:
        fake = ctypes.c_void_p(0x100000)
        for p in [_lib.AdamParams(1e-2, 0.9, 0.999, 1e-8, 0.0, 0),
                  _lib.AdamParams(float("nan"), 0.9, 0.999, 1e-8, 0.0, 1),
                  _lib.AdamParams(1e-2, 1.0, 0.999, 1e-8, 0.0, 1),
                  _lib.AdamParams(1e-2, 0.9, 0.999, -1.0, 0.0, 1)]:
            assert L().tg_adam_step(h, ctypes.byref(p), None, fake, 1 << 20, 0, None) == 1
        p = _lib.AdamParams(1e-2, 0.9, 0.999, 1e-8, 0.0, 1)
        assert L().tg_adam_step(h, ctypes.byref(p), None, fake, 16, 0, None) == 4  # scratch too small
        assert L().tg_adam_step(h, ctypes.byref(p), None, fake, 1 << 20, 8, None) == 1  # bad flag
    finally:
        L().tg_destroy(h)


def test_loss_validation():
    fake = ctypes.c_void_p(0x100000)
    big = L().tg_reduce_workspace_bytes()
    assert L().tg_sdf_loss(4, 10, fake, fake, fake, 0.1, 0.0, fake, fake, fake, fake, big, None) == 1
    assert L().tg_sdf_loss(3, 10, None, fake, fake, 0.1, 0.0, fake, fake, fake, fake, big, None) == 1
    assert L().tg_sdf_loss(3, 10, fake, fake, fake, 0.1, 0.0, fake, None, fake, fake, big, None) == 1
    assert L().tg_sdf_loss(3, 10, fake, fake, fake, float("inf"), 0.0, fake, fake, fake, fake, big, None) == 1
    assert L().tg_sdf_loss(3, 10, fake, fake, fake, 0.1, 0.0, fake, fake, fake, fake, 8, None) == 4
    # Eq. 7's k must be finite and non-negative
    assert L().tg_sdf_loss(3, 10, fake, fake, fake, 0.1, -1.0, fake, fake, fake, fake, big, None) == 1
    assert L().tg_sdf_loss(3, 10, fake, fake, fake, 0.1, float("nan"), fake, fake, fake, fake, big, None) == 1


def test_objective_validation():
    """TV, the fused adjoint's flags and the training step's objective: each call departs from
    a valid set in one argument and is refused before anything is enqueued."""
    fake = ctypes.c_void_p(0x100000)
    b = _lib.GridBuffers()
    b.coeffs = b.master = b.adam_m = b.adam_v = 0x1000
    st, h = _create(_desc(res=(16, 16, 16)), b)
    assert st == 0
    b2 = _lib.GridBuffers()
    b2.coeffs = b2.master = b2.adam_m = b2.adam_v = b2.grad = 0x1000
    st, hg = _create(_desc(res=(16, 16, 16)), b2)
    assert st == 0
    try:
        red = L().tg_reduce_workspace_bytes()
        # tg_tv_loss: needs master and grad, a finite weight, known flags, a reduction workspace
        assert L().tg_tv_loss(h, 1e-3, fake, 0, fake, red, None) == 1              # no grad buffer
        assert L().tg_tv_loss(None, 1e-3, fake, 0, fake, red, None) == 1
        assert L().tg_tv_loss(hg, float("inf"), fake, 0, fake, red, None) == 1
        assert L().tg_tv_loss(hg, 1e-3, None, 0, fake, red, None) == 1
        assert L().tg_tv_loss(hg, 1e-3, fake, 6, fake, red, None) == 1
        assert L().tg_tv_loss(hg, 1e-3, fake, 0, fake, red - 1, None) == 4
        assert L().tg_tv_loss(hg, 1e-3, fake, 0, ctypes.c_void_p(0x100010), red, None) == 1
        n = 1000
        ws = L().tg_workspace_bytes(hg, n)
        p = _lib.AdamParams(1e-2, 0.9, 0.999, 1e-8, 0.0, 1)
        # tg_backward_adam: TG_BWD_ADD_GRAD needs bufs.grad; unknown flags
        assert L().tg_backward_adam(h, fake, n, fake, ws, fake, None, ctypes.byref(p), None, 1, None) == 1
        assert L().tg_backward_adam(hg, fake, n, fake, ws, fake, None, ctypes.byref(p), None, 4, None) == 1
        # tg_train_step: objective required and finite, k >= 0, TV needs bufs.grad
        ok = _lib.SdfObjective(0.1, 0.0, 0.0)
        for obj, handle in ((None, hg), (_lib.SdfObjective(float("nan"), 0.0, 0.0), hg),
                            (_lib.SdfObjective(0.1, -2.0, 0.0), hg), (_lib.SdfObjective(0.1, 0.0, float("inf")), hg),
                            (_lib.SdfObjective(0.1, 0.0, 1e-3), h)):
            ref = ctypes.byref(obj) if obj is not None else None
            assert L().tg_train_step(handle, fake, fake, n, ref, ctypes.byref(p), fake, None, fake, ws, None, None) == 1
        # the valid objective only fails on the short workspace, before any launch
        assert L().tg_train_step(hg, fake, fake, n, ctypes.byref(ok), ctypes.byref(p), fake, None, fake, ws - 1,
                                 None, None) == 4
    finally:
        assert L().tg_destroy(h) == 0
        assert L().tg_destroy(hg) == 0


def test_composite_validation():
    """Argument errors of tg_composite come back before any launch (no GPU needed)."""
    fake = ctypes.c_void_p(0x100000)
    big = L().tg_reduce_workspace_bytes()

    # every call below changes one argument of a valid set to an invalid value
    def call(n_rays=4, ns=256, f=fake, c=fake, delta=fake, target=fake, loss=fake, g_f=fake, g_c=fake, ws=fake, wsb=big):
        return L().tg_composite(n_rays, ns, f, c, delta, target, None, loss, g_f, g_c, ws, wsb, None)

    assert call(ns=0) == 1 and call(ns=1025) == 1 and call(n_rays=-1) == 1
    assert call(f=None) == 1 and call(c=None) == 1 and call(delta=None) == 1
    assert call(target=fake, loss=None) == 1 and call(target=fake, g_c=None) == 1 and call(target=None) == 1
    assert call(ws=None) == 1 and call(ws=ctypes.c_void_p(0x100010)) == 1
    assert call(wsb=8) == 4
    assert call(n_rays=1 << 30, ns=1024) == 4  # more samples than the library takes


def test_query_validation():
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    st, h = _create(_desc(), b)
    assert st == 0
    try:
        hs = (ctypes.c_void_p * 1)(h.value)
        r = (_lib.Request * 1)()
        r[0].grid = 1
        r[0].n = 10
        r[0].q = r[0].sdf = 0x5000
        assert L().tg_query(hs, 1, r, 1, None) == 1  # grid index out of range
        r[0].grid = 0
        r[0].q = None
        assert L().tg_query(hs, 1, r, 1, None) == 1  # NULL q
        assert L().tg_query(hs, 1, r, 0, None) == 0  # empty batch is a no-op
        assert L().tg_query(hs, 1, r, -1, None) == 1
    finally:
        L().tg_destroy(h)


def test_quality_validation():
    """IoU, mesh and Chamfer: each call departs from a valid set in one argument."""
    fake = ctypes.c_void_p(0x100000)
    red = L().tg_reduce_workspace_bytes()
    assert L().tg_iou_counts(-1, fake, fake, fake, fake, red, None) == 1
    assert L().tg_iou_counts(10, None, fake, fake, fake, red, None) == 1
    assert L().tg_iou_counts(10, fake, fake, None, fake, red, None) == 1
    assert L().tg_iou_counts(10, fake, fake, fake, fake, red - 1, None) == 4
    n = (ctypes.c_int32 * 3)(9, 10, 11)
    lo = (ctypes.c_float * 3)(-1, -1, -1)
    hi = (ctypes.c_float * 3)(1, 1, 1)
    wsb = L().tg_mesh_workspace_bytes(n)
    assert wsb >= 8 * 9 * 10 * 4
    assert L().tg_mesh_workspace_bytes((ctypes.c_int32 * 3)(1, 10, 11)) == 0
    assert L().tg_mesh_workspace_bytes((ctypes.c_int32 * 3)(65536, 65536, 65536)) == 0  # over 2^28 cells
    assert L().tg_mesh((ctypes.c_int32 * 3)(1, 10, 11), lo, hi, fake, fake, 10, fake, fake, wsb, None) == 1
    assert L().tg_mesh((ctypes.c_int32 * 3)(4097, 4097, 4097), lo, hi, fake, fake, 10, fake, fake, 1 << 40,
                       None) == 4
    assert L().tg_mesh(n, lo, lo, fake, fake, 10, fake, fake, wsb, None) == 1          # empty box
    assert L().tg_mesh(n, lo, hi, None, fake, 10, fake, fake, wsb, None) == 1
    assert L().tg_mesh(n, lo, hi, fake, None, 10, fake, fake, wsb, None) == 1        # no output buffer
    assert L().tg_mesh(n, lo, hi, fake, fake, -1, fake, fake, wsb, None) == 1
    assert L().tg_mesh(n, lo, hi, fake, fake, 10, None, fake, wsb, None) == 1
    assert L().tg_mesh(n, lo, hi, fake, fake, 10, fake, fake, wsb - 1, None) == 4
    assert L().tg_chamfer(fake, 0, fake, 5, 1, fake, fake, red, None) == 1
    assert L().tg_chamfer(fake, 5, None, 5, 1, fake, fake, red, None) == 1
    assert L().tg_chamfer(fake, 5, fake, 5, 3, fake, fake, 1 << 30, None) == 1  # norm 1 or 2 only
    chb = L().tg_chamfer_workspace_bytes(5, 5)
    assert chb >= red and L().tg_chamfer_workspace_bytes(0, 5) == 0
    assert L().tg_chamfer_workspace_bytes(1_000_000, 100_000) > L().tg_chamfer_workspace_bytes(1_000_000, 2048)
    assert L().tg_chamfer(fake, 5, fake, 5, 2, fake, fake, chb - 1, None) == 4


def test_full_hessian_layout_validation():
    """The full-Hessian layout: order 2 only, a known layout code, 13 coefficients in 3D (a
    larger workspace), and the serving call refuses it."""
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    d = _desc(order=2)
    d.hessian = 1
    st, h = _create(d, b)
    assert st == 0
    d2 = _desc(order=2)
    st, hs = _create(d2, b)
    assert st == 0
    try:
        assert L().tg_workspace_bytes(h, 1 << 16) > L().tg_workspace_bytes(hs, 1 << 16)
        req = (_lib.Request * 1)()
        req[0].grid = 0
        req[0].n = 10
        req[0].q = req[0].sdf = 0x100000
        grids = (ctypes.c_void_p * 1)(h.value)
        assert L().tg_query(grids, 1, req, 1, None) == 2  # TG_ERR_UNSUPPORTED
    finally:
        assert L().tg_destroy(h) == 0
        assert L().tg_destroy(hs) == 0
    for order, layout in ((1, 1), (0, 1), (2, 2), (2, -1)):
        d = _desc(order=order)
        d.hessian = layout
        st, _ = _create(d, b)
        assert st == 1, (order, layout)


def test_channels_validation():
    """Three channels need order 1 and the symmetric layout; 1 and 3 are the only counts; a
    three-channel grid is refused by serving, and its adjoint takes g_f only."""
    b = _lib.GridBuffers()
    b.coeffs = b.master = b.grad = 0x1000
    for order, ch, hess in ((2, 3, 0), (0, 3, 0), (1, 2, 0), (1, -1, 0)):
        d = _desc(order=order)
        d.channels = ch
        d.hessian = hess
        st, _ = _create(d, b)
        assert st == 1, (order, ch)
    d = _desc(order=1)
    d.channels = 3
    st, h = _create(d, b)
    assert st == 0
    d1 = _desc(order=1)
    st, h1 = _create(d1, b)
    assert st == 0
    try:
        n = 1000
        assert L().tg_workspace_bytes(h, n) > L().tg_workspace_bytes(h1, n)  # 12 coefficients, not 4
        req = (_lib.Request * 1)()
        req[0].grid, req[0].n = 0, 10
        req[0].q = req[0].sdf = 0x100000
        assert L().tg_query((ctypes.c_void_p * 1)(h.value), 1, req, 1, None) == 2
        fake = ctypes.c_void_p(0x100000)
        ws = L().tg_workspace_bytes(h, n)
        # the adjoint of a three-channel grid takes neither g_grad nor dq, and needs g_f
        assert L().tg_backward(h, fake, n, fake, ws, fake, fake, None, 0, None) == 2
        assert L().tg_backward(h, fake, n, fake, ws, fake, None, fake, 0, None) == 2
        assert L().tg_backward(h, fake, n, fake, ws, None, None, None, 0, None) == 1
        # tg_forward without a grad_f output only
        assert L().tg_forward(h, fake, n, fake, ws, fake, fake, None) == 2
    finally:
        assert L().tg_destroy(h) == 0
        assert L().tg_destroy(h1) == 0


def test_packed_layout_validation():
    """tg_forward_packed and TG_BWD_PACKED: a 16-byte aligned [n][4] array, g_grad NULL,
    single-channel grids only.  A call that passes validation stops at the missing sort
    (TG_ERR_STATE); nothing is enqueued."""
    fake = ctypes.c_void_p(0x100000)
    odd = ctypes.c_void_p(0x100004)  # 4-byte but not 16-byte aligned
    b = _lib.GridBuffers()
    b.coeffs = b.master = b.grad = b.adam_m = b.adam_v = 0x1000
    st, h = _create(_desc(order=2), b)
    assert st == 0
    d3 = _desc(order=1)
    d3.channels = 3
    st, hc = _create(d3, b)
    assert st == 0
    try:
        n = 1000
        ws, wsc = L().tg_workspace_bytes(h, n), L().tg_workspace_bytes(hc, n)
        P = _lib.TG_BWD_PACKED
        assert L().tg_forward_packed(h, fake, n, fake, ws, fake, None) == 5
        assert L().tg_forward_packed(h, fake, n, fake, ws, odd, None) == 1
        assert L().tg_forward_packed(h, fake, n, fake, ws, None, None) == 1
        assert L().tg_forward_packed(hc, fake, n, fake, wsc, fake, None) == 2
        assert L().tg_forward_packed(None, fake, n, fake, ws, fake, None) == 1
        for flags in (P, P | _lib.TG_BWD_ACCUMULATE):
            assert L().tg_backward(h, fake, n, fake, ws, fake, None, None, flags, None) == 5
            assert L().tg_backward(h, fake, n, fake, ws, fake, None, fake, flags, None) == 5  # with dq
            assert L().tg_backward(h, fake, n, fake, ws, fake, fake, None, flags, None) == 1  # g_grad given
            assert L().tg_backward(h, fake, n, fake, ws, odd, None, None, flags, None) == 1
            assert L().tg_backward(h, fake, n, fake, ws, None, None, None, flags, None) == 1
            assert L().tg_backward(hc, fake, n, fake, wsc, fake, None, None, flags, None) == 2
        assert L().tg_backward(h, fake, n, fake, ws, fake, None, None, 4, None) == 1  # unknown flag
        p = _lib.AdamParams(1e-2, 0.9, 0.999, 1e-8, 0.0, 1)
        for flags in (P, P | _lib.TG_BWD_ADD_GRAD):
            assert L().tg_backward_adam(h, fake, n, fake, ws, fake, None, ctypes.byref(p), None, flags, None) == 5
            assert L().tg_backward_adam(h, fake, n, fake, ws, fake, fake, ctypes.byref(p), None, flags, None) == 1
            assert L().tg_backward_adam(h, fake, n, fake, ws, odd, None, ctypes.byref(p), None, flags, None) == 1
    finally:
        assert L().tg_destroy(h) == 0
        assert L().tg_destroy(hc) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_sorted_query_count_is_capped(dim):
    """A query makes up to 2^dim sort records with int32 positions, so the sorted calls
    accept n <= (2^31 - 1) >> dim and refuse one more before anything is enqueued."""
    st, h = _create(_desc(dim=dim, res=(16,) * dim))
    assert st == 0
    cap = (2 ** 31 - 1) >> dim
    assert L().tg_workspace_bytes(h, cap) > 0
    assert L().tg_workspace_bytes(h, cap + 1) == 0
    big = 1 << 40  # a fake workspace size: validation fails before it is used
    st = L().tg_sort_queries(h, ctypes.c_void_p(0x1000), cap + 1, ctypes.c_void_p(0x100000), big, None)
    assert st == 4 and b"2^31" in L().tg_last_error()
    L().tg_destroy(h)


def test_sync_storage_validation():
    st, h = _create(_desc(storage=1))
    assert st == 0
    assert L().tg_sync_storage(None, None) == 1
    assert L().tg_sync_storage(h, None) == 1  # 16-bit storage without buffers
    L().tg_destroy(h)
    st, h = _create(_desc(storage=0))
    assert L().tg_sync_storage(h, None) == 0  # FP32 storage: nothing to do, nothing enqueued
    L().tg_destroy(h)


def test_field_lattice_validation():
    """tg_field_lattice: 3D single-channel symmetric grids, 1 <= s <= 64, fewer than 2^31
    points; refused before anything is enqueued."""
    b = _lib.GridBuffers()
    b.coeffs = b.master = 0x1000
    fake = ctypes.c_void_p(0x2000)
    st, h = _create(_desc(), b)
    assert st == 0
    assert L().tg_field_lattice(None, 2, fake, None) == 1
    assert L().tg_field_lattice(h, 0, fake, None) == 1
    assert L().tg_field_lattice(h, 65, fake, None) == 1
    assert L().tg_field_lattice(h, 2, None, None) == 1
    L().tg_destroy(h)
    st, h = _create(_desc(res=(2000, 2000, 2000)), b)
    assert L().tg_field_lattice(h, 1, fake, None) == 4  # 8e9 points
    L().tg_destroy(h)
    st, h = _create(_desc(dim=2, res=(16, 16)), b)
    assert L().tg_field_lattice(h, 2, fake, None) == 2
    L().tg_destroy(h)
