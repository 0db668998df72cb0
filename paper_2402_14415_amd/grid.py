"""Python surface of the TaylorGrid library: a grid that owns its device tensors.

Every call marshals torch tensors into the C ABI (include/taylorgrid.h) and enqueues the
HIP kernels on torch's current stream; no arithmetic of the method runs in Python.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

_STORAGE = {"f32": (_lib.TG_F32, torch.float32), "bf16": (_lib.TG_BF16, torch.bfloat16),
            "f16": (_lib.TG_F16, torch.float16)}


def coeffs_per_vertex(dim: int, order: int) -> int:
    c = _lib.lib().tg_coeffs_per_vertex(dim, order)
    if c < 0:
        raise ValueError(f"unsupported dim={dim} order={order}")
    return int(c)


_sort_generations = iter(range(1, 1 << 62))


def _new_sort(q, ws):
    """Record that ws now holds the sort of q; any earlier sort in ws is superseded (the
    library checks the same rule by the workspace's address)."""
    gen = next(_sort_generations)
    ws._tg_sort_generation = gen
    return (q, ws, gen)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(name, t, dtype, device, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


class TaylorGrid:
    """A dense TaylorGrid (arXiv 2402.14415, Sec. 3.1) with its optimiser state on one GPU.

    Tensors (all [res_z, res_y, res_x, C] or [res_y, res_x, C]):
      master  FP32 coefficients (the optimised parameters)
      coeffs  storage copy read by the kernels (== master for f32 storage)
      grad    FP32 gradient written by ``backward``
      adam_m, adam_v  FP32 Adam moments
    """

    def __init__(self, dim, res, order, lo, hi, storage="f32", device="cuda", coeffs=None, optimizer=True,
                 hessian="symmetric", channels=1):
        self.dim = int(dim)
        res = [int(r) for r in (res if hasattr(res, "__len__") else [res] * self.dim)]
        self.res = tuple(res[: self.dim])
        self.order = int(order)
        lo = [float(v) for v in (lo if hasattr(lo, "__len__") else [lo] * self.dim)]
        hi = [float(v) for v in (hi if hasattr(hi, "__len__") else [hi] * self.dim)]
        self.lo = tuple(lo[: self.dim])
        self.hi = tuple(hi[: self.dim])
        self.storage = storage
        st, sdt = _STORAGE[storage]
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        if hessian not in ("symmetric", "full"):
            raise ValueError(f"unknown Hessian layout {hessian!r}")
        self.hessian = hessian
        if channels not in (1, 3):
            raise ValueError("channels must be 1 or 3")
        self.channels = channels
        if hessian == "full":
            self.C = 1 + self.dim + self.dim * self.dim
        elif channels == 3:
            self.C = 3 * (1 + self.dim)
        else:
            self.C = coeffs_per_vertex(self.dim, self.order)
        self.shape = tuple(reversed(self.res)) + (self.C,)

        # the grid owns its master: a copy, never a view of the caller's tensor
        master = torch.zeros(self.shape, dtype=torch.float32, device=self.device)
        if coeffs is not None:
            master.copy_(torch.as_tensor(coeffs).reshape(self.shape))
        self.master = master
        self.coeffs = master if storage == "f32" else torch.empty(self.shape, dtype=sdt, device=self.device)
        self.grad = torch.zeros_like(master)
        if optimizer:
            self.adam_m = torch.zeros_like(master)
            self.adam_v = torch.zeros_like(master)
        else:
            self.adam_m = self.adam_v = None
        self.step_count = 0

        desc = _lib.GridDesc()
        desc.dim = self.dim
        desc.order = self.order
        desc.storage = st
        desc.hessian = _lib.TG_HESSIAN_FULL if hessian == "full" else _lib.TG_HESSIAN_SYMMETRIC
        desc.channels = channels
        for a in range(3):
            desc.res[a] = self.res[a] if a < self.dim else 1
            desc.lo[a] = self.lo[a] if a < self.dim else 0.0
            desc.hi[a] = self.hi[a] if a < self.dim else 1.0
        self._desc = desc
        handle = ctypes.c_void_p()
        _lib.call("tg_create", ctypes.byref(desc), ctypes.byref(self._buffers()), ctypes.byref(handle))
        self._h = handle
        self._sorted = None  # (q tensor, ws tensor, sort generation) of the last sort
        self.sync_storage()

    # ------------------------------------------------------------------ plumbing
    def _buffers(self, grad=None):
        b = _lib.GridBuffers()
        b.coeffs = self.coeffs.data_ptr()
        b.master = self.master.data_ptr()
        b.grad = (self.grad if grad is None else grad).data_ptr()
        b.adam_m = self.adam_m.data_ptr() if self.adam_m is not None else None
        b.adam_v = self.adam_v.data_ptr() if self.adam_v is not None else None
        return b

    def rebind(self, grad=None):
        """Point the handle at the current tensors (after replacing one of them)."""
        _lib.call("tg_set_buffers", self._h, ctypes.byref(self._buffers(grad)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib.lib().tg_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def sync_storage(self):
        """Refresh the storage copy from the master in the library (round to nearest even,
        FP16 saturating at +-65504); call it after changing ``master`` outside the library."""
        _lib.call("tg_sync_storage", self._h, _stream(self.device))

    def workspace_bytes(self, n):
        return int(_lib.lib().tg_workspace_bytes(self._h, int(n)))

    def workspace(self, n):
        """A device workspace for n queries (sort + reduction scratch)."""
        return torch.empty(self.workspace_bytes(n), dtype=torch.uint8, device=self.device)

    def _q(self, q):
        _check_tensor("q", q, torch.float32, self.device)
        if q.dim() != 2 or q.shape[1] != self.dim:
            raise ValueError(f"q must be [n, {self.dim}]")
        return q.shape[0]

    # ------------------------------------------------------------------ hot path
    def sort(self, q, ws):
        n = self._q(q)
        _lib.call("tg_sort_queries", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _stream(self.device))
        self._sorted = _new_sort(q, ws)

    def share_sort(self, other, q, ws):
        """Reuse the sort of q that ``other`` (a grid of the same dim, res, lo and hi) holds in ws."""
        n = self._q(q)
        _lib.call("tg_share_sort", self._h, other._h, _ptr(q), n, _ptr(ws), ws.numel())
        self._sorted = other._sorted

    def ensure_sorted(self, q, ws):
        s = self._sorted
        if s is None or s[0] is not q or s[1] is not ws or getattr(ws, "_tg_sort_generation", None) != s[2]:
            self.sort(q, ws)

    def forward(self, q, ws, want_grad=True, out=None):
        """f [n] and grad f [n, dim] (or None); a three-channel grid gives f [3, n] and no grad f."""
        n = self._q(q)
        if self.channels == 3:
            want_grad = False
        if out is None:
            f = torch.empty((n,) if self.channels == 1 else (3, n), dtype=torch.float32, device=self.device)
            g = torch.empty((n, self.dim), dtype=torch.float32, device=self.device) if want_grad else None
        else:
            f, g = out
        _check_tensor("f", f, torch.float32, self.device, self.channels * n)
        if g is not None:
            _check_tensor("grad_f", g, torch.float32, self.device, n * self.dim)
        _lib.call("tg_forward", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _ptr(f), _ptr(g), _stream(self.device))
        return f, g

    def forward_packed(self, q, ws, out=None):
        """f and grad f of each query in one 16-byte row: a [n, 4] tensor (f, grad f; in 2D
        the last column is 0).  ``out[:, 0]`` and ``out[:, 1:1 + dim]`` are views of f and
        grad f; ``backward(..., packed=...)`` takes upstream gradients in the same layout."""
        n = self._q(q)
        fg = torch.empty((n, 4), dtype=torch.float32, device=self.device) if out is None else out
        _check_tensor("out", fg, torch.float32, self.device, 4 * n)
        _lib.call("tg_forward_packed", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _ptr(fg), _stream(self.device))
        return fg

    def _upstream(self, n, g_f, g_grad, packed):
        """Checks the upstream gradients; returns (g_f pointer tensor, g_grad, flag bits)."""
        if packed is not None:
            if g_f is not None or g_grad is not None:
                raise ValueError("pass either packed or g_f / g_grad")
            _check_tensor("packed", packed, torch.float32, self.device, 4 * n)
            return packed, None, _lib.TG_BWD_PACKED
        if g_f is not None:
            _check_tensor("g_f", g_f, torch.float32, self.device, self.channels * n)
        if g_grad is not None:
            _check_tensor("g_grad", g_grad, torch.float32, self.device, n * self.dim)
        return g_f, g_grad, 0

    def backward(self, q, ws, g_f=None, g_grad=None, want_dq=False, accumulate=False, grad_out=None, dq_out=None,
                 packed=None):
        """Writes (or accumulates) dL/dC into ``grad`` (or ``grad_out``); returns dq or None.
        ``packed`` ([n, 4], the layout of ``forward_packed``) replaces g_f and g_grad."""
        n = self._q(q)
        g_f, g_grad, pflag = self._upstream(n, g_f, g_grad, packed)
        dq = None
        if want_dq:
            dq = dq_out if dq_out is not None else torch.empty((n, self.dim), dtype=torch.float32, device=self.device)
        flags = (_lib.TG_BWD_ACCUMULATE if accumulate else 0) | pflag
        if grad_out is not None:
            _check_tensor("grad_out", grad_out, torch.float32, self.device, self.master.numel())
            self.rebind(grad=grad_out)
        try:
            _lib.call("tg_backward", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _ptr(g_f), _ptr(g_grad), _ptr(dq),
                      flags, _stream(self.device))
        finally:
            if grad_out is not None:
                self.rebind()
        return dq

    def forward_sdf_loss(self, q, ws, d, eik_weight, g_f=None, g_grad=None, loss=None, eikonal=True, f_out=None,
                         grad_out=None, surface_k=0.0):
        """Forward and SDF loss in one pass: returns (loss float64[3], g_f, g_grad or None);
        ``surface_k`` is Eq. 7's k (0: unweighted L1).
        ``eikonal=False`` drops the eikonal term; f_out / grad_out optionally receive f and
        grad f."""
        n = self._q(q)
        _check_tensor("d", d, torch.float32, self.device, n)
        g_f = torch.empty(n, dtype=torch.float32, device=self.device) if g_f is None else g_f
        _check_tensor("g_f", g_f, torch.float32, self.device, n)
        if eikonal:
            if g_grad is None:
                g_grad = torch.empty((n, self.dim), dtype=torch.float32, device=self.device)
            _check_tensor("g_grad", g_grad, torch.float32, self.device, n * self.dim)
        else:
            g_grad = None
        loss = torch.empty(3, dtype=torch.float64, device=self.device) if loss is None else loss
        _check_tensor("loss", loss, torch.float64, self.device, 3)
        for name, t, k in (("f_out", f_out, n), ("grad_out", grad_out, n * self.dim)):
            if t is not None:
                _check_tensor(name, t, torch.float32, self.device, k)
        _lib.call("tg_forward_sdf_loss", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _ptr(d), float(eik_weight),
                  float(surface_k), _ptr(g_f), _ptr(g_grad), _ptr(loss), _ptr(f_out), _ptr(grad_out),
                  _stream(self.device))
        return loss, g_f, g_grad

    def _adam_params(self, lr, betas, eps, weight_decay, step):
        if self.adam_m is None:
            raise RuntimeError("grid was created without optimiser state")
        self.step_count = self.step_count + 1 if step is None else int(step)
        return _lib.AdamParams(lr, betas[0], betas[1], eps, weight_decay, self.step_count)

    def backward_adam(self, q, ws, g_f=None, g_grad=None, lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0,
                      grad_norm_sq=None, step=None, add_grad=False, packed=None):
        """Adjoint and Adam step in one pass (``grad`` is not written); grad_norm_sq
        (device float64 [1]) receives sum(dC^2).  ``add_grad`` adds the gradient already in
        ``grad`` (e.g. the TV term's) to the adjoint before the update.  ``packed`` ([n, 4],
        the layout of ``forward_packed``) replaces g_f and g_grad."""
        n = self._q(q)
        g_f, g_grad, pflag = self._upstream(n, g_f, g_grad, packed)
        if grad_norm_sq is not None:
            _check_tensor("grad_norm_sq", grad_norm_sq, torch.float64, self.device)
        p = self._adam_params(lr, betas, eps, weight_decay, step)
        _lib.call("tg_backward_adam", self._h, _ptr(q), n, _ptr(ws), ws.numel(), _ptr(g_f), _ptr(g_grad),
                  ctypes.byref(p), _ptr(grad_norm_sq), (_lib.TG_BWD_ADD_GRAD if add_grad else 0) | pflag,
                  _stream(self.device))

    def upsample_from(self, coarse):
        """Start this grid (same box) from the field of ``coarse``: value, gradient and Hessian
        of the coarse field at this grid's vertices, truncated to this grid's order; the Adam
        moments are zeroed and the step count restarts."""
        _lib.call("tg_upsample", coarse._h, self._h, _stream(self.device))
        self.step_count = 0

    def tv_loss(self, weight, ws, accumulate=False, loss=None):
        """TV of the master coefficients (device float64 [1]); writes (or adds) weight * dTV/dC
        into ``grad``."""
        loss = torch.empty(1, dtype=torch.float64, device=self.device) if loss is None else loss
        _check_tensor("loss", loss, torch.float64, self.device)
        _lib.call("tg_tv_loss", self._h, float(weight), _ptr(loss), _lib.TG_BWD_ACCUMULATE if accumulate else 0,
                  _ptr(ws), ws.numel(), _stream(self.device))
        return loss

    def twin(self):
        """A second handle on the same tensors (coefficients, gradient, moments), with its own
        record of a sort: a training loop can sort the next batch into a second workspace with
        the twin while this grid steps on the current one (``train_step(presorted=True)``)."""
        import copy

        t = copy.copy(self)
        handle = ctypes.c_void_p()
        _lib.call("tg_create", ctypes.byref(self._desc), ctypes.byref(self._buffers()), ctypes.byref(handle))
        t._h = handle
        t._sorted = None
        return t

    def train_step(self, q, d, ws, eik_weight=0.1, lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0,
                   loss=None, grad_norm_sq=None, step=None, stage_events=None, surface_k=0.0, tv_weight=0.0,
                   presorted=False):
        """One SDF-fitting step (sort, forward + loss, adjoint + Adam) in one call; returns the
        loss (device float64 [3]: total, weighted L1 mean, eikonal mean; with a TV term [4],
        the TV value last).  ``surface_k`` is Eq. 7's k (0: unweighted), ``tv_weight`` the TV
        term's weight (0: none; else ``grad`` holds the TV gradient).  stage_events: optional
        three recorded torch.cuda.Events, re-recorded after each stage (for timing).  With
        ``presorted`` the step reuses the sort of (q, ws) that ``sort`` wrote (tg_train_step_sorted)."""
        n = self._q(q)
        _check_tensor("d", d, torch.float32, self.device, n)
        nl = 4 if tv_weight != 0.0 else 3
        loss = torch.empty(nl, dtype=torch.float64, device=self.device) if loss is None else loss
        _check_tensor("loss", loss, torch.float64, self.device, nl)
        if grad_norm_sq is not None:
            _check_tensor("grad_norm_sq", grad_norm_sq, torch.float64, self.device)
        p = self._adam_params(lr, betas, eps, weight_decay, step)
        evs = None
        if stage_events is not None:
            if len(stage_events) != 3:
                raise ValueError("stage_events must hold three events")
            evs = (ctypes.c_void_p * 3)(*[e.cuda_event for e in stage_events])
        obj = _lib.SdfObjective(eik_weight, surface_k, tv_weight)
        _lib.call("tg_train_step_sorted" if presorted else "tg_train_step", self._h, _ptr(q), _ptr(d), n,
                  ctypes.byref(obj), ctypes.byref(p), _ptr(loss), _ptr(grad_norm_sq), _ptr(ws), ws.numel(), evs,
                  _stream(self.device))
        if not presorted:
            self._sorted = _new_sort(q, ws)
        return loss

    def adam_step(self, ws, lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0, grad_norm_sq=None,
                  zero_grad=False, step=None):
        """One fused Adam step; grad_norm_sq (device float64 [1]) receives sum(grad^2)."""
        p = self._adam_params(lr, betas, eps, weight_decay, step)
        if grad_norm_sq is not None:
            _check_tensor("grad_norm_sq", grad_norm_sq, torch.float64, self.device)
        flags = _lib.TG_ADAM_ZERO_GRAD if zero_grad else 0
        _lib.call("tg_adam_step", self._h, ctypes.byref(p), _ptr(grad_norm_sq), _ptr(ws), ws.numel(), flags,
                  _stream(self.device))


def sdf_loss(f, grad_f, d, eik_weight, ws, g_f=None, g_grad=None, loss=None, surface_k=0.0):
    """L1 (weighted by Eq. 7 with k = surface_k; 0 = unweighted) + eikonal SDF objective;
    returns (loss float64[3] on device, g_f, g_grad)."""
    n = f.numel()
    dev = f.device
    dim = grad_f.shape[1] if grad_f is not None else 3
    g_f = torch.empty(n, dtype=torch.float32, device=dev) if g_f is None else g_f
    if grad_f is not None and g_grad is None:
        g_grad = torch.empty((n, dim), dtype=torch.float32, device=dev)
    loss = torch.empty(3, dtype=torch.float64, device=dev) if loss is None else loss
    _check_tensor("f", f, torch.float32, dev)
    _check_tensor("d", d, torch.float32, dev, n)
    if grad_f is not None:
        _check_tensor("grad_f", grad_f, torch.float32, dev, n * dim)
    _lib.call("tg_sdf_loss", dim, n, _ptr(f), _ptr(grad_f), _ptr(d), float(eik_weight), float(surface_k), _ptr(g_f),
              _ptr(g_grad) if grad_f is not None else None, _ptr(loss), _ptr(ws), ws.numel(), _stream(dev))
    return loss, g_f, g_grad


def query(grids, requests, stream=None):
    """Serve a batch: ``requests`` is a list of (grid index, q, sdf_out, normal_out or None)."""
    if not requests:
        return
    dev = requests[0][1].device
    hs = (ctypes.c_void_p * len(grids))(*[g.handle.value for g in grids])
    reqs = (_lib.Request * len(requests))()
    for i, (gi, q, sdf, normal) in enumerate(requests):
        reqs[i].grid = gi
        reqs[i].n = q.shape[0]
        reqs[i].q = q.data_ptr() if q.numel() else None
        reqs[i].sdf = sdf.data_ptr() if sdf.numel() else None
        reqs[i].normal = normal.data_ptr() if (normal is not None and normal.numel()) else None
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(dev)
    _lib.call("tg_query", hs, len(grids), reqs, len(requests), s)
