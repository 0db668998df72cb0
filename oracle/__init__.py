"""FP64 CPU oracle of the TaylorGrid query path (arXiv 2402.14415, Sec. 3.1, Eq. 1-4).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's CPU-baseline
leg use it to check the GPU library; the GPU library never imports, links or calls it.  It
shares no code, header, table or constant with the GPU path.

Two independent implementations live here:
  * ``liboracle.so`` (``taylorgrid_oracle.c``): plain C, FP64, the definition written out
    step by step (cell query Eq. 2, corner Taylor polynomials Eq. 1/3, trilinear blend Eq. 4,
    and their exact derivatives), wrapped below with ctypes;
  * ``brute.py``: a NumPy brute force for tiny grids (matrix form of Eq. 1, adjoint by
    probing with unit coefficient vectors), used to cross-check the C oracle.

Parity status: every function is pinned by tests in ``tests/test_oracle_pins.py`` (library
routines, closed forms, invariants, finite differences, brute force); none is unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "taylorgrid_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over queries)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("res", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
    ]


def _bind(path):
    """Load a compiled oracle and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    gp = ctypes.POINTER(_Geom)
    lib.og_num_coeffs.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.og_num_coeffs.restype = ctypes.c_int32
    lib.og_exponents.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.og_exponents.restype = ctypes.c_int32
    lib.og_forward.argtypes = [gp, dp, dp, ctypes.c_int64, dp, dp, dp]
    lib.og_forward.restype = None
    lib.og_backward.argtypes = [gp, dp, dp, ctypes.c_int64, dp, dp, dp, dp]
    lib.og_backward.restype = None
    lib.og_sdf_loss.argtypes = [ctypes.c_int32, ctypes.c_int64, dp, dp, dp, ctypes.c_double, dp, dp, dp]
    lib.og_sdf_loss.restype = None
    lib.og_adam.argtypes = [ctypes.c_int64, dp, dp, dp, dp] + [ctypes.c_double] * 5 + [ctypes.c_int64]
    lib.og_adam.restype = ctypes.c_double
    return lib


def build_variant(source_text: str, out_dir: str) -> "ctypes.CDLL":
    """Compile an edited copy of the oracle source (used by tests that plant a mistake in
    the oracle to show that the pins catch it) and return the bound library."""
    src = os.path.join(out_dir, "variant.c")
    lib = os.path.join(out_dir, "libvariant.so")
    with open(src, "w") as fh:
        fh.write(source_text)
    with open(os.path.join(_HERE, "taylorgrid_oracle.h")) as fh:
        hdr = fh.read()
    with open(os.path.join(out_dir, "taylorgrid_oracle.h"), "w") as fh:
        fh.write(hdr)
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", lib, src, "-lm"], check=True, cwd=out_dir)
    return _bind(lib)


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            _lib = _bind(_LIB)
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Geometry:
    """A grid: ``res`` vertices per axis on the closed box [lo, hi], Taylor order ``order``."""

    def __init__(self, dim, res, order, lo, hi):
        self.dim = int(dim)
        self.res = tuple(int(r) for r in res)[: self.dim]
        self.order = int(order)
        self.lo = tuple(float(v) for v in lo)[: self.dim]
        self.hi = tuple(float(v) for v in hi)[: self.dim]
        assert self.dim in (2, 3) and len(self.res) == self.dim
        assert all(r >= 2 for r in self.res) and 0 <= self.order <= 4

    def _c(self):
        g = _Geom()
        g.dim = self.dim
        g.order = self.order
        for a in range(3):
            g.res[a] = self.res[a] if a < self.dim else 1
            g.lo[a] = self.lo[a] if a < self.dim else 0.0
            g.hi[a] = self.hi[a] if a < self.dim else 1.0
        return g

    @property
    def num_vertices(self):
        return int(np.prod(self.res))

    @property
    def num_coeffs(self):
        return num_coeffs(self.dim, self.order)

    @property
    def coeff_shape(self):
        """Array shape of the coefficient grid: (res_z, res_y, res_x, C) or (res_y, res_x, C)."""
        return tuple(reversed(self.res)) + (self.num_coeffs,)


def num_coeffs(dim, order, lib=None):
    return int((lib or _load()).og_num_coeffs(dim, order))


def exponents(dim, order):
    nc = num_coeffs(dim, order)
    out = np.zeros((nc, 3), dtype=np.int32)
    _load().og_exponents(dim, order, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out[:, :dim]


def forward(geom: Geometry, coeffs, q, want_grad=True, want_hess=False, lib=None):
    """Field value f[n], gradient [n, dim] and optionally Hessian [n, dim, dim] in FP64."""
    C = _f64(coeffs).reshape(-1)
    assert C.size == geom.num_vertices * geom.num_coeffs
    q = _f64(q).reshape(-1, geom.dim)
    n = q.shape[0]
    f = np.zeros(n)
    g = np.zeros((n, geom.dim)) if want_grad else None
    h = np.zeros((n, geom.dim, geom.dim)) if want_hess else None
    gc = geom._c()
    (lib or _load()).og_forward(ctypes.byref(gc), _ptr(C), _ptr(q), n, _ptr(f), _ptr(g), _ptr(h))
    out = [f]
    if want_grad:
        out.append(g)
    if want_hess:
        out.append(h)
    return out[0] if len(out) == 1 else tuple(out)


def backward(geom: Geometry, coeffs, q, gf=None, gg=None, want_dq=False, dcoeffs=None, lib=None):
    """Adjoint: returns (dC with the coefficient array's shape, dq or None)."""
    C = _f64(coeffs).reshape(-1)
    q = _f64(q).reshape(-1, geom.dim)
    n = q.shape[0]
    gf = None if gf is None else _f64(gf).reshape(n)
    gg = None if gg is None else _f64(gg).reshape(n, geom.dim)
    dC = np.zeros(C.size) if dcoeffs is None else _f64(dcoeffs).reshape(-1).copy()
    dq = np.zeros((n, geom.dim)) if want_dq else None
    gc = geom._c()
    (lib or _load()).og_backward(ctypes.byref(gc), _ptr(C), _ptr(q), n, _ptr(gf), _ptr(gg), _ptr(dC), _ptr(dq))
    return dC.reshape(geom.coeff_shape), dq


def sdf_loss(f, grad, d, w_eik, lib=None):
    """Returns (loss[3] = total, recon, eik), gf[n], gg[n, dim] or None."""
    f = _f64(f).reshape(-1)
    n = f.shape[0]
    d = _f64(d).reshape(n)
    dim = 0 if grad is None else int(np.asarray(grad).shape[-1])
    grad = None if grad is None else _f64(grad).reshape(n, dim)
    gf = np.zeros(n)
    gg = None if grad is None else np.zeros((n, dim))
    out = np.zeros(3)
    (lib or _load()).og_sdf_loss(dim, n, _ptr(f), _ptr(grad), _ptr(d), float(w_eik), _ptr(gf), _ptr(gg), _ptr(out))
    return out, gf, gg


def adam(theta, m, v, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, step=1, lib=None):
    """One Adam step on copies; returns (theta, m, v, sum(grad^2))."""
    theta = _f64(theta).copy()
    m = _f64(m).copy()
    v = _f64(v).copy()
    grad = _f64(grad)
    n = theta.size
    s = (lib or _load()).og_adam(n, _ptr(theta), _ptr(m), _ptr(v), _ptr(grad), lr, beta1, beta2, eps, weight_decay, int(step))
    return theta, m, v, float(s)


def threads():
    """OpenMP threads the oracle's query loops use."""
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
