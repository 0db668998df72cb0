"""ctypes declarations of the C ABI in include/taylorgrid.h (argument marshalling only).

The library is the in-tree ``libtaylorgrid.so`` built by ``paper_2402_14415_amd.build``.
There is no fallback: if it is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtaylorgrid.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "taylorgrid.h")

TG_OK = 0
STATUS_NAMES = {0: "TG_OK", 1: "TG_ERR_INVALID_ARG", 2: "TG_ERR_UNSUPPORTED", 3: "TG_ERR_DEVICE",
                4: "TG_ERR_CAPACITY", 5: "TG_ERR_STATE"}
TG_F32, TG_BF16, TG_F16 = 0, 1, 2
TG_BWD_ACCUMULATE = 1
TG_ADAM_ZERO_GRAD = 1
TG_BWD_ADD_GRAD = 1
TG_BWD_PACKED = 2
TG_HESSIAN_SYMMETRIC, TG_HESSIAN_FULL = 0, 1
TG_QUERY_MAX_REQS = 32
TG_QUERY_MAX_GRIDS = 16


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("res", ctypes.c_int32 * 3), ("order", ctypes.c_int32),
                ("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3), ("storage", ctypes.c_int32),
                ("hessian", ctypes.c_int32), ("channels", ctypes.c_int32)]


class GridBuffers(ctypes.Structure):
    _fields_ = [("coeffs", ctypes.c_void_p), ("master", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p)]


class SdfObjective(ctypes.Structure):
    _fields_ = [("eik_weight", ctypes.c_float), ("surface_k", ctypes.c_float), ("tv_weight", ctypes.c_float)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float), ("step", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("pad_", ctypes.c_int32), ("n", ctypes.c_int64),
                ("q", ctypes.c_void_p), ("sdf", ctypes.c_void_p), ("normal", ctypes.c_void_p)]


class TaylorGridError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn} failed: {STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "tg_coeffs_per_vertex": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "tg_create": ([ctypes.POINTER(GridDesc), ctypes.POINTER(GridBuffers), ctypes.POINTER(_P)], ctypes.c_int),
    "tg_set_buffers": ([_P, ctypes.POINTER(GridBuffers)], ctypes.c_int),
    "tg_destroy": ([_P], ctypes.c_int),
    "tg_workspace_bytes": ([_P, ctypes.c_int64], ctypes.c_size_t),
    "tg_reduce_workspace_bytes": ([], ctypes.c_size_t),
    "tg_sort_queries": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tg_share_sort": ([_P, _P, _P, ctypes.c_int64, _P, ctypes.c_size_t], ctypes.c_int),
    "tg_forward": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P, _P], ctypes.c_int),
    "tg_forward_packed": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P], ctypes.c_int),
    "tg_sdf_loss": ([ctypes.c_int32, ctypes.c_int64, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P, _P,
                     ctypes.c_size_t, _P], ctypes.c_int),
    "tg_tv_loss": ([_P, ctypes.c_float, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tg_upsample": ([_P, _P, _P], ctypes.c_int),
    "tg_iou_counts": ([ctypes.c_int64, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tg_mesh_workspace_bytes": ([ctypes.POINTER(ctypes.c_int32)], ctypes.c_size_t),
    "tg_chamfer_workspace_bytes": ([ctypes.c_int64, ctypes.c_int64], ctypes.c_size_t),
    "tg_mesh": ([ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _P,
                 _P, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tg_chamfer": ([_P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tg_backward": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "tg_forward_sdf_loss": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P, ctypes.c_float, ctypes.c_float, _P, _P,
                             _P, _P, _P, _P], ctypes.c_int),
    "tg_backward_adam": ([_P, _P, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(AdamParams), _P,
                          ctypes.c_int32, _P], ctypes.c_int),
    "tg_train_step": ([_P, _P, _P, ctypes.c_int64, ctypes.POINTER(SdfObjective), ctypes.POINTER(AdamParams), _P, _P,
                       _P, ctypes.c_size_t, ctypes.POINTER(_P), _P], ctypes.c_int),
    "tg_train_step_sorted": ([_P, _P, _P, ctypes.c_int64, ctypes.POINTER(SdfObjective), ctypes.POINTER(AdamParams), _P,
                              _P, _P, ctypes.c_size_t, ctypes.POINTER(_P), _P], ctypes.c_int),
    "tg_composite": ([ctypes.c_int64, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                     ctypes.c_int),
    "tg_adam_step": ([_P, ctypes.POINTER(AdamParams), _P, _P, ctypes.c_size_t, ctypes.c_int32, _P], ctypes.c_int),
    "tg_query": ([ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(Request), ctypes.c_int32, _P], ctypes.c_int),
    "tg_sync_storage": ([_P, _P], ctypes.c_int),
    "tg_field_lattice": ([_P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "tg_sdf_loss_noalloc": ([ctypes.c_int32, ctypes.c_int64, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P,
                             _P], ctypes.c_int),
    "tg_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "tg_last_error": ([], ctypes.c_char_p),
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_14415_amd.build`")
            handle = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                fn = getattr(handle, name)
                fn.argtypes = args
                fn.restype = res
            _lib = handle
    return _lib


def check(fn_name, status):
    if status != TG_OK:
        detail = lib().tg_last_error().decode(errors="replace")
        raise TaylorGridError(fn_name, status, detail)


def call(fn_name, *args):
    """Call an entry point and raise TaylorGridError on a non-zero status."""
    st = getattr(lib(), fn_name)(*args)
    check(fn_name, st)
    return st


def declared_functions():
    """Names of the functions include/taylorgrid.h declares."""
    import re

    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tg_[a-z_]+)\s*\(", text)))
