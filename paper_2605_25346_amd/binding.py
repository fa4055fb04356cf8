"""ctypes binding of libdiffreach.so: the C-ABI entry points under the same names.

Only argument marshalling happens here; every step of the bound computation runs
in the library's HIP kernels.  Importing this module does not touch the GPU.  The
library must have been built (``paper_2605_25346_amd.build.build()``); a missing
library is an error, never a silent fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdiffreach.so")

# Status codes and per-result bits (mirrors include/diffreach.h)
DR_OK, DR_EINVAL, DR_ESHAPE, DR_ENOMEM, DR_EDEVICE, DR_ECAPACITY = 0, -1, -2, -3, -4, -5
DR_RES_OK, DR_RES_INFEASIBLE, DR_RES_NONFINITE, DR_RES_MARGIN, DR_RES_BADSPLIT = 0, 1, 2, 4, 8
DR_PREC_F32, DR_PREC_F64 = 0, 1
DR_DTYPE_F32, DR_DTYPE_F64 = 0, 1
DR_INTER_CROWN_IBP, DR_INTER_IBP = 0, 1
DR_MARGIN_RIGOROUS, DR_MARGIN_OFF = 0, 1
DR_TILE_GLOBAL_WEIGHTS, DR_TILE_PAIRED_TILES, DR_TILE_NO_ITEM_CACHE = 1 << 16, 1 << 17, 1 << 18

EXPORTED = [
    "dr_create", "dr_bound_init", "dr_propagate_backward", "dr_concretize", "dr_optimize_duals",
    "dr_param_grad_workspace", "dr_param_grad", "dr_param_grad_static", "dr_set_weights",
    "dr_reach_dt", "dr_reach_dt_exo", "dr_reach_dt_joint", "dr_reach_grad_workspace", "dr_reach_dt_grad",
    "dr_flowpipe_ct", "dr_reach_ct",
    "dr_get_bounds", "dr_get_rows", "dr_get_margins", "dr_hidden_max", "dr_spec_rows",
    "dr_last_error", "dr_destroy",
]


class dr_network(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int),
        ("widths", ctypes.POINTER(ctypes.c_int)),
        ("wdtype", ctypes.c_int),
        ("W", ctypes.POINTER(ctypes.c_void_p)),
        ("b", ctypes.POINTER(ctypes.c_void_p)),
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("n_state", ctypes.c_int),
        ("spec", ctypes.c_void_p),
        ("n_spec", ctypes.c_int),
    ]


class dr_batch(ctypes.Structure):
    _fields_ = [
        ("n_sub", ctypes.c_int),
        ("net_id", ctypes.c_void_p),
        ("x_center", ctypes.c_void_p),
        ("x_radius", ctypes.c_void_p),
        ("split_ptr", ctypes.c_void_p),
        ("split_packed", ctypes.c_void_p),
    ]


class dr_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("intermediate", ctypes.c_int),
        ("max_sub", ctypes.c_int),
        ("max_splits", ctypes.c_int),
        ("tile_cfg", ctypes.c_int),
        ("margin_mode", ctypes.c_int),
        ("fuse_spec", ctypes.c_int),
    ]


class dr_ct_field(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("n_u", ctypes.c_int),
        ("a", ctypes.c_void_p),
        ("F", ctypes.c_void_p),
        ("G", ctypes.c_void_p),
        ("Q", ctypes.c_void_p),
    ]


class dr_ct_options(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("steps", ctypes.c_int),
        ("intervals", ctypes.c_int),
        ("tries", ctypes.c_int),
        ("rounds", ctypes.c_int),
        ("eps", ctypes.c_double),
    ]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load the built library (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is missing: build it with paper_2605_25346_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, F, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_void_p
    sig = {
        "dr_create": (I, [ctypes.POINTER(P), ctypes.POINTER(dr_network), I, ctypes.POINTER(dr_options), P]),
        "dr_bound_init": (I, [P, ctypes.POINTER(dr_batch), P, P]),
        "dr_propagate_backward": (I, [P, P, P, P, P, P]),
        "dr_concretize": (I, [P, P, P, P, P, P, P, P, P]),
        "dr_optimize_duals": (I, [P, I, F, I, P, P, P, P, P, P, P, P]),
        "dr_param_grad_workspace": (ctypes.c_size_t, [P, I]),
        "dr_set_weights": (I, [P, I, ctypes.POINTER(dr_network), P]),
        "dr_param_grad": (I, [P, P, P, I, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]),
        "dr_param_grad_static": (I, [P, P, P, I, P, P, P, P, P, P, P, P, P, P]),
        "dr_reach_dt": (I, [P, ctypes.POINTER(dr_batch), I, P, P, P]),
        "dr_reach_dt_exo": (I, [P, ctypes.POINTER(dr_batch), I, P, P, P, P]),
        "dr_reach_dt_joint": (I, [P, ctypes.POINTER(dr_batch), I, P, P, P, P, P]),
        "dr_reach_grad_workspace": (ctypes.c_size_t, [P, I, I]),
        "dr_reach_dt_grad": (I, [P, ctypes.POINTER(dr_batch), I, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]),
        "dr_flowpipe_ct": (I, [ctypes.POINTER(dr_ct_field), ctypes.POINTER(dr_ct_options), I, P, P, P, P, P, P]),
        "dr_reach_ct": (I, [P, ctypes.POINTER(dr_ct_field), ctypes.POINTER(dr_ct_options), ctypes.POINTER(dr_batch),
                            P, P, P, P]),
        "dr_get_bounds": (I, [P, P, P, P]),
        "dr_get_rows": (I, [P, P, P]),
        "dr_get_margins": (I, [P, P, P]),
        "dr_hidden_max": (I, [P]),
        "dr_spec_rows": (I, [P]),
        "dr_last_error": (ctypes.c_char_p, [P]),
        "dr_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status, ctx=None):
    if status != DR_OK:
        lib = load()
        msg = lib.dr_last_error(ctx).decode() if ctx is not None else lib.dr_last_error(None).decode()
        raise DrError(status, msg)
