"""ctypes declarations of liblbmax.so (include/lbmax.h).

Argument marshalling only.  Loading fails loudly if the library has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmax.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE, LB_ENONFINITE = 0, -1, -2, -3, -4, -5
LB_F64, LB_F32, LB_F32_P64 = 0, 1, 2
LB_CHECK_FINITE, LB_CHECK_MACH = 1, 2
LB_WARN_MACH = 1
STATUS_NAMES = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EDEVICE",
                -4: "LB_ESTATE", -5: "LB_ENONFINITE"}


class ChannelDesc(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
        ("tau_lb", ctypes.c_double),
        ("g_inf", ctypes.c_double), ("tau_m", ctypes.c_double), ("gamma_c", ctypes.c_double),
        ("n_hist", ctypes.c_int32),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("u0", ctypes.POINTER(ctypes.c_double)),
        ("hist_blocks", ctypes.c_int32), ("hist_block_len", ctypes.c_int32),
        ("finger", ctypes.c_int32), ("paper_coupling", ctypes.c_int32),
        ("law", ctypes.c_int32),
    ]


# Channel.law names -> lb_channel_desc.law
LAWS = {"nlm": 0, "strain_damping": 1, "instantaneous": 2}


class LBError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_D = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/lbmax.h
SIGNATURES = {
    "lb_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ChannelDesc), ctypes.c_int32, ctypes.c_int]),
    "lb_init": (ctypes.c_int, [ctypes.POINTER(ChannelDesc), ctypes.c_int32, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]),
    "lb_set_force": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
    "lb_step": (ctypes.c_int, [_H, ctypes.c_int64]),
    "lb_time": (ctypes.c_int64, [_H]),
    "lb_set_checks": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_warnings": (ctypes.c_int32, [_H]),
    "lb_fields": (ctypes.c_int, [_H, ctypes.c_int32, _D, _D, _D]),
    "lb_stress": (ctypes.c_int, [_H, ctypes.c_int32, _D, _D]),
    "lb_grad": (ctypes.c_int, [_H, ctypes.c_int32, _D]),
    "lb_state_bytes": (ctypes.c_size_t, [_H]),
    "lb_save_state": (ctypes.c_int, [_H, ctypes.c_void_p]),
    "lb_load_state": (ctypes.c_int, [_H, ctypes.c_void_p]),
    "lb_max_chunks": (ctypes.c_int32, [_H, ctypes.c_int32]),
    "lb_set_tiling": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lb_get_tiling": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "lb_set_graph": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_set_block": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_get_block": (ctypes.c_int32, [_H]),
    "lb_set_fused": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_get_fused": (ctypes.c_int32, [_H]),
    "lb_set_adjoint_block": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_get_adjoint_block": (ctypes.c_int32, [_H]),
    "lb_set_persistent": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_profile": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_kernel_time": (ctypes.c_int, [_H, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lb_set_params": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]),
    "lb_adjoint_workspace_bytes": (ctypes.c_size_t, [_H, ctypes.c_int32]),
    "lb_adjoint_begin": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32]),
    "lb_adjoint_begin_noalloc": (ctypes.c_int, [_H, ctypes.c_int32]),
    "lb_adjoint_segment": (ctypes.c_int, [_H, ctypes.c_void_p, _D, ctypes.c_int32]),
    "lb_adjoint_end": (ctypes.c_int, [_H, _D]),
    "lb_destroy": (ctypes.c_int, [_H]),
    "lb_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1504_06123_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().lb_last_error().decode()


def check(status: int, where: str):
    if status != LB_OK:
        raise LBError(status, where, last_error())
