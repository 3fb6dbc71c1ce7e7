"""ctypes loader for libfitnll.so and the C prototypes of include/fitnll.h.

Loading fails loudly when the library has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfitnll.so")

FN_OK = 0
FN_E_INVALID = -1
FN_E_DOMAIN = -2
FN_E_NONFINITE = -3
FN_E_NOMEM = -4
FN_E_HIP = -5
FN_E_BUDGET = -6
FN_E_CANCELLED = -7

FN_FIT_IDLE, FN_FIT_RUNNING, FN_FIT_CONVERGED, FN_FIT_FAILED = 0, 1, 2, 3

STATUS_NAMES = {
    FN_E_INVALID: "FN_E_INVALID", FN_E_DOMAIN: "FN_E_DOMAIN", FN_E_NONFINITE: "FN_E_NONFINITE",
    FN_E_NOMEM: "FN_E_NOMEM", FN_E_HIP: "FN_E_HIP", FN_E_BUDGET: "FN_E_BUDGET",
    FN_E_CANCELLED: "FN_E_CANCELLED",
}

vp = C.c_void_p
dp = C.POINTER(C.c_double)
i32 = C.c_int32
i64 = C.c_int64

# name -> (restype, argtypes); mirrors include/fitnll.h
PROTOTYPES = {
    "fn_last_error": (C.c_char_p, []),
    "fn_version": (i32, []),
    "fn_ctx_create": (i32, [i32, C.POINTER(vp)]),
    "fn_ctx_destroy": (i32, [vp]),
    "fn_model_create": (i32, [vp, C.c_char_p, C.POINTER(vp)]),
    "fn_model_check_compile": (i32, [C.c_char_p, C.c_char_p]),
    "fn_model_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
    "fn_model_destroy": (i32, [vp]),
    "fn_events_check": (i32, [vp, vp, i64, i64, C.POINTER(i64), vp]),
    "fn_nll": (i32, [vp, dp, vp, i64, i64, dp, dp, vp]),
    "fn_nll_async": (i32, [vp, vp, vp, i64, i64, vp, i32, vp]),
    "fn_nll_async_noalloc": (i32, [vp, vp, vp, i64, i64, vp, i32, vp]),
    "fn_norm": (i32, [vp, dp, dp, dp, vp]),
    "fn_eval": (i32, [vp, dp, vp, i64, i64, vp, vp]),
    "fn_model_set_norm_sample": (i32, [vp, vp, i64, i64, vp]),
    "fn_model_fixed": (i32, [vp, C.POINTER(i32), dp]),
    "fn_model_timing": (i32, [vp, i32]),
    "fn_model_kernel_time": (i32, [vp, dp, C.POINTER(i64)]),
    "fn_fit": (i32, [vp, dp, C.POINTER(i32), vp, i64, i64, i32, C.c_double, i32, dp, dp, dp,
                     C.POINTER(i32), C.POINTER(i32), vp]),
    "fn_vbatch_create": (i32, [vp, i32, C.POINTER(vp)]),
    "fn_vbatch_destroy": (i32, [vp]),
    "fn_vbatch_set_fixed": (i32, [vp, i32, dp]),
    "fn_vbatch_nll": (i32, [vp, dp, vp, i64, i64, dp, dp, vp]),
    "fn_vbatch_fit": (i32, [vp, dp, C.POINTER(i32), vp, i64, i64, C.c_double, i32, i32, C.POINTER(i32), dp, dp,
                            dp, C.POINTER(i32), C.POINTER(i32), vp]),
    "fn_vbatch_serve": (i32, [vp, vp, i32, C.POINTER(i32), vp, i64, i64, C.c_double, i32, i32, C.POINTER(i32),
                              dp, dp, dp, C.POINTER(i32), C.POINTER(i32), dp, dp, vp]),
    "fn_batch_create": (i32, [vp, i32, i64, C.POINTER(vp)]),
    "fn_batch_destroy": (i32, [vp]),
    "fn_batch_set_slot": (i32, [vp, i32, vp, i64, dp, C.POINTER(i32)]),
    "fn_batch_clear_slot": (i32, [vp, i32]),
    "fn_batch_config": (i32, [vp, C.c_double, i32, i32]),
    "fn_batch_run": (i32, [vp, i32, i32, C.POINTER(i32), C.POINTER(i32)]),
    "fn_batch_results": (i32, [vp, C.POINTER(i32), dp, dp, dp, C.POINTER(i32), C.POINTER(i32)]),
    "fn_batch_set": (i32, [vp, i32, C.POINTER(vp), C.POINTER(i64), C.POINTER(i64), vp]),
    "fn_batch_step": (i32, [vp, vp]),
    "fn_batch_status": (i32, [vp, C.POINTER(i32), dp, dp, dp]),
    "fn_generate_mix1d": (i32, [C.c_uint32, C.c_uint32, i64, dp, C.c_double, C.c_double, vp, vp]),
    "fn_generate": (i32, [vp, dp, C.c_uint32, C.c_uint32, i64, C.c_double, vp, i64, dp, vp]),
    "fn_model_autotune": (i32, [vp, dp, vp, i64, i64, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), dp,
                                vp]),
    "fn_model_generate_norm_sample": (i32, [vp, C.c_uint32, C.c_uint32, i64, vp]),
    "fn_nll_binned": (i32, [vp, dp, vp, i64, i32, dp, dp, vp]),
    "fn_fit_binned": (i32, [vp, dp, C.POINTER(i32), vp, i64, i32, i32, C.c_double, i32, dp, dp, dp,
                            C.POINTER(i32), C.POINTER(i32), vp]),
    "fn_server_create": (i32, [vp, i32, i64, i64, C.POINTER(vp)]),
    "fn_server_destroy": (i32, [vp]),
    "fn_server_submit": (i32, [vp, vp, i32]),
    "fn_server_run": (i32, [vp, i32, C.c_double, C.POINTER(i32)]),
    "fn_server_results": (i32, [vp, vp, i32, C.POINTER(i32)]),
}

_lib = None


class FitNLLError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libfitnll.so once and attach prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1710_08826_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != FN_OK:
        msg = load().fn_last_error().decode("utf-8", "replace")
        raise FitNLLError(status, msg)
