"""ctypes declarations of libdedisp.so (the C-ABI of include/dedisp.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdedisp.so")

i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
vp, cp, sz = ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t
P_i32 = ctypes.POINTER(i32)

OK, E_INVALID, E_SHAPE, E_DTYPE, E_ALIGN, E_NOMEM, E_HIP, E_UNTUNED, E_WORKSPACE = range(9)
F32, U8, I32 = 0, 1, 2

# name -> (restype, argtypes)
SIGNATURES = {
    "dedisp_plan_create": (i32, [ctypes.POINTER(vp), i32, vp, f64, i32, vp]),
    "dedisp_compute_delays": (i32, [i32, vp, f64, i32, vp, vp, P_i32]),
    "dedisp_plan_destroy": (i32, [vp]),
    "dedisp_plan_info": (i32, [vp, P_i32, P_i32, P_i32]),
    "dedisp_plan_delays": (i32, [vp, vp]),
    "dedisp_plan_prepare": (i32, [vp, i32, i32]),
    "dedisp_execute": (i32, [vp, i32, i32, vp, i32, i64, vp, vp, i32, i64, vp]),
    "dedisp_adjoint": (i32, [vp, i32, i32, i32, vp, i64, vp, vp, i64, vp, i64, vp, vp, sz, vp]),
    "dedisp_adjoint_workspace_bytes": (sz, [vp, i32, i32]),
    "dedisp_adjoint_noalloc": (i32, [vp, i32, i32, i32, vp, i64, vp, vp, i64, vp, i64, vp, vp]),
    "dedisp_adjoint_noalloc_bytes": (sz, [vp, i32, i32]),
    "dedisp_batch_create": (i32, [ctypes.POINTER(vp), i32, vp, vp, vp, i32, vp, vp, vp, vp, i32, cp]),
    "dedisp_batch_cache_hit": (i32, [vp]),
    "dedisp_execute_batched": (i32, [vp, vp]),
    "dedisp_execute_per_beam": (i32, [vp, vp]),
    "dedisp_batch_set_variant": (i32, [vp, i32]),
    "dedisp_batch_variant": (i32, [vp]),
    "dedisp_batch_queues": (i32, [vp]),
    "dedisp_batch_set_queues": (i32, [vp, i32]),
    "dedisp_batch_destroy": (i32, [vp]),
    "dedisp_autotune": (i32, [vp, i32, i32, i32, cp]),
    "dedisp_autotune_times": (i32, [vp, i32, vp, i32]),
    "dedisp_autotune_adjoint": (i32, [vp, i32, i32, vp, i32]),
    "dedisp_variant_count": (i32, [i32]),
    "dedisp_variant_name": (cp, [i32, i32]),
    "dedisp_plan_set_variant": (i32, [vp, i32, i32]),
    "dedisp_plan_variant": (i32, [vp, i32]),
    "dedisp_plan_set_adjoint_variant": (i32, [vp, i32]),
    "dedisp_plan_adjoint_variant": (i32, [vp]),
    "dedisp_detect": (i32, [vp, i32, i32, vp, i32, i64, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
    "dedisp_detect_workspace_bytes": (sz, [vp, i32, i32, i32]),
    "dedisp_detect_variant": (i32, [vp, i32]),
    "dedisp_plan_set_detect_variant": (i32, [vp, i32, i32]),
    "dedisp_detect_autotune": (i32, [vp, i32, i32, i32, i32, vp, i32]),
    "dedisp_detect_rows": (i32, [i32, i32, vp, i32, i64, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
    "dedisp_detect_rows_workspace_bytes": (sz, [i32, i32]),
    "dedisp_status_string": (cp, [i32]),
    "dedisp_last_error": (cp, []),
}

_lib = None


class DedispError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.dedisp_status_string(status).decode()
        detail = lib.dedisp_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def load():
    """Load libdedisp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1601_01165_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != OK:
        raise DedispError(status, where)
