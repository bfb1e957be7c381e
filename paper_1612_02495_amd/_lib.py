"""ctypes loader for libswept.so (the C ABI declared in include/swept.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If the library is missing it is built once (hipcc, gfx950); if it
cannot be loaded the import fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswept.so")

SWEPT_OK = 0
SWEPT_EINVAL = -1
SWEPT_EUNSUPPORTED = -2
SWEPT_ENOMEM = -3
SWEPT_EDEVICE = -4
SWEPT_ENONFINITE = -5
SWEPT_CHECK_NONFINITE = 1

SWEPT_HEAT_FTCS = 0
SWEPT_HEAT_INSULATED = 2
SWEPT_KS_RK2 = 1
SWEPT_F32 = 0
SWEPT_F64 = 1
SWEPT_ENGINE_AUTO = 0
SWEPT_ENGINE_LDS = 1
SWEPT_ENGINE_WAVE = 2
SWEPT_ENGINE_COMPACT = 3
SWEPT_ENGINE_RESIDENT = 4

_lock = threading.Lock()
_lib = None


class TuneResult(ctypes.Structure):
    """swept_tune_result of include/swept.h."""
    _fields_ = [("tile_width", ctypes.c_int32), ("steps_per_cycle", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ns_per_cell_update", ctypes.c_double)]


class SweptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swept error {code}: {msg}")
        self.code = code


def _declare(lib):
    i32, i64, dbl, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sz = ctypes.c_size_t
    lib.swept_plan_create.argtypes = [ctypes.POINTER(vp), i64, i32, i32, dbl, dbl, dbl, i32, i32]
    lib.swept_run.argtypes = [vp, vp, i64, vp]
    lib.naive_run.argtypes = [vp, vp, i64, vp]
    lib.swept_run_noalloc.argtypes = [i64, i32, i32, dbl, dbl, dbl, i32, i32, vp, i64, vp]
    lib.swept_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz)]
    lib.swept_plan_set_engine.argtypes = [vp, i32]
    lib.swept_plan_set_checks.argtypes = [vp, i32]
    lib.swept_plan_destroy.argtypes = [vp]
    lib.swept_plan_destroy.restype = None
    lib.swept_last_error.argtypes = []
    lib.swept_last_error.restype = ctypes.c_char_p
    lib.swept_schedule.argtypes = [i32, i32, i32, i64, ctypes.POINTER(ctypes.c_int32), i64,
                                   ctypes.POINTER(i64)]
    pi = ctypes.POINTER(i32)
    pd = ctypes.POINTER(dbl)
    lib.swept_tile_geometry.argtypes = [i32, i32, pi, pi, pi]
    lib.swept_autotune.argtypes = [i64, i32, i32, dbl, dbl, dbl, i64, ctypes.POINTER(TuneResult), i32, pi,
                                   pi, pi, pi]
    lib.swept_autotune_lookup.argtypes = [i64, i32, i32, pi, pi, pi, pd]
    lib.swept_autotune_forget.argtypes = []
    lib.swept_autotune_forget.restype = None
    pl = ctypes.POINTER(i64)
    lib.swept_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, pl, i32, i32, pd, pd, pd, i64]
    lib.swept_batch_run.argtypes = [vp, vp, i32, vp]
    lib.swept_batch_set_engine.argtypes = [vp, i32]
    lib.swept_batch_set_checks.argtypes = [vp, i32]
    lib.swept_batch_info.argtypes = [vp, pl, pl, ctypes.POINTER(sz), pi]
    lib.swept_batch_destroy.argtypes = [vp]
    lib.swept_batch_destroy.restype = None
    lib.swept_adjoint_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64, i32, dbl, dbl, i64]
    lib.swept_adjoint_create_segmented.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64, i32, dbl, dbl, i64, i32]
    lib.swept_forward_ckpt.argtypes = [vp, vp, vp, vp, vp]
    lib.swept_adjoint_run.argtypes = [vp, vp, vp, vp, vp]
    lib.swept_adjoint_info.argtypes = [vp, ctypes.POINTER(sz), pi, pi, pl]
    lib.swept_adjoint_destroy.argtypes = [vp]
    lib.swept_adjoint_destroy.restype = None
    lib.swept_ks_adjoint_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64, i32, dbl, dbl, i64]
    lib.swept_ks_forward_ckpt.argtypes = [vp, vp, vp, vp]
    lib.swept_ks_adjoint_run.argtypes = [vp, vp, vp, vp]
    lib.swept_ks_adjoint_info.argtypes = [vp, ctypes.POINTER(sz), pi, pi, pl]
    lib.swept_ks_adjoint_destroy.argtypes = [vp]
    lib.swept_ks_adjoint_destroy.restype = None
    for name in ("swept_ks_adjoint_create", "swept_ks_forward_ckpt", "swept_ks_adjoint_run",
                 "swept_ks_adjoint_info", "swept_adjoint_create", "swept_adjoint_create_segmented", "swept_forward_ckpt", "swept_adjoint_run", "swept_adjoint_info",
                 "swept_batch_create", "swept_batch_run", "swept_batch_set_engine", "swept_batch_info", "swept_autotune", "swept_autotune_lookup", "swept_tile_geometry", "swept_plan_create", "swept_run", "swept_run_noalloc", "naive_run", "swept_plan_info",
                 "swept_plan_set_engine", "swept_schedule", "swept_plan_set_checks", "swept_batch_set_checks"):
        getattr(lib, name).restype = i32
    return lib


def lib():
    """Load (building first if absent) and return the ctypes handle."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    from . import build as _build
                    _build.build()
                _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def last_error() -> str:
    return lib().swept_last_error().decode(errors="replace")


def check(rc: int) -> None:
    if rc != SWEPT_OK:
        raise SweptError(rc, last_error())
