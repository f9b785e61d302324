"""ctypes declarations of libhullprep.so (C ABI in include/hullprep.h).

Argument marshalling only: every step of the path runs in the HIP library.
Importing this module raises if the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhullprep.so")

HP_OK, HP_EINVAL, HP_ERANGE, HP_ECAPACITY, HP_EDEVICE, HP_ENOMEM, HP_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
HP_P_MAX = (1 << 30) - 64
HP_INFO_STATUS, HP_INFO_K, HP_INFO_S, HP_INFO_H, HP_INFO_WORDS = 0, 1, 2, 3, 4
HP_STRATEGY_AUTO, HP_STRATEGY_LDS, HP_STRATEGY_GLOBAL, HP_STRATEGY_LDS_PARTIAL, HP_STRATEGY_WINDOW = 0, 1, 2, 3, 4
HP_STRATEGY_SAMPLED = 5
HP_STRATEGY_BINNED = 6
HP_STRATEGY_SPARSE = 7
HP_NOALLOC_SCRATCH_BYTES = 128 << 20

# every entry point the header declares, with (restype, argtypes)
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_szp = ctypes.POINTER(ctypes.c_size_t)

SIGNATURES = {
    "hp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hp_last_error": (ctypes.c_char_p, []),
    "hp_abi_version": (ctypes.c_int, []),
    "hp_lds_max_p": (_i32, []),
    "hp_set_strategy": (ctypes.c_int, [ctypes.c_int]),
    "hp_reduce_strategy": (ctypes.c_int, [_i64, _i32, _i32p]),
    "hp_tune_set": (ctypes.c_int, [_i32, _i32, _i32, _i32]),
    "hp_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "hp_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "hp_timing_read": (ctypes.c_int, [_i32p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
    "hp_workspace_bytes": (ctypes.c_int, [_i64, _i32, _szp]),
    "hp_precondition": (ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32,
                                       _vp, _vp, _sz, _vp]),
    "hp_hull_workspace_bytes": (ctypes.c_int, [_i32, _szp]),
    "hp_rescan_y_workspace_bytes": (ctypes.c_int, [_i32, _i32, _szp]),
    "hp_rescan_y": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _sz,
                                   _vp]),
    "hp_hull_melkman_workspace_bytes": (ctypes.c_int, [_i32, _szp]),
    "hp_hull_melkman": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "hp_bitset_words": (ctypes.c_int, [_i32, _i32, _i64p]),
    "hp_bitset_clear": (ctypes.c_int, [_vp, _i64, _vp]),
    "hp_bitset_insert": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "hp_bitset_extract_workspace_bytes": (ctypes.c_int, [_i32, _szp]),
    "hp_bitset_build_workspace_bytes": (ctypes.c_int, [_i64, _i32, _szp]),
    "hp_bitset_build": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "hp_bitset_extract": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i32, _vp, _vp, _sz, _vp]),
    "hp_bbox_workspace_bytes": (ctypes.c_int, [_szp]),
    "hp_transpose_points": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "hp_bbox_f32": (ctypes.c_int, [_vp, _i64, _vp, _vp, _sz, _vp]),
    "hp_quantize_f32": (ctypes.c_int, [_vp, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                       _vp]),
    "hp_bbox": (ctypes.c_int, [_vp, _i64, _vp, _vp, _sz, _vp]),
    "hp_run_origin": (ctypes.c_int, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                     _i32, _vp, _vp, _sz, _vp]),
    "hp_workspace_bytes_rect": (ctypes.c_int, [_i64, _i32, _i32, _szp]),
    "hp_run_rect": (ctypes.c_int, [_vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                   _i32, _vp, _vp, _sz, _vp]),
    "hp_run_auto_workspace_bytes": (ctypes.c_int, [_i64, _i32, _i32, _szp]),
    "hp_run_auto": (ctypes.c_int, [_vp, _i64, _i32, _i32, _i64p, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                   _i32, _vp, _vp, _sz, _vp]),
    "hp_run_auto_f32_workspace_bytes": (ctypes.c_int, [_i64, _i32, _szp]),
    "hp_run_auto_f32": (ctypes.c_int, [_vp, _i64, _i32, ctypes.POINTER(ctypes.c_double), _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "hp_hull": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "hp_run": (ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                              _i32, _vp, _vp, _sz, _vp]),
    "hp_run_noalloc": (ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                      _i32, _vp, _vp]),
    "hp_plan_create": (ctypes.c_int, [_i64p, _i32p, _i32, ctypes.POINTER(_vp)]),
    "hp_plan_query": (ctypes.c_int, [_vp, _i64p, _i64p, _szp, _i64p, _i64p]),
    "hp_batched_run": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "hp_batched_run_percloud": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                               _vp]),
    "hp_plan_destroy": (None, [_vp]),
    "hp_server_create": (ctypes.c_int, [_sz, _i32, ctypes.POINTER(_vp)]),
    "hp_server_request_bytes": (ctypes.c_int, [_i64, _i32, _i32, _szp]),
    "hp_server_submit": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp,
                                        _i64p]),
    "hp_server_wait": (ctypes.c_int, [_vp, _i64, _i64, _i64p]),
    "hp_server_stats": (ctypes.c_int, [_vp, _i64p]),
    "hp_server_destroy": (ctypes.c_int, [_vp]),
    "hp_clock_ns": (_i64, []),
}


class HullprepError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({detail})" if detail else
                         f"{where}: {status_string(code)}")


_lib: ctypes.CDLL | None = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the HIP library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -m paper_1505_00914_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load().hp_status_string(code).decode()
    except ImportError:
        return f"status {code}"


def check(code: int, where: str) -> int:
    if code < 0:
        detail = load().hp_last_error().decode()
        raise HullprepError(code, where, detail)
    return code


def call(name: str, *args) -> int:
    fn = getattr(load(), name)
    return check(fn(*args), name)
