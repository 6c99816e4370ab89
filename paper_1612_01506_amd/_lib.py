"""ctypes loader for libsm.so (argument marshalling only; all work runs in the HIP library).

There is no fallback: if the library is missing this module raises, so a user
or test can never silently run anything but the HIP path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsm.so")

SM_OK, SM_EINVAL, SM_ENOMEM, SM_EDEVICE = 0, -1, -2, -3
SM_ORDER_LTR, SM_ORDER_FREQ, SM_ORDER_H, SM_ORDER_HS = 0, 1, 2, 3
SM_NONOVERLAP = 1
SM_BITMAP = 2

# Every symbol declared in include/sm.h.
EXPORTS = (
    "sm_version", "sm_last_error", "sm_device_cus", "sm_shutdown", "sm_histogram", "sm_order",
    "sm_count", "sm_count_ex", "sm_count_async", "sm_report", "sm_report_ex", "sm_count_batch",
    "sm_patterns_create", "sm_patterns_destroy", "sm_patterns_count", "sm_patterns_report",
    "sm_report_async", "sm_patterns_report_async", "sm_patterns_create_ordered",
    "sm_batch_create", "sm_batch_run", "sm_batch_destroy", "sm_bigram", "sm_order_bigram",
    "sm_report_batch", "sm_patterns_report_noalloc",
)


class SmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsm error {code}: {msg}")
        self.code = code


class sm_batch_tune(ctypes.Structure):
    _fields_ = [("bm_min", ctypes.c_int32 * 4), ("bm_chunk", ctypes.c_int32 * 4), ("peel", ctypes.c_int32 * 4),
                ("tile_kib", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("deal_wgs_per_cu", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class sm_params(ctypes.Structure):
    _fields_ = [("peel", ctypes.c_int32), ("tile_kib", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("batch", ctypes.POINTER(sm_batch_tune))]


class sm_text(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("n", ctypes.c_uint64), ("hist", ctypes.c_void_p)]


class sm_query(ctypes.Structure):
    _fields_ = [("text_id", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("p", ctypes.c_void_p),
                ("m", ctypes.c_uint64), ("order", ctypes.c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1612_01506_amd.build` "
                          "(the HIP library is required, there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, i64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "sm_version": ([], i32),
        "sm_last_error": ([], ctypes.c_char_p),
        "sm_device_cus": ([], i32),
        "sm_shutdown": ([], i32),
        "sm_histogram": ([vp, u64, vp, vp], i32),
        "sm_order": ([i32, vp, u64, vp, vp], i32),
        "sm_count": ([vp, u64, vp, u64, vp], i64),
        "sm_count_ex": ([vp, u64, vp, u64, vp, P(sm_params), vp], i64),
        "sm_count_async": ([vp, u64, vp, u64, vp, P(sm_params), vp, vp], i32),
        "sm_report": ([vp, u64, vp, u64, vp, vp, u64], i64),
        "sm_report_ex": ([vp, u64, vp, u64, vp, P(sm_params), vp, u64, vp], i64),
        "sm_count_batch": ([P(sm_query), u64, P(sm_text), u64, vp, P(sm_params), vp], i32),
        "sm_patterns_create": ([u64, P(vp), P(u64), P(vp), P(vp)], i32),
        "sm_batch_create": ([P(sm_query), u64, P(sm_text), u64, P(sm_params), P(vp)], i32),
        "sm_batch_run": ([vp, vp, vp], i32),
        "sm_batch_destroy": ([vp], i32),
        "sm_bigram": ([vp, u64, vp, vp, vp], i32),
        "sm_report_batch": ([P(sm_query), u64, P(sm_text), u64, vp, vp, vp, P(sm_params), vp], i32),
        "sm_order_bigram": ([vp, u64, vp, vp, vp], i32),
        "sm_patterns_destroy": ([vp], i32),
        "sm_patterns_create_ordered": ([u64, P(vp), P(u64), i32, vp, P(vp)], i32),
        "sm_patterns_count": ([vp, u64, vp, u64, P(sm_params), vp, vp], i32),
        "sm_patterns_report": ([vp, u64, vp, u64, P(sm_params), vp, u64, vp], i64),
        "sm_report_async": ([vp, u64, vp, u64, vp, P(sm_params), vp, u64, vp, vp], i32),
        "sm_patterns_report_async": ([vp, u64, vp, u64, P(sm_params), vp, u64, vp, vp], i32),
        "sm_patterns_report_noalloc": ([vp, u64, vp, u64, P(sm_params), vp, u64, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(rc: int) -> int:
    if rc < 0:
        raise SmError(rc, load().sm_last_error().decode(errors="replace"))
    return rc
