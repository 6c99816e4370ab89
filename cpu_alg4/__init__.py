"""The paper's Algorithm 4 on the host CPU (AVX2, 32 starts per vector): a CPU baseline.

``bench.py`` times it beside the oracle: it is the method itself (Sections
2.1-2.3: frequency-ordered compares, the first r peeled, a zero test after each
later compare), as the paper ran it, on the GPU machine's host cores.  The C code in
``alg4.c`` is separate from both the oracle (which stays the plain definition)
and the GPU path; ``tests/test_cpu_alg4.py`` checks its counts against the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libalg4.so")
_lib = None


def build() -> None:
    """Compile alg4.c (gcc, AVX2, OpenMP)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O3", "-mavx2", "-mpopcnt", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                    os.path.join(_HERE, "alg4.c")], check=True)
    os.replace(tmp, _LIB_PATH)


def available() -> bool:
    """Whether this host has AVX2."""
    try:
        return any(line.startswith("flags") and " avx2" in line for line in open("/proc/cpuinfo"))
    except OSError:
        return False


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.alg4_avx2_count.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint64, vp, ctypes.c_uint32, ctypes.c_int]
        lib.alg4_avx2_count.restype = ctypes.c_int64
        _lib = lib
    return _lib


def freq_order(p, hist) -> np.ndarray:
    """Positions of p by increasing frequency of their symbol, ties by position (Section 2.2)."""
    a = np.frombuffer(bytes(p), dtype=np.uint8)
    return np.argsort(np.asarray(hist, dtype=np.uint64)[a], kind="stable").astype(np.int32)


def count(p, t, order=None, r: int = 2, nthreads: int = 1) -> int:
    """Overlapping occurrences of p in t; order = compare order (default left to right)."""
    pb = bytes(p)
    ta = np.ascontiguousarray(t, dtype=np.uint8)
    m = len(pb)
    o = np.arange(m, dtype=np.int32) if order is None else np.ascontiguousarray(order, dtype=np.int32)
    pa = np.frombuffer(pb, dtype=np.uint8) if m else np.zeros(1, dtype=np.uint8)
    res = _load().alg4_avx2_count(pa.ctypes.data, m, ta.ctypes.data if ta.size else None, ta.size,
                                  o.ctypes.data, min(max(int(r), 1), max(m, 1)), int(nthreads))
    if res < 0:
        raise ValueError("bad arguments (m == 0 or order) or out of memory")
    return int(res)
