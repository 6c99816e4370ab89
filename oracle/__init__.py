"""CPU oracle for exact string matching (arXiv 1612.01506) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The product path (``paper_1612_01506_amd``) never
imports, links or runs it, and it shares no code with that path.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module only
marshals arguments.  Functions and the passages they follow:

* ``count``      -- Algorithm 1 (Section 2.1): starts s in [0, n-m] with t[s:s+m] == p.
* ``report``     -- the reporting version of Algorithm 1 (Section 2.1).
* ``count_nonoverlap`` / ``report_nonoverlap`` -- disjoint occurrences by greedy leftmost selection
  (not defined in the paper; the reading taken for the optional non-overlapping mode).
* ``hist``       -- symbol frequencies (Section 2.2).
* ``order_freq`` -- compare order by increasing symbol frequency (Section 2.2), ties by position.
* ``order_h`` / ``order_hs`` -- the fixed orders pi_h and pi_hs (Section 2.4).
* ``bigram`` / ``order_bigram`` -- adjacent-pair frequencies and the bigram-aware order (the
  conditional-probability strategy Section 2.2 discusses, restricted to adjacent pairs).
* ``alg4_count`` -- Algorithm 4 (Section 2.3) emulated with a 64-bit found word.

Every function is pinned by ``tests/test_oracle.py`` against brute force, the
worked example of Figure 1, closed forms and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# Test hook: tests/test_oracle_mutants.py points this at deliberately broken builds
# of oracle.c to show that the pins catch each planted mistake.
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")
_lib = None


def build() -> None:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                    os.path.join(_HERE, "oracle.c")], check=True)
    os.replace(tmp, _LIB_PATH)


def _load():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB_PATH
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        u8p, u64, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64
        lib.oracle_count.argtypes = [u8p, u64, u8p, u64, ctypes.c_int]
        lib.oracle_count.restype = i64
        lib.oracle_report.argtypes = [u8p, u64, u8p, u64, u8p, u64]
        lib.oracle_report.restype = i64
        lib.oracle_hist.argtypes = [u8p, u64, u8p]
        lib.oracle_hist.restype = None
        lib.oracle_order_freq.argtypes = [u8p, u64, u8p, u8p]
        lib.oracle_order_freq.restype = ctypes.c_int
        lib.oracle_order_h.argtypes = [u64, u8p]
        lib.oracle_order_h.restype = ctypes.c_int
        lib.oracle_order_hs.argtypes = [u8p, u64, u8p]
        lib.oracle_order_hs.restype = ctypes.c_int
        lib.oracle_report_nonoverlap.argtypes = [u8p, u64, u8p, u64, u8p, u64]
        lib.oracle_report_nonoverlap.restype = i64
        lib.oracle_bigram.argtypes = [u8p, u64, u8p]
        lib.oracle_bigram.restype = None
        lib.oracle_order_bigram.argtypes = [u8p, u64, u8p, u8p, u8p]
        lib.oracle_order_bigram.restype = ctypes.c_int
        lib.oracle_alg4_count.argtypes = [u8p, u64, u8p, u64, u8p, u64]
        lib.oracle_alg4_count.restype = i64
        _lib = lib
    return _lib


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    a = np.ascontiguousarray(x, dtype=np.uint8)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def count(p, t, nthreads: int | None = None) -> int:
    p, t = _u8(p), _u8(t)
    r = _load().oracle_count(_ptr(p), p.size, _ptr(t), t.size, nthreads or default_threads())
    if r < 0:
        raise ValueError("pattern length must be >= 1")
    return int(r)


def report(p, t, cap: int | None = None) -> np.ndarray:
    """Ascending 0-based start positions (all of them when cap is None)."""
    p, t = _u8(p), _u8(t)
    lib = _load()
    if cap is None:
        cap = count(p, t)
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    r = lib.oracle_report(_ptr(p), p.size, _ptr(t), t.size, out.ctypes.data, cap)
    if r < 0:
        raise ValueError("pattern length must be >= 1")
    return out[:min(r, cap)]


def report_full(p, t, cap: int) -> tuple[int, np.ndarray]:
    p, t = _u8(p), _u8(t)
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    r = _load().oracle_report(_ptr(p), p.size, _ptr(t), t.size, out.ctypes.data, cap)
    if r < 0:
        raise ValueError("pattern length must be >= 1")
    return int(r), out[:min(r, cap)]


def report_nonoverlap_full(p, t, cap: int) -> tuple[int, np.ndarray]:
    """(count of disjoint occurrences taken greedily from the left, first min(count, cap) of their starts)."""
    p, t = _u8(p), _u8(t)
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    r = _load().oracle_report_nonoverlap(_ptr(p), p.size, _ptr(t), t.size, out.ctypes.data, cap)
    if r < 0:
        raise ValueError("pattern length must be >= 1")
    return int(r), out[:min(r, cap)]


def count_nonoverlap(p, t) -> int:
    return report_nonoverlap_full(p, t, 0)[0]


def report_nonoverlap(p, t, cap: int | None = None) -> np.ndarray:
    if cap is None:
        cap = count_nonoverlap(p, t)
    return report_nonoverlap_full(p, t, cap)[1]


def hist(t) -> np.ndarray:
    t = _u8(t)
    h = np.zeros(256, dtype=np.uint64)
    _load().oracle_hist(_ptr(t), t.size, h.ctypes.data)
    return h


def order_freq(p, h) -> np.ndarray:
    p = _u8(p)
    h = np.ascontiguousarray(h, dtype=np.uint64)
    out = np.zeros(max(p.size, 1), dtype=np.int32)
    if _load().oracle_order_freq(_ptr(p), p.size, h.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("bad pattern length")
    return out[:p.size]


def order_h(m: int) -> np.ndarray:
    out = np.zeros(max(m, 1), dtype=np.int32)
    if _load().oracle_order_h(m, out.ctypes.data) != 0:
        raise ValueError("bad pattern length")
    return out[:m]


def order_hs(p) -> np.ndarray:
    p = _u8(p)
    out = np.zeros(max(p.size, 1), dtype=np.int32)
    if _load().oracle_order_hs(_ptr(p), p.size, out.ctypes.data) != 0:
        raise ValueError("bad pattern length")
    return out[:p.size]


def bigram(t) -> np.ndarray:
    """(256, 256) uint64: [a, b] = number of s with t[s] == a and t[s+1] == b."""
    t = _u8(t)
    out = np.zeros(65536, dtype=np.uint64)
    _load().oracle_bigram(_ptr(t), t.size, out.ctypes.data)
    return out.reshape(256, 256)


def order_bigram(p, h, bg) -> np.ndarray:
    p = _u8(p)
    h = np.ascontiguousarray(h, dtype=np.uint64)
    bg = np.ascontiguousarray(bg, dtype=np.uint64).reshape(65536)
    out = np.zeros(max(p.size, 1), dtype=np.int32)
    if _load().oracle_order_bigram(_ptr(p), p.size, h.ctypes.data, bg.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("bad pattern length")
    return out[:p.size]


def alg4_count(p, t, order=None, r: int = 2) -> int:
    p, t = _u8(p), _u8(t)
    o = None
    if order is not None:
        o = np.ascontiguousarray(order, dtype=np.int32)
        assert o.size == p.size
    res = _load().oracle_alg4_count(_ptr(p), p.size, _ptr(t), t.size,
                                    o.ctypes.data if o is not None else None, r)
    if res < 0:
        raise ValueError("pattern length must be >= 1")
    return int(res)
