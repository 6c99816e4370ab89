"""C-ABI library checks that need no GPU: exports, argument validation, host-side orders."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1612_01506_amd as sm
from paper_1612_01506_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "sm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    syms = header_symbols()
    assert syms, "no declarations parsed"
    for name in syms:
        assert hasattr(lib, name), name
    assert set(syms) == set(_lib.EXPORTS)


def test_version():
    assert sm.version() == 10200


def _err(rc):
    assert rc < 0
    return _lib.load().sm_last_error().decode()


def test_validation_before_any_device_call():
    lib = _lib.load()
    p = np.frombuffer(b"abc", dtype=np.uint8)
    # m == 0
    assert "m must be" in _err(lib.sm_count(p.ctypes.data, 0, None, 0, None))
    # p NULL
    assert lib.sm_count(None, 3, None, 0, None) == _lib.SM_EINVAL
    # order not a permutation
    bad = np.array([0, 0, 2], dtype=np.int32)
    assert "permutation" in _err(lib.sm_count(p.ctypes.data, 3, None, 0, bad.ctypes.data))
    bad = np.array([0, 1, 3], dtype=np.int32)
    assert "permutation" in _err(lib.sm_count(p.ctypes.data, 3, None, 0, bad.ctypes.data))
    bad = np.array([0, -1, 2], dtype=np.int32)
    assert "permutation" in _err(lib.sm_count(p.ctypes.data, 3, None, 0, bad.ctypes.data))
    # m >= 2^32
    assert "2^32" in _err(lib.sm_count(p.ctypes.data, 1 << 32, None, 0, None))
    # t NULL with n > 0
    assert "t is NULL" in _err(lib.sm_count(p.ctypes.data, 3, None, 10, None))
    # report: pos NULL with cap > 0
    assert lib.sm_report(p.ctypes.data, 3, None, 0, None, None, 5) == _lib.SM_EINVAL
    # batch: NULL arrays
    assert lib.sm_count_batch(None, 1, None, 0, None, None, None) == _lib.SM_EINVAL
    # batch plans: NULL arrays, NULL output handle, NULL plan
    h = ctypes.c_void_p(1)
    assert lib.sm_batch_create(None, 1, None, 0, None, ctypes.byref(h)) == _lib.SM_EINVAL
    assert h.value is None
    assert lib.sm_batch_create(None, 0, None, 0, None, None) == _lib.SM_EINVAL
    assert "NULL" in _err(lib.sm_batch_run(None, None, None))
    assert lib.sm_batch_destroy(None) == _lib.SM_OK
    # sm_params fields out of range are rejected, never replaced by defaults
    for fields, word in (((0, 32, 0, 0), "tile_kib"), ((0, 3, 0, 0), "tile_kib"), ((9, 0, 0, 0), "peel"),
                         ((-1, 0, 0, 0), "peel"), ((0, 0, 33, 0), "wgs_per_cu"), ((0, 0, -2, 0), "wgs_per_cu")):
        bad = _lib.sm_params(*fields)
        assert word in _err(lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(bad), None)), fields
    for field, val in (("bm_chunk", 32), ("bm_chunk", 2048), ("peel", 9), ("bm_min", -1)):
        bt = _lib.sm_batch_tune()
        getattr(bt, field)[2] = val
        bad = _lib.sm_params(0, 0, 0, 0)
        bad.batch = ctypes.pointer(bt)
        assert "sm_batch_tune" in _err(lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(bad), None))
    for field, val in (("tile_kib", 12), ("deal_wgs_per_cu", 65), ("wgs_per_cu", 40)):
        bt = _lib.sm_batch_tune()
        setattr(bt, field, val)
        bad = _lib.sm_params(0, 0, 0, 0)
        bad.batch = ctypes.pointer(bt)
        assert "sm_batch_tune" in _err(lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(bad), None))
    good = _lib.sm_params(8, 16, 32, 0)
    assert lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(good), None) == 0
    # SM_BITMAP: bitmap tiles of 8, 16 or 32 KiB (32 only with the flag, 4 only without)
    for tile in (8, 16, 32):
        ok = _lib.sm_params(0, tile, 0, _lib.SM_BITMAP)
        assert lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(ok), None) == 0   # m > n
    for tile in (4, 12, 64):
        bad = _lib.sm_params(0, tile, 0, _lib.SM_BITMAP)
        assert "SM_BITMAP" in _err(lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(bad), None))
    both = _lib.sm_params(0, 16, 0, _lib.SM_BITMAP | _lib.SM_NONOVERLAP)
    assert lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(both), None) == 0
    # sm_params.flags: unknown bits everywhere, SM_NONOVERLAP outside the synchronous calls
    bad_flags = _lib.sm_params(0, 0, 0, 4)
    assert "flags" in _err(lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(bad_flags), None))
    no = _lib.sm_params(0, 0, 0, _lib.SM_NONOVERLAP)
    assert lib.sm_count_ex(p.ctypes.data, 3, None, 0, None, ctypes.byref(no), None) == 0   # m > n: no device work
    assert "synchronous" in _err(lib.sm_count_async(p.ctypes.data, 3, None, 0, None, ctypes.byref(no), 8, None))
    assert "synchronous" in _err(lib.sm_report_async(p.ctypes.data, 3, None, 0, None, ctypes.byref(no), None, 0, 8,
                                                     None))
    q = np.zeros(1, dtype=sm._QUERY_DT)
    assert "synchronous" in _err(lib.sm_count_batch(q.ctypes.data_as(ctypes.POINTER(_lib.sm_query)), 1, None, 0, 8,
                                                    ctypes.byref(no), None))
    # reporting batch: NULL caps / totals
    assert "caps" in _err(lib.sm_report_batch(q.ctypes.data_as(ctypes.POINTER(_lib.sm_query)), 1, None, 0, None,
                                              None, 8, None, None))
    assert lib.sm_report_batch(None, 0, None, 0, None, None, None, None, None) == _lib.SM_OK
    # histogram: NULL output
    assert lib.sm_histogram(None, 0, None, None) == _lib.SM_EINVAL


def test_text_must_be_device_memory():
    """A host pointer as text is rejected (needs the HIP runtime, which may be absent here)."""
    lib = _lib.load()
    p = np.frombuffer(b"abc", dtype=np.uint8)
    t = np.frombuffer(b"xxabcxx", dtype=np.uint8)
    rc = lib.sm_count(p.ctypes.data, 3, t.ctypes.data, t.size, None)
    assert rc in (_lib.SM_EINVAL, _lib.SM_EDEVICE)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 64, 1000, 1023, 1024, 5000])
def test_library_orders_match_oracle(m):
    """Below 1024 bytes the library ranks the pattern's own symbols, from 1024 on the whole histogram."""
    g = np.random.default_rng(m)
    p = g.integers(0, 256, size=m, dtype=np.uint8).tobytes()
    p = bytes(b if g.random() > 0.2 else 0x20 for b in p)
    h = g.integers(0, 30, size=256).astype(np.uint64)
    assert sm.order("freq", p, h).tolist() == oracle.order_freq(p, h).tolist()
    assert sm.order("h", p).tolist() == oracle.order_h(m).tolist()
    assert sm.order("hs", p).tolist() == oracle.order_hs(p).tolist()
    assert sm.order("ltr", p).tolist() == list(range(m))


def test_order_errors():
    with pytest.raises(sm.SmError):
        sm.order("freq", b"abc")          # needs a histogram
    with pytest.raises(ValueError):
        sm.order("h", b"")


def test_freq_order_ties_and_skew():
    """Equal frequencies of different symbols keep position order (ties across symbols)."""
    h = np.zeros(256, np.uint64)
    h[ord("a")] = 5
    h[ord("b")] = 5
    h[ord("c")] = 1
    h[ord("d")] = 9
    for p in (b"abcdab", b"ddddc", b"babab", b"c", bytes(range(256)), b"dcba" * 50, b"dcba" * 300,
              bytes(range(256)) * 5):
        assert sm.order("freq", p, h).tolist() == oracle.order_freq(p, h).tolist()
    # frequencies too large to pack next to a symbol in 64 bits
    big = np.full(256, 1 << 60, dtype=np.uint64)
    big[ord("x")] = (1 << 60) - 1
    big[ord("y")] = 3
    for p in (b"axbyxa", b"yyxxaa" * 200):
        assert sm.order("freq", p, big).tolist() == oracle.order_freq(p, big).tolist()


@pytest.mark.parametrize("seed", range(6))
def test_library_bigram_order_matches_oracle(seed):
    """The library's heap-based bigram order equals the oracle's direct definition."""
    g = np.random.default_rng(seed)
    sigma = [2, 4, 20, 95, 256, 3][seed]
    # a correlated text: each symbol mostly followed by one favourite successor
    fav = g.integers(0, sigma, size=sigma)
    t = np.empty(20_000, dtype=np.int64)
    t[0] = 0
    r = g.random(t.size)
    x = g.integers(0, sigma, size=t.size)
    for i in range(1, t.size):
        t[i] = fav[t[i - 1]] if r[i] < 0.6 else x[i]
    t = (t % 256).astype(np.uint8)
    h, bg = oracle.hist(t), oracle.bigram(t)
    for m in (1, 2, 3, 8, 33, 200, 1500):
        o = g.integers(0, t.size - m)
        p = bytes(t[o:o + m]) if g.random() < 0.8 else bytes(g.integers(0, 256, size=m, dtype=np.uint8))
        assert sm.order("bigram", p, h, bg).tolist() == oracle.order_bigram(p, h, bg).tolist(), (seed, m)


def test_bigram_order_validation():
    lib = _lib.load()
    p = np.frombuffer(b"abc", dtype=np.uint8)
    h = np.ones(256, dtype=np.uint64)
    out = np.zeros(3, dtype=np.int32)
    assert "NULL" in _err(lib.sm_order_bigram(p.ctypes.data, 3, h.ctypes.data, None, out.ctypes.data))
    assert "m must be" in _err(lib.sm_order_bigram(p.ctypes.data, 0, h.ctypes.data, h.ctypes.data, out.ctypes.data))
    with pytest.raises(ValueError):
        sm.order("bigram", b"abc", h)
    assert lib.sm_bigram(None, 0, None, None, None) == _lib.SM_EINVAL
