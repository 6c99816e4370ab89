"""Exact string matching on AMD Instinct MI355X (gfx950): Python binding of libsm.

Implements the SIMD naive search of Tarhio, Holub and Giaquinta (arXiv
1612.01506): every (overlapping) occurrence of a byte pattern in a byte text,
pattern symbols compared in a chosen order (Section 2.2) with the first r
compares peeled (Section 2.3).  This module only marshals arguments to the C
ABI declared in include/sm.h; texts live in device memory as torch uint8
tensors, patterns are host bytes.

    import torch, paper_1612_01506_amd as sm
    t = torch.frombuffer(bytearray(b"abracadabra"), dtype=torch.uint8).cuda()
    sm.count(t, b"abra")                    # 2
    sm.count(t, b"abra", order="freq")      # 2, rarest symbols compared first
    sm.report(t, b"a")                      # tensor([0, 3, 5, 7, 10])
"""
from __future__ import annotations

import array
import ctypes
from operator import itemgetter
from typing import Iterable, Sequence

import numpy as np
import torch

from ._lib import (SM_BITMAP, SM_NONOVERLAP, SM_ORDER_FREQ, SM_ORDER_H, SM_ORDER_HS, SM_ORDER_LTR, SmError, check, load,
                   sm_batch_tune, sm_params, sm_query, sm_text)

__all__ = ["Text", "PackedTexts", "Patterns", "SmError", "histogram", "order", "count", "count_async", "report",
           "report_async", "count_batch", "report_batch", "BatchPlan", "bigram", "version", "device_cus"]

ORDER_KINDS = {"ltr": SM_ORDER_LTR, "freq": SM_ORDER_FREQ, "h": SM_ORDER_H, "hs": SM_ORDER_HS}


# ------------------------------------------------------------------ marshalling
def _pat(p) -> np.ndarray:
    if isinstance(p, (bytes, bytearray, memoryview)):
        a = np.frombuffer(bytes(p), dtype=np.uint8)
    elif isinstance(p, str):
        a = np.frombuffer(p.encode(), dtype=np.uint8)
    elif isinstance(p, torch.Tensor):
        a = p.detach().cpu().numpy()
    else:
        a = np.asarray(p)
    if a.dtype != np.uint8:
        raise TypeError("pattern must be uint8 bytes")
    return np.ascontiguousarray(a.reshape(-1))


def _ptr(a: np.ndarray | None):
    return None if a is None or a.size == 0 else a.ctypes.data


def _dev_text(t) -> tuple[int, int]:
    if isinstance(t, Text):
        t = t.t
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError("text must be a CUDA (HIP) torch.uint8 tensor")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError("text must be a contiguous 1-D tensor")
    return t.data_ptr(), t.numel()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _batch_params(peel=None, tile_kib=None, wgs_per_cu=None, tune=True):
    """sm_params for a batched call: explicit values, else the tuning table's batch section for
    this device (tune=True) or the given dict of the same form (bm_min, bm_chunk, peel: four
    values per alphabet class; tile_kib, wgs_per_cu, deal_wgs_per_cu), passed as an
    sm_batch_tune record, else the library's defaults."""
    if peel is not None or tile_kib is not None or wgs_per_cu is not None or tune is False or tune is None:
        return _params(peel, tile_kib, wgs_per_cu)
    if isinstance(tune, dict):
        bt = {"bm_min": [0] * 4, "bm_chunk": [0] * 4, "peel": [0] * 4, **tune}
    else:
        from . import autotune
        bt = autotune.batch_tune()
        if bt is None:
            return None
    rec = sm_batch_tune()
    for c in range(4):
        rec.bm_min[c] = int(bt["bm_min"][c])
        rec.bm_chunk[c] = int(bt["bm_chunk"][c])
        rec.peel[c] = int(bt["peel"][c])
    rec.tile_kib = int(bt.get("tile_kib", 0))
    rec.wgs_per_cu = int(bt.get("wgs_per_cu", 0))
    rec.deal_wgs_per_cu = int(bt.get("deal_wgs_per_cu", 0))
    p = sm_params(0, 0, 0, 0)
    p.batch = ctypes.pointer(rec)
    p._keep = rec
    return ctypes.byref(p)


def _params(peel=None, tile_kib=None, wgs_per_cu=None, text=None, m=None, overlap: bool = True, bitmap=None):
    """sm_params for a call; with no tuning given and a Text whose histogram is known, the
    autotuner's table (if one exists for this device) supplies it, the compare mode included.
    overlap=False selects the non-overlapping mode (SM_NONOVERLAP); bitmap=True / False asks for
    or declines the bitmap compares of count calls (SM_BITMAP; None: the table's choice)."""
    flags = 0 if overlap else SM_NONOVERLAP
    if bitmap:
        flags |= SM_BITMAP
    if peel is None and tile_kib is None and wgs_per_cu is None:
        if isinstance(text, Text) and text._hist is not None and m:
            from . import autotune
            tp = autotune.params_for(text._hist, int(m), text.n)
            if tp:
                cell_bm = bool(tp.get("bitmap"))
                if bitmap is None and cell_bm:
                    flags |= SM_BITMAP
                # the cell's tile size is in the units of its own mode
                tile = tp["tile_kib"] if cell_bm == bool(flags & SM_BITMAP) else 0
                return ctypes.byref(sm_params(tp["peel"], tile, tp["wgs_per_cu"], flags))
        return ctypes.byref(sm_params(0, 0, 0, flags)) if flags else None
    return ctypes.byref(sm_params(int(peel or 0), int(tile_kib or 0), int(wgs_per_cu or 0), flags))


# ---------------------------------------------------------------------- texts
class Text:
    """A device-resident text and its lazily computed symbol histogram (Section 2.2)."""

    def __init__(self, t: torch.Tensor):
        _dev_text(t)
        self.t = t
        self._hist: np.ndarray | None = None
        self._bigram: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.t.numel()

    @property
    def hist(self) -> np.ndarray:
        if self._hist is None:
            self._hist = histogram(self.t).cpu().numpy().view(np.uint64).copy()
        return self._hist

    @property
    def bigram(self) -> np.ndarray:
        """(256, 256) adjacent-pair counts, computed on the device once."""
        if self._bigram is None:
            self._bigram = bigram(self.t, self.hist).cpu().numpy().view(np.uint64).copy()
        return self._bigram


def version() -> int:
    return int(load().sm_version())


def device_cus() -> int:
    return check(load().sm_device_cus())


def histogram(t, stream=None) -> torch.Tensor:
    """hist[b] = number of text bytes equal to b, as a device int64 tensor of 256 (asynchronous)."""
    ptr, n = _dev_text(t)
    dev = t.t.device if isinstance(t, Text) else t.device
    out = torch.empty(256, dtype=torch.int64, device=dev)
    check(load().sm_histogram(ptr, n, out.data_ptr(), _stream(stream)))
    return out


def bigram(t, hist=None, stream=None) -> torch.Tensor:
    """Adjacent-pair counts: (256, 256) device int64 tensor, [a, b] = #{s : t[s] == a, t[s+1] == b}
    (asynchronous).  hist is accepted for compatibility and ignored: the table never depends on it."""
    ptr, n = _dev_text(t)
    dev = t.t.device if isinstance(t, Text) else t.device
    h = None if hist is None else np.ascontiguousarray(np.asarray(hist).astype(np.uint64))
    out = torch.empty((256, 256), dtype=torch.int64, device=dev)
    check(load().sm_bigram(ptr, n, _ptr(h), out.data_ptr(), _stream(stream)))
    return out


def order(kind: str, p, hist=None, bigram=None) -> np.ndarray:
    """Compare order pi (0-based permutation): 'ltr', 'freq' (needs hist), 'h', 'hs' or 'bigram'
    (needs hist and the (256, 256) pair counts)."""
    a = _pat(p)
    if a.size == 0:
        raise ValueError("pattern length must be >= 1")
    h = None
    if hist is not None:
        h = np.ascontiguousarray(np.asarray(hist).astype(np.uint64))
        if h.size != 256:
            raise ValueError("hist must have 256 entries")
    out = np.empty(a.size, dtype=np.int32)
    if kind == "bigram":
        if h is None or bigram is None:
            raise ValueError("the bigram order needs hist and bigram")
        bg = np.ascontiguousarray(np.asarray(bigram).astype(np.uint64)).reshape(-1)
        if bg.size != 65536:
            raise ValueError("bigram must have 256 x 256 entries")
        check(load().sm_order_bigram(_ptr(a), a.size, _ptr(h), _ptr(bg), out.ctypes.data))
        return out
    check(load().sm_order(ORDER_KINDS[kind], _ptr(a), a.size, _ptr(h), out.ctypes.data))
    return out


def _resolve_order(order_arg, p: np.ndarray, text) -> np.ndarray | None:
    if order_arg is None or (isinstance(order_arg, str) and order_arg == "ltr"):
        return None
    if isinstance(order_arg, str):
        if order_arg in ("freq", "bigram"):
            if not isinstance(text, Text):
                text = Text(text)
            if order_arg == "bigram":
                return order("bigram", p, text.hist, text.bigram)
            return order("freq", p, text.hist)
        return order(order_arg, p)
    o = np.ascontiguousarray(np.asarray(order_arg, dtype=np.int32))
    if o.size != p.size:
        raise ValueError("order must have one entry per pattern position")
    return o


# -------------------------------------------------------------------- searches
def count(t, p, order=None, peel=None, tile_kib=None, wgs_per_cu=None, stream=None, overlap: bool = True,
          bitmap=None) -> int:
    """Number of occurrences of p in t; synchronous.  All starts are counted (overlapping
    occurrences included); overlap=False counts disjoint occurrences taken greedily from the left.
    bitmap=True compares through per-tile symbol bitmaps (patterns of at most 4 distinct symbols;
    tile_kib is then 8, 16 or 32)."""
    a = _pat(p)
    ptr, n = _dev_text(t)
    o = _resolve_order(order, a, t)
    return check(load().sm_count_ex(_ptr(a), a.size, ptr, n, _ptr(o),
                                    _params(peel, tile_kib, wgs_per_cu, t, a.size, overlap, bitmap),
                                    _stream(stream)))


def count_async(t, p, out: torch.Tensor, order=None, peel=None, tile_kib=None, wgs_per_cu=None,
                stream=None, bitmap=None) -> None:
    """ADD the count of p in t to out[0] (device int64) without waiting."""
    a = _pat(p)
    ptr, n = _dev_text(t)
    if out.dtype != torch.int64 or not out.is_cuda:
        raise TypeError("out must be a CUDA int64 tensor")
    o = _resolve_order(order, a, t)
    check(load().sm_count_async(_ptr(a), a.size, ptr, n, _ptr(o),
                                _params(peel, tile_kib, wgs_per_cu, t, a.size, bitmap=bitmap),
                                out.data_ptr(), _stream(stream)))


def report(t, p, order=None, cap: int | None = None, peel=None, tile_kib=None, wgs_per_cu=None,
           stream=None, return_count: bool = False, overlap: bool = True):
    """Increasing 0-based start positions of p in t (device int64 tensor); synchronous.

    With cap given, at most cap positions are written; return_count=True also
    returns the full count (> cap means truncated).  overlap=False reports the
    disjoint occurrences taken greedily from the left.
    """
    a = _pat(p)
    ptr, n = _dev_text(t)
    o = _resolve_order(order, a, t)
    dev = t.t.device if isinstance(t, Text) else t.device
    params = _params(peel, tile_kib, wgs_per_cu, t, a.size, overlap)
    if cap is None:
        cap = check(load().sm_count_ex(_ptr(a), a.size, ptr, n, _ptr(o), params, _stream(stream)))
    pos = torch.empty(max(int(cap), 1), dtype=torch.int64, device=dev)
    total = check(load().sm_report_ex(_ptr(a), a.size, ptr, n, _ptr(o), params, pos.data_ptr(), int(cap),
                                      _stream(stream)))
    out = pos[:min(total, int(cap))]
    return (out, total) if return_count else out


def report_async(t, p, out: torch.Tensor, total: torch.Tensor, order=None, peel=None, tile_kib=None,
                 wgs_per_cu=None, stream=None) -> None:
    """Write up to out.numel() increasing positions of p in t into out and the full count into
    total[0] (device int64), without waiting."""
    a = _pat(p)
    ptr, n = _dev_text(t)
    o = _resolve_order(order, a, t)
    check(load().sm_report_async(_ptr(a), a.size, ptr, n, _ptr(o), _params(peel, tile_kib, wgs_per_cu, t, a.size),
                                 out.data_ptr(), out.numel(), total.data_ptr(), _stream(stream)))


_QUERY_DT = np.dtype([("text_id", "<u4"), ("flags", "<u4"), ("p", "<u8"), ("m", "<u8"), ("order", "<u8")])
_TEXT_DT = np.dtype([("t", "<u8"), ("n", "<u8"), ("hist", "<u8")])


class PackedTexts:
    """Many texts stored back to back in one device uint8 buffer: text i is
    buf[offsets[i] : offsets[i] + lengths[i]].  hists (optional, host, shape
    (ntexts, 256)) enables frequency orders and the bitmap mode.  They are
    symbol frequencies of any provenance (each text's own, another text's of
    the same kind, an estimate): they steer the compare order, the peel and
    the kernel only, and counts stay exact whatever their values."""

    def __init__(self, buf: torch.Tensor, offsets, lengths, hists=None):
        _dev_text(buf)
        self.buf = buf
        self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
        if self.offsets.shape != self.lengths.shape:
            raise ValueError("offsets and lengths differ in size")
        if self.offsets.size and int((self.offsets + self.lengths).max()) > buf.numel():
            raise ValueError("a text runs past the end of the buffer")
        self.hists = None if hists is None else np.ascontiguousarray(hists, dtype=np.uint64).reshape(-1, 256)

    def __len__(self):
        return int(self.offsets.size)

    def table(self) -> np.ndarray:
        if getattr(self, "_table", None) is not None:
            return self._table
        t = np.zeros(max(len(self), 1), dtype=_TEXT_DT)
        t["t"][:len(self)] = np.uint64(self.buf.data_ptr()) + self.offsets
        t["n"][:len(self)] = self.lengths
        if self.hists is not None:
            t["hist"][:len(self)] = np.uint64(self.hists.ctypes.data) + 2048 * np.arange(len(self), dtype=np.uint64)
        self._table = t  # the buffer, offsets, lengths and histograms are fixed at construction
        return t


def _marshal_batch(texts, queries, use_hist: bool):
    """(query array, text array, #texts, #queries, device, objects to keep alive) for the batch calls."""
    assert _TEXT_DT.itemsize == ctypes.sizeof(sm_text) and _QUERY_DT.itemsize == ctypes.sizeof(sm_query)
    keep = []
    dev = None
    if isinstance(texts, PackedTexts):
        tarr, dev = texts.table(), texts.buf.device
        keep.append(texts)
        texts = [None] * len(texts)
    else:
        texts = list(texts)
        tarr = np.zeros(max(len(texts), 1), dtype=_TEXT_DT)
        for i, tx in enumerate(texts):
            ptr, n = _dev_text(tx)
            dev = dev or (tx.t.device if isinstance(tx, Text) else tx.device)
            h = 0
            if use_hist and isinstance(tx, Text):
                ha = np.ascontiguousarray(tx.hist, dtype=np.uint64)
                keep.append(ha)
                h = ha.ctypes.data
            tarr[i] = (ptr, n, h)
    qs = list(queries)
    nq = len(qs)
    qarr = np.zeros(max(nq, 1), dtype=_QUERY_DT)
    if nq:
        sizes = set(map(len, qs))
        tids = list(map(itemgetter(0), qs))         # column-wise in C (twice as fast as zip(*qs))
        raw = list(map(itemgetter(1), qs))
        if set(map(type, raw)) == {bytes}:          # fast path: one join, no per-pattern arrays
            blob = np.frombuffer(b"".join(raw) or b"\0", dtype=np.uint8)
            lens = np.frombuffer(array.array("Q", map(len, raw)), dtype=np.uint64)
        else:
            pats = [_pat(p) for p in raw]
            lens = np.fromiter((p.size for p in pats), dtype=np.uint64, count=nq)
            blob = np.concatenate(pats) if int(lens.sum()) else np.zeros(1, dtype=np.uint8)
        keep.append(blob)
        offs = np.empty(nq, dtype=np.uint64)
        offs[0] = 0
        np.cumsum(lens[:-1], out=offs[1:])
        qarr["text_id"][:nq] = np.frombuffer(array.array("q", tids), dtype=np.int64).astype(np.uint32)
        qarr["p"][:nq] = offs + np.uint64(blob.ctypes.data)   # an empty pattern is rejected whatever p is
        qarr["m"][:nq] = lens
        for i, q in (enumerate(qs) if max(sizes) > 2 else ()):   # queries with their own order
            if len(q) > 2 and q[2] is not None:
                tid = int(q[0])
                tx = texts[tid] if 0 <= tid < len(texts) else None
                o = _resolve_order(q[2], _pat(raw[i]), tx)
                if o is not None:
                    keep.append(o)
                    qarr["order"][i] = o.ctypes.data
    return qarr, tarr, len(texts), nq, dev, keep


def count_batch(texts: Sequence, queries: Iterable, peel=None, tile_kib=None, wgs_per_cu=None,
                stream=None, use_hist: bool = True, tune: bool = True) -> torch.Tensor:
    """Counts of many (text_id, pattern[, order]) queries in a few persistent launches (asynchronous).

    Returns a device int64 tensor with one count per query.  Queries without an
    explicit order use the frequency order when the text's histogram is known
    (texts given as Text objects and use_hist), else left to right.  Texts with
    a histogram and at least 32 queries (or the tuned threshold of their alphabet
    class) run in the bitmap mode.  With no explicit peel / tile_kib / wgs_per_cu
    and tune, the tuning table's batch section for this device is passed.
    """
    qarr, tarr, nt, nq, dev, keep = _marshal_batch(texts, queries, use_hist)
    out = torch.empty(max(nq, 1), dtype=torch.int64, device=dev or "cuda")
    check(load().sm_count_batch(qarr.ctypes.data_as(ctypes.POINTER(sm_query)), nq,
                                tarr.ctypes.data_as(ctypes.POINTER(sm_text)), nt, out.data_ptr(),
                                _batch_params(peel, tile_kib, wgs_per_cu, tune), _stream(stream)))
    del keep
    return out[:nq]


def report_batch(texts: Sequence, queries: Iterable, caps, peel=None, tile_kib=None, wgs_per_cu=None,
                 stream=None, use_hist: bool = True, tune: bool = True):
    """Ordered start positions of many (text_id, pattern[, order]) queries, one pass per text
    (asynchronous).  caps[i] bounds query i's list.  Returns (positions, totals): positions is one
    device int64 tensor holding query i's min(total_i, caps[i]) smallest starts at offset
    sum(caps[:i]); totals holds every full count (device int64)."""
    qarr, tarr, nt, nq, dev, keep = _marshal_batch(texts, queries, use_hist)
    caps = np.ascontiguousarray(np.asarray(caps, dtype=np.uint64).reshape(-1))
    if caps.size != nq:
        raise ValueError("one cap per query")
    dev = dev or "cuda"
    pos = torch.empty(max(int(caps.sum()), 1), dtype=torch.int64, device=dev)
    totals = torch.empty(max(nq, 1), dtype=torch.int64, device=dev)
    check(load().sm_report_batch(qarr.ctypes.data_as(ctypes.POINTER(sm_query)), nq,
                                 tarr.ctypes.data_as(ctypes.POINTER(sm_text)), nt, _ptr(caps), pos.data_ptr(),
                                 totals.data_ptr(), _batch_params(peel, tile_kib, wgs_per_cu, tune), _stream(stream)))
    del keep
    return pos, totals[:nq]


class BatchPlan:
    """A batch of (text_id, pattern[, order]) count queries planned and uploaded once (sm_batch_*).

    run() only launches kernels (no allocation, no copy, no synchronisation), so
    it can be captured in a CUDA/HIP graph and replayed.  The texts must stay
    allocated while the plan lives; their contents may change between runs.
    """

    def __init__(self, texts: Sequence, queries: Iterable, peel=None, tile_kib=None, wgs_per_cu=None,
                 use_hist: bool = True, tune: bool = True):
        qarr, tarr, nt, nq, dev, keep = _marshal_batch(texts, queries, use_hist)
        self.nq = nq
        self.device = torch.device(dev) if dev is not None else torch.device("cuda", torch.cuda.current_device())
        self._texts = texts                 # keeps the device texts alive
        h = ctypes.c_void_p()
        check(load().sm_batch_create(qarr.ctypes.data_as(ctypes.POINTER(sm_query)), nq,
                                     tarr.ctypes.data_as(ctypes.POINTER(sm_text)), nt,
                                     _batch_params(peel, tile_kib, wgs_per_cu, tune), ctypes.byref(h)))
        del keep
        self._h = h

    def run(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Overwrites out[:nq] (device int64) with the counts; allocates out when None (not under capture)."""
        if self._h is None:
            raise ValueError("plan is closed")
        if out is None:
            out = torch.empty(max(self.nq, 1), dtype=torch.int64, device=self.device)
        if out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous() or out.numel() < self.nq:
            raise ValueError("out must be a contiguous device int64 tensor with at least nq entries")
        check(load().sm_batch_run(self._h, out.data_ptr(), _stream(stream)))
        return out[:self.nq]

    def close(self) -> None:
        if self._h is not None:
            check(load().sm_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------- prepared patterns
class Patterns:
    """Patterns whose step tables are uploaded to the device once (sm_patterns_*).

    Searches through a Patterns object issue no host-to-device copy, so they can
    run back to back on a stream (or inside a captured graph).
    """

    def __init__(self, patterns, orders=None, hist=None):
        """orders: None (left to right), a list of per-pattern orders (None entries allowed), or one
        of 'ltr', 'freq' (needs hist, the text's 256-entry histogram), 'h', 'hs' for all patterns."""
        pats = [_pat(p) for p in patterns]
        n = len(pats)
        self.m = [int(p.size) for p in pats]
        parr = (ctypes.c_void_p * max(n, 1))(*[_ptr(p) for p in pats])
        marr = (ctypes.c_uint64 * max(n, 1))(*self.m)
        h = ctypes.c_void_p()
        if isinstance(orders, str):
            hh = None
            if hist is not None:
                hh = np.ascontiguousarray(np.asarray(hist).astype(np.uint64))
            check(load().sm_patterns_create_ordered(n, parr, marr, ORDER_KINDS[orders], _ptr(hh),
                                                    ctypes.byref(h)))
        else:
            ords = [None] * n if orders is None else [
                None if o is None else np.ascontiguousarray(np.asarray(o, dtype=np.int32)) for o in orders]
            if len(ords) != n:
                raise ValueError("one order per pattern")
            oarr = (ctypes.c_void_p * max(n, 1))(*[_ptr(o) for o in ords])
            check(load().sm_patterns_create(n, parr, marr, oarr, ctypes.byref(h)))
        self._h = h

    def __len__(self):
        return len(self.m)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(load().sm_patterns_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def count_async(self, i: int, t, out: torch.Tensor, peel=None, tile_kib=None, wgs_per_cu=None,
                    stream=None, bitmap=None) -> None:
        """ADD the count of pattern i in t to out[0] (device int64), asynchronously."""
        ptr, n = _dev_text(t)
        check(load().sm_patterns_count(self._h, i, ptr, n,
                                       _params(peel, tile_kib, wgs_per_cu, t, self.m[i], bitmap=bitmap),
                                       out.data_ptr(), _stream(stream)))

    def count(self, i: int, t, **kw) -> int:
        dev = t.t.device if isinstance(t, Text) else t.device
        out = torch.zeros(1, dtype=torch.int64, device=dev)
        self.count_async(i, t, out, **kw)
        return int(out.item())

    def report(self, i: int, t, out: torch.Tensor, peel=None, tile_kib=None, wgs_per_cu=None,
               stream=None, overlap: bool = True) -> int:
        """Write up to out.numel() increasing positions of pattern i into out; return the full count
        (overlap=False: disjoint occurrences taken greedily from the left)."""
        ptr, n = _dev_text(t)
        return check(load().sm_patterns_report(self._h, i, ptr, n,
                                               _params(peel, tile_kib, wgs_per_cu, t, self.m[i], overlap),
                                               out.data_ptr(), out.numel(), _stream(stream)))

    def report_async(self, i: int, t, out: torch.Tensor, total: torch.Tensor, peel=None, tile_kib=None,
                     wgs_per_cu=None, stream=None) -> None:
        """Positions of pattern i into out (up to out.numel()), full count into total[0]; no wait."""
        ptr, n = _dev_text(t)
        check(load().sm_patterns_report_async(self._h, i, ptr, n, _params(peel, tile_kib, wgs_per_cu, t, self.m[i]),
                                              out.data_ptr(), out.numel(), total.data_ptr(), _stream(stream)))

    def report_noalloc(self, i: int, t, out: torch.Tensor, total: torch.Tensor, peel=None, tile_kib=None,
                       wgs_per_cu=None, stream=None) -> None:
        """As report_async, with the library's fixed device scratch: allocates nothing (usable under
        graph capture).  Texts up to 1 GiB; calls overlapping on one device race."""
        ptr, n = _dev_text(t)
        check(load().sm_patterns_report_noalloc(self._h, i, ptr, n,
                                                _params(peel, tile_kib, wgs_per_cu, t, self.m[i]),
                                                out.data_ptr(), out.numel(), total.data_ptr(), _stream(stream)))
