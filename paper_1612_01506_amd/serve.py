"""Continuous-batching search service over device-resident texts.

Requests (text id, pattern, count or report mode) arrive at any time.  The
scheduler keeps up to `max_inflight` device batches in flight on separate
streams; whenever a slot frees up, the requests queued by then are admitted,
in arrival order, while the batch's estimated device time stays within
`batch_budget_us` (and at most `max_batch` requests), and sent to the device
in one batched count (sm_count_batch: a few persistent launches, each text
tile staged once for all patterns of its text).  The estimate comes from a cost model of the executor
(per text pass, per query by alphabet class and kernel mode), so a burst of
arrivals is split into batches of bounded latency instead of one long one.
A reporting request is counted first; its position buffer (count x 8 bytes)
is then reserved against an HBM budget.  Reporting requests whose buffers fit
go, as many as fit and within the device-time budget, into one batched
report (sm_report_batch: one shared pass per text, then ordered writes per
request).  Each finished report gets its own position buffer, and its
reservation is held until the caller has consumed it: until on_done returns
(the server then drops its reference), or, without on_done, until the caller
calls release().  A request whose position list alone exceeds the budget is
rejected; others wait until reserved memory frees up.

Each request's result is the same alone and in the mix: the counts of a
batch are those of independent searches (Section 1 problem statement, one
per query), and nothing in a batch depends on which other queries share it.

The scheduler is independent of the device: `GpuExecutor` is the executor
that runs on the HIP library; any object with the same methods can drive it.
"""
from __future__ import annotations

import collections
import itertools
import time
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Request", "GpuExecutor", "Server"]


@dataclass
class Request:
    rid: int
    text_id: int
    pattern: bytes
    report: bool = False
    t_submit: float = 0.0
    t_done: float | None = None
    count: int | None = None
    positions: object = None     # reporting mode: increasing start positions (device tensor on the GPU executor)
    status: str = "queued"       # queued, counting, waiting_memory, reporting, done, rejected, error
    error: str | None = None

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_submit


class CostModel:
    """Estimated device time of batched searches, in microseconds (admission only: a result never
    depends on it).

    A batch reads each of its texts once per pass and runs every query over the shared tiles, so
    its cost is, per text touched, one pass over the text plus a per-query term.  The per-query
    term depends on the kernel the text's queries take: fewer than `bitmap_min` queries of a text
    run in byte tiles (compare work per query close to a single search's), more run in bitmap
    mode (one funnel shift and AND per compare, plus one bitmap build per chunk of up to 1024
    queries).  Both terms grow with the text length and depend on the alphabet size (smaller
    alphabets need more compares per start).  The defaults are MI355X measurements:
    single-search and batched launch times per GiB on uniform 2-, 4- and 20-letter and Zipf
    95-letter texts, for patterns of 2 to 1024 symbols.  A report adds its count pass and the
    ordered write, taken as one more byte-tile query plus `report_us`.
    """

    CLASSES = (2, 4, 20, 95)

    def __init__(self, pass_us_per_gib: float = 175.0, byte_us_per_gib=None, bitmap_us_per_gib=None,
                 bitmap_build_us_per_gib: float = 1500.0, bitmap_min: int = 32, bitmap_chunk: int = 1024,
                 report_us: float = 30.0):
        self.pass_us = pass_us_per_gib
        self.byte_us = dict(byte_us_per_gib or {2: 480.0, 4: 250.0, 20: 110.0, 95: 80.0})
        self.bitmap_us = dict(bitmap_us_per_gib or {2: 55.0, 4: 32.0, 20: 20.0, 95: 13.5})
        self.build_us = bitmap_build_us_per_gib
        self.bitmap_min = bitmap_min
        self.bitmap_chunk = bitmap_chunk
        self.report_us = report_us

    @classmethod
    def alphabet_class(cls, nsym: int) -> int:
        """The smallest class at least as large as the text's number of distinct symbols."""
        for c in cls.CLASSES:
            if nsym <= c:
                return c
        return cls.CLASSES[-1]

    def text_cost(self, gib: float, cls: int, k: int) -> float:
        """Device microseconds of k count queries on one text of `gib` GiB in one batch."""
        if k <= 0:
            return 0.0
        if k < self.bitmap_min:
            return gib * (self.pass_us + k * self.byte_us[cls])
        chunks = -(-k // self.bitmap_chunk)
        return gib * (chunks * self.build_us + k * self.bitmap_us[cls])

    def report_cost(self, gib: float, cls: int) -> float:
        return gib * self.byte_us[cls] + self.report_us


class _BatchCost:
    """Running cost of a batch being assembled: per text, its queries so far."""

    def __init__(self, model: CostModel | None, text_info):
        self.model = model
        self.info = text_info          # text id -> (GiB, alphabet class)
        self.k: dict[int, int] = {}
        self.report_us = 0.0
        self.total = 0.0

    def add_count(self, tid: int) -> float:
        """Cost after adding one count query of text tid (not yet committed)."""
        if self.model is None:
            return 0.0
        gib, cls = self.info(tid)
        k = self.k.get(tid, 0)
        return self.total - self.model.text_cost(gib, cls, k) + self.model.text_cost(gib, cls, k + 1)

    def add_report(self, tid: int) -> float:
        if self.model is None:
            return 0.0
        gib, cls = self.info(tid)
        k = self.k.get(tid, 0)
        first = self.model.pass_us * gib if k == 0 else 0.0
        return self.total + first + self.model.report_cost(gib, cls)

    def commit(self, tid: int, total: float) -> None:
        self.k[tid] = self.k.get(tid, 0) + 1
        self.total = total


@dataclass
class _Flight:
    kind: str                    # "count" or "report"
    handle: object
    reqs: list
    reserved: int = 0
    slot: int = 0


class GpuExecutor:
    """Runs batches on the HIP library: texts and their histograms stay resident in HBM."""

    def __init__(self, texts, nstreams: int = 2, cost_model: CostModel | None = None):
        import torch

        from . import Text

        self.torch = torch
        self.texts = [t if isinstance(t, Text) else Text(t) for t in texts]
        for t in self.texts:
            t.hist  # symbol histogram computed once, kept for frequency orders and bitmap mode
        dev = self.texts[0].t.device if self.texts else torch.device("cuda:0")
        self.device = dev
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]  # default priority
        self.cost_model = cost_model or CostModel()
        self._info = [(t.n / float(1 << 30), CostModel.alphabet_class(int(np.count_nonzero(t.hist))))
                      for t in self.texts]

    def text_info(self, tid: int):
        """(GiB, alphabet class) of text tid, for the cost model."""
        return self._info[tid]

    @property
    def nslots(self) -> int:
        return len(self.streams)

    def launch_counts(self, slot: int, reqs: list):
        """One batched count (a lone request takes the single-search path: no batch planning)."""
        from . import count_async, count_batch

        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            if len(reqs) == 1:
                r = reqs[0]
                counts = torch.zeros(1, dtype=torch.int64, device=self.device)
                count_async(self.texts[r.text_id], r.pattern, counts, order="freq", stream=s)
            else:
                counts = count_batch(self.texts, [(r.text_id, r.pattern) for r in reqs], stream=s)
            host = torch.empty(len(reqs), dtype=torch.int64, pin_memory=True)
            host.copy_(counts, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, host, counts)

    def launch_reports(self, slot: int, reqs: list, caps: list):
        """One batched report (a lone request takes the single-search report path, which is
        faster for one pattern)."""
        from . import report_async, report_batch

        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            if len(reqs) == 1:
                r, cap = reqs[0], int(caps[0])
                pos = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
                totals = torch.empty(1, dtype=torch.int64, device=self.device)
                report_async(self.texts[r.text_id], r.pattern, pos[:cap], totals, order="freq", stream=s)
            else:
                pos, totals = report_batch(self.texts, [(r.text_id, r.pattern) for r in reqs], caps, stream=s)
            htot = torch.empty(len(reqs), dtype=torch.int64, pin_memory=True)
            htot.copy_(totals, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, pos, htot, totals, list(caps))

    def ready(self, handle) -> bool:
        return handle[0].query()

    def counts(self, handle) -> np.ndarray:
        return handle[1].numpy().copy()

    def reports(self, handle) -> list:
        """[(full count, positions as a device int64 tensor of its own)] per request of the batch;
        the batch's shared buffer is freed once these copies are made."""
        _, pos, htot, _, caps = handle
        out, off = [], 0
        for total, cap in zip(htot.numpy().tolist(), caps):
            out.append((int(total), pos[off:off + min(int(total), cap)].clone()))
            off += cap
        return out


class Server:
    """Continuous batching with device-time and memory-based admission."""

    def __init__(self, executor, max_inflight: int | None = None, max_batch: int = 16384,
                 hbm_budget: int = 1 << 30, clock=time.perf_counter, on_done=None,
                 batch_budget_us: float | None = 10_000.0, adaptive: bool = True):
        """hbm_budget bounds the position buffers of reporting searches, from their admission until
        the caller has consumed them: on_done(request) is called as each request finishes, and a
        report's reservation is released when on_done returns (the server then drops its
        reference to the positions, so on_done must copy what it keeps); without on_done the
        positions stay on the request and the reservation is held until release(request).
        batch_budget_us bounds the estimated device time of each batch (the executor's
        cost_model and text_info; None, or an executor without them, admits up to max_batch).
        With adaptive, a batch may also take as much device time as its oldest request has
        already waited: under light load batches stay within the budget, and under overload they
        grow with the backlog instead of falling behind at an inefficient size (a batch's texts
        are read once whatever its size, so larger batches serve more requests per second)."""
        self.ex = executor
        self.on_done = on_done
        self.max_inflight = max_inflight or executor.nslots
        self.max_batch = max_batch
        self.hbm_budget = hbm_budget
        self.batch_budget_us = batch_budget_us
        self.adaptive = adaptive
        model = getattr(executor, "cost_model", None)
        self.cost_model = model if (batch_budget_us is not None and hasattr(executor, "text_info")) else None
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.mem_wait: collections.deque[Request] = collections.deque()
        self.inflight: list[_Flight] = []
        self.reserved = 0
        self.peak_reserved = 0
        self.held: dict[int, int] = {}   # request id -> bytes reserved until released
        self.batch_costs_us: list[float] = []
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.batches = 0
        self.batch_sizes: list[int] = []
        self._next_rid = 0

    # ------------------------------------------------------------------ API
    def submit(self, text_id: int, pattern: bytes, report: bool = False, t_submit: float | None = None) -> Request:
        r = Request(self._next_rid, int(text_id), bytes(pattern), bool(report),
                    self.clock() if t_submit is None else t_submit)
        self._next_rid += 1
        if not r.pattern:
            self._finish_error(r, "empty pattern")
            return r
        self.queue.append(r)
        return r

    def idle(self) -> bool:
        return not self.queue and not self.mem_wait and not self.inflight

    def release(self, r: Request) -> None:
        """The caller is done with r.positions: its HBM reservation is returned (reports without
        on_done; a no-op otherwise)."""
        b = self.held.pop(r.rid, 0)
        if b:
            self._release(b)
        r.positions = None

    def step(self) -> int:
        """Collect finished device work, then admit new work into free slots.  Returns #completions."""
        n = self._collect()
        self._admit()
        return n

    def drain(self, timeout: float = 600.0) -> None:
        t_end = self.clock() + timeout
        while not self.idle():
            self.step()
            if self.clock() > t_end:
                raise TimeoutError("server did not drain")

    def stats(self) -> dict:
        out = {"completed": len(self.done), "rejected": len(self.rejected), "batches": self.batches,
               "peak_reserved_bytes": self.peak_reserved, "hbm_budget_bytes": self.hbm_budget}
        for tag, sel in (("", lambda r: True), ("count_", lambda r: not r.report), ("report_", lambda r: r.report)):
            lat = np.array([r.latency for r in self.done if r.latency is not None and sel(r)])
            if lat.size:
                out.update({f"{tag}p50_ms": float(np.percentile(lat, 50) * 1e3),
                            f"{tag}p99_ms": float(np.percentile(lat, 99) * 1e3),
                            f"{tag}mean_ms": float(lat.mean() * 1e3)})
        if self.batch_sizes:
            out["mean_batch"] = float(np.mean(self.batch_sizes))
        if self.batch_costs_us:
            out["max_batch_cost_us"] = float(np.max(self.batch_costs_us))
        return out

    # ------------------------------------------------------------- internals
    def _free_slot(self):
        used = {f.slot for f in self.inflight}
        for s in range(self.ex.nslots):
            if s not in used:
                return s
        return None

    def _admit(self) -> None:
        # reporting searches whose position buffers now fit: as many as fit go into one batch
        while self.mem_wait and len(self.inflight) < self.max_inflight:
            slot = self._free_slot()
            if slot is None:
                break
            group, need = [], 0
            cost = _BatchCost(self.cost_model, getattr(self.ex, "text_info", None))
            budget = self._budget(self.mem_wait[0]) if self.cost_model is not None else 0.0
            while self.mem_wait and len(group) < self.max_batch:
                r = self.mem_wait[0]
                b = 8 * r.count
                if self.reserved + need + b > self.hbm_budget:
                    break
                c = cost.add_report(r.text_id)
                if group and self.cost_model is not None and c > budget:
                    break
                cost.commit(r.text_id, c)
                group.append(self.mem_wait.popleft())
                need += b
            if not group:
                break
            self._reserve(need)
            for r in group:
                r.status = "reporting"
            try:
                h = self.ex.launch_reports(slot, group, [r.count for r in group])
            except Exception as e:  # noqa: BLE001 - a device error fails these requests only
                self._release(need)
                for r in group:
                    self._finish_error(r, str(e))
                continue
            self.inflight.append(_Flight("report", h, group, need, slot))
            self.batch_costs_us.append(cost.total)
        # the requests queued so far go into one batched count, within the device-time budget
        while self.queue and len(self.inflight) < self.max_inflight:
            slot = self._free_slot()
            if slot is None:
                break
            take, total = self._count_prefix()
            reqs = [self.queue.popleft() for _ in range(take)]
            self.batch_costs_us.append(total)
            for r in reqs:
                r.status = "counting"
            try:
                h = self.ex.launch_counts(slot, reqs)
            except Exception as e:  # noqa: BLE001
                for r in reqs:
                    self._finish_error(r, str(e))
                continue
            self.inflight.append(_Flight("count", h, reqs, 0, slot))
            self.batches += 1
            self.batch_sizes.append(len(reqs))

    def _budget(self, oldest: Request) -> float:
        """Device-time budget of the next batch, whose oldest request is `oldest`."""
        if not self.adaptive:
            return self.batch_budget_us
        return max(self.batch_budget_us, (self.clock() - oldest.t_submit) * 1e6)

    def _count_prefix(self) -> tuple[int, float]:
        """How many queued requests, in arrival order, the next count batch takes, and its
        modelled device time: the longest prefix (at least one request, at most max_batch) whose
        modelled time fits the budget.  The model is not monotonic -- a text's queries become
        cheaper when enough of them share a bitmap pass -- so the scan goes on past the first
        prefix over the budget, up to twice the budget."""
        if self.cost_model is None:
            return min(self.max_batch, len(self.queue)), 0.0
        budget = self._budget(self.queue[0])
        cost = _BatchCost(self.cost_model, self.ex.text_info)
        best, best_cost = 1, None
        for i, r in enumerate(itertools.islice(self.queue, self.max_batch)):
            c = cost.add_count(r.text_id)
            cost.commit(r.text_id, c)
            if best_cost is None:
                best_cost = c
            if c <= budget:
                best, best_cost = i + 1, c
            elif c > 2.0 * budget:
                break
        return best, best_cost

    def _collect(self) -> int:
        n = 0
        still = []
        for f in self.inflight:
            if not self.ex.ready(f.handle):
                still.append(f)
                continue
            now = self.clock()
            if f.kind == "count":
                counts = self.ex.counts(f.handle)
                for r, c in zip(f.reqs, counts):
                    r.count = int(c)
                    if r.report and r.count > 0:
                        if 8 * r.count > self.hbm_budget:
                            r.status = "rejected"
                            r.error = f"position list of {8 * r.count} bytes exceeds the HBM budget"
                            r.t_done = now
                            self.rejected.append(r)
                        else:
                            r.status = "waiting_memory"
                            self.mem_wait.append(r)
                        continue
                    if r.report:
                        r.positions = np.zeros(0, dtype=np.int64)
                    self._finish(r, now)
                    n += 1
            else:
                results = self.ex.reports(f.handle)
                for r, (total, pos) in zip(f.reqs, results):
                    b = 8 * r.count
                    if total != r.count:
                        self._release(b)
                        self._finish_error(r, f"report total {total} != count {r.count}")
                        continue
                    r.positions = pos
                    self.held[r.rid] = b       # released when the caller has consumed the positions
                    self._finish(r, now)
                    n += 1
        self.inflight = still
        return n

    def _reserve(self, b: int) -> None:
        self.reserved += b
        self.peak_reserved = max(self.peak_reserved, self.reserved)

    def _release(self, b: int) -> None:
        self.reserved -= b

    def _finish(self, r: Request, now: float) -> None:
        r.status = "done"
        r.t_done = now
        self.done.append(r)
        if self.on_done is not None:
            try:
                self.on_done(r)
            finally:
                if r.rid in self.held:   # consumed: the buffer goes, and its reservation with it
                    self.release(r)

    def _finish_error(self, r: Request, msg: str) -> None:
        r.status = "error"
        r.error = msg
        r.t_done = self.clock()
        self.rejected.append(r)
