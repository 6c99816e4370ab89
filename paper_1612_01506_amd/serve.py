"""Continuous-batching search service over device-resident texts.

Requests (text id, pattern, count or report mode) arrive at any time.  The
scheduler keeps up to `max_inflight` device batches in flight on separate
streams; whenever a slot frees up, every request queued by then (up to
`max_batch`) is admitted and sent to the device in one batched count
(sm_count_batch: one persistent launch shared by all patterns of a text).
A reporting request is counted first; its position buffer (count x 8 bytes)
is then reserved against an HBM budget.  Reporting requests whose buffers fit
go, as many as fit, into one batched report (sm_report_batch: one shared pass
per text, then ordered writes per request).  A request whose position list
alone exceeds the budget is rejected; others wait until reserved memory frees
up.

Each request's result is the same alone and in the mix: the counts of a
batch are those of independent searches (Section 1 problem statement, one
per query), and nothing in a batch depends on which other queries share it.

The scheduler is independent of the device: `GpuExecutor` is the executor
that runs on the HIP library; any object with the same methods can drive it.
"""
from __future__ import annotations

import collections
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


@dataclass
class _Flight:
    kind: str                    # "count" or "report"
    handle: object
    reqs: list
    reserved: int = 0
    slot: int = 0


class GpuExecutor:
    """Runs batches on the HIP library: texts and their histograms stay resident in HBM."""

    def __init__(self, texts, nstreams: int = 2):
        import torch

        from . import Text

        self.torch = torch
        self.texts = [t if isinstance(t, Text) else Text(t) for t in texts]
        for t in self.texts:
            t.hist  # symbol histogram computed once, kept for frequency orders and bitmap mode
        dev = self.texts[0].t.device if self.texts else torch.device("cuda:0")
        self.device = dev
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]  # default priority

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
        """[(full count, positions as a device int64 tensor)] per request of the batch."""
        _, pos, htot, _, caps = handle
        out, off = [], 0
        for total, cap in zip(htot.numpy().tolist(), caps):
            out.append((int(total), pos[off:off + min(int(total), cap)]))
            off += cap
        return out


class Server:
    """Continuous batching with memory-based admission of reporting requests."""

    def __init__(self, executor, max_inflight: int | None = None, max_batch: int = 16384,
                 hbm_budget: int = 1 << 30, clock=time.perf_counter, on_done=None):
        """hbm_budget bounds the position buffers of the reporting searches in flight; a
        finished request's buffer belongs to the caller (on_done(request) is called as each
        request finishes, e.g. to consume and drop its positions)."""
        self.ex = executor
        self.on_done = on_done
        self.max_inflight = max_inflight or executor.nslots
        self.max_batch = max_batch
        self.hbm_budget = hbm_budget
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.mem_wait: collections.deque[Request] = collections.deque()
        self.inflight: list[_Flight] = []
        self.reserved = 0
        self.peak_reserved = 0
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
            while self.mem_wait and len(group) < self.max_batch:
                b = 8 * self.mem_wait[0].count
                if self.reserved + need + b > self.hbm_budget:
                    break
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
        # everything queued so far goes into one batched count
        while self.queue and len(self.inflight) < self.max_inflight:
            slot = self._free_slot()
            if slot is None:
                break
            reqs = [self.queue.popleft() for _ in range(min(self.max_batch, len(self.queue)))]
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
                self._release(f.reserved)
                for r, (total, pos) in zip(f.reqs, results):
                    if total != r.count:
                        self._finish_error(r, f"report total {total} != count {r.count}")
                    else:
                        r.positions = pos
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
            self.on_done(r)

    def _finish_error(self, r: Request, msg: str) -> None:
        r.status = "error"
        r.error = msg
        r.t_done = self.clock()
        self.rejected.append(r)
