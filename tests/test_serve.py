"""Serving scheduler on the CPU: a test-only executor answers with the oracle.

Checks continuous batching (requests arriving while batches are in flight go
into later batches, never more than max_inflight at once), results equal to
independent searches, memory-based admission of reporting requests, and that
failures stay confined to the requests they hit.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_1612_01506_amd.serve import Server


class FakeExecutor:
    """Completes a launch after `delay` polls; counts and positions come from the oracle."""

    def __init__(self, texts, nslots=2, delay=3, fail_batches=()):
        self.texts = texts
        self.nslots = nslots
        self.delay = delay
        self.fail_batches = set(fail_batches)
        self.launches = 0
        self.report_batches = []
        self.active = 0
        self.max_active = 0

    def _start(self):
        self.launches += 1
        self.active += 1
        self.max_active = max(self.max_active, self.active)

    def launch_counts(self, slot, reqs):
        if self.launches in self.fail_batches:
            self.launches += 1
            raise RuntimeError("injected launch failure")
        self._start()
        counts = np.array([oracle.count(r.pattern, self.texts[r.text_id]) for r in reqs], dtype=np.int64)
        return {"left": self.delay, "counts": counts}

    def launch_reports(self, slot, reqs, caps):
        self._start()
        self.report_batches.append(len(reqs))
        res = []
        for r, cap in zip(reqs, caps):
            pos = oracle.report(r.pattern, self.texts[r.text_id])
            res.append((int(pos.size), pos[:cap]))
        return {"left": self.delay, "reports": res}

    def ready(self, h):
        if h["left"] > 0:
            h["left"] -= 1
            return False
        if not h.get("seen"):
            h["seen"] = True
            self.active -= 1
        return True

    def counts(self, h):
        return h["counts"]

    def reports(self, h):
        return h["reports"]


def make_texts():
    return [synth.zipf_text(20_000, 95, 1.0, family=5, stream=i) for i in range(3)] + \
           [synth.uniform_text(20_000, 4, family=5, stream=9)]


def test_results_equal_independent_searches():
    texts = make_texts()
    ex = FakeExecutor(texts, nslots=2, delay=2)
    srv = Server(ex, max_batch=7)
    g = np.random.default_rng(1)
    reqs = []
    for k in range(200):
        ti = int(g.integers(0, len(texts)))
        m = int(synth.loguniform_ints(1, 40, 1, g)[0])
        p = synth.substring_pattern(texts[ti], m, g)[0] if k % 2 else synth.random_pattern(b"ACGT", m, g)
        reqs.append(srv.submit(ti, p, report=(k % 10 == 0)))
        if k % 3 == 0:
            srv.step()
    srv.drain()
    assert all(r.status == "done" for r in reqs)
    for r in reqs:
        assert r.count == oracle.count(r.pattern, texts[r.text_id])
        if r.report:
            assert np.array_equal(np.asarray(r.positions, dtype=np.uint64), oracle.report(r.pattern, texts[r.text_id]))
    assert ex.max_active <= 2
    st = srv.stats()
    assert st["completed"] == 200 and st["rejected"] == 0
    assert st["batches"] > 3            # arrivals during flight were batched later
    assert "p50_ms" in st and "p99_ms" in st


def test_continuous_batching_admits_while_busy():
    texts = make_texts()
    ex = FakeExecutor(texts, nslots=1, delay=5)
    srv = Server(ex)
    first = [srv.submit(0, b"ab") for _ in range(3)]
    srv.step()                          # batch 1 in flight
    late = [srv.submit(1, b"a") for _ in range(4)]
    srv.step()                          # no free slot: late requests wait
    assert all(r.status == "queued" for r in late)
    srv.drain()
    assert srv.batch_sizes == [3, 4]
    assert all(r.status == "done" for r in first + late)


def test_report_memory_admission_and_rejection():
    t = np.frombuffer(b"a" * 1000, dtype=np.uint8)
    ex = FakeExecutor([t], nslots=2, delay=1)
    seen = {}

    def consume(r):  # positions are checked while the server still holds their reservation
        assert srv.reserved >= 8 * r.count
        seen[r.rid] = np.asarray(r.positions, dtype=np.uint64).copy()

    # budget fits one report of "a" (1000 positions = 8000 B) but not two at once
    srv = Server(ex, hbm_budget=10_000, on_done=consume)
    r1 = srv.submit(0, b"a", report=True)
    r2 = srv.submit(0, b"a", report=True)
    r3 = srv.submit(0, b"aa", report=True)  # 999 positions
    big = Server(FakeExecutor([t], nslots=1, delay=0), hbm_budget=1000)
    r4 = big.submit(0, b"a", report=True)   # 8000 B > budget: rejected
    srv.drain()
    big.drain()
    for r in (r1, r2, r3):
        assert r.status == "done" and r.positions is None      # consumed and dropped
        assert np.array_equal(seen[r.rid], oracle.report(r.pattern, t))
    assert srv.peak_reserved <= 10_000 and srv.reserved == 0
    assert r4.status == "rejected" and "budget" in r4.error


def test_report_reservation_held_until_released():
    """Without on_done the positions stay with the request and keep their reservation until the
    caller releases them; a report that does not fit waits for that."""
    t = np.frombuffer(b"ab" * 500, dtype=np.uint8)
    ex = FakeExecutor([t], nslots=2, delay=0)
    srv = Server(ex, hbm_budget=6_000)                # one list of 500 positions (4000 B) at a time
    r1 = srv.submit(0, b"ab", report=True)
    r2 = srv.submit(0, b"ba", report=True)            # 499 positions
    for _ in range(20):
        srv.step()
    assert r1.status == "done" and r2.status == "waiting_memory"
    assert srv.reserved == 8 * r1.count
    assert np.array_equal(np.asarray(r1.positions, dtype=np.uint64), oracle.report(b"ab", t))
    srv.release(r1)
    assert r1.positions is None
    srv.drain()
    assert r2.status == "done" and srv.reserved == 8 * r2.count
    srv.release(r2)
    srv.release(r2)                                   # a second release is a no-op
    assert srv.reserved == 0


class CostedExecutor(FakeExecutor):
    """FakeExecutor with the GPU executor's cost model and per-text (GiB, alphabet class)."""

    def __init__(self, texts, gib, cls=95, **kw):
        super().__init__(texts, **kw)
        from paper_1612_01506_amd.serve import CostModel
        self.cost_model = CostModel()
        self.gib = gib
        self.cls = cls

    def text_info(self, tid):
        return self.gib[tid], self.cls


def test_batches_bounded_by_device_time():
    """A burst is split into batches whose modelled device time stays within the budget, counts and
    reports alike; a request whose cost alone exceeds it still runs, alone."""
    from paper_1612_01506_amd.serve import CostModel
    texts = make_texts()
    # pretend text 0 is 1 GiB and text 1 is 64 GiB: a byte-tile query on the 1 GiB text costs
    # 175 + 80 us, a bitmap query 13.5 us; one query on the 64 GiB text exceeds a 10 ms budget
    ex = CostedExecutor(texts, gib=[1.0, 64.0, 1.0, 1.0], nslots=1, delay=0)
    budget = 10_000.0
    srv = Server(ex, batch_budget_us=budget, adaptive=False)
    g = np.random.default_rng(7)
    reqs = [srv.submit(0, synth.substring_pattern(texts[0], 8, g)[0]) for _ in range(3000)]
    huge = srv.submit(1, b"ab")
    rep = [srv.submit(2, synth.substring_pattern(texts[2], 4, g)[0], report=True) for _ in range(200)]
    srv.drain()
    assert all(r.status == "done" for r in reqs + [huge] + rep)
    for r in reqs[::97] + rep[::17]:
        assert r.count == oracle.count(r.pattern, texts[r.text_id])
    m = CostModel()
    costs = srv.batch_costs_us
    over = [c for c in costs if c > budget]
    assert len(over) == 1 and abs(over[0] - m.text_cost(64.0, 95, 1)) < 1e-6   # the huge one, alone
    assert len(srv.batch_sizes) >= 5 and max(srv.batch_sizes) < 3000
    # bitmap-mode batches hold about (budget - builds) / 13.5 queries of the 1 GiB text
    assert max(srv.batch_sizes) > 600
    assert len(ex.report_batches) >= 2                                        # 200 reports > one batch


def test_no_budget_admits_everything_queued():
    texts = make_texts()
    ex = CostedExecutor(texts, gib=[64.0] * 4, nslots=1, delay=0)
    srv = Server(ex, batch_budget_us=None)
    reqs = [srv.submit(k % 4, b"ab") for k in range(50)]
    srv.drain()
    assert srv.batch_sizes == [50] and all(r.status == "done" for r in reqs)


def test_failures_stay_confined():
    texts = make_texts()
    ex = FakeExecutor(texts, nslots=1, delay=0, fail_batches={0})
    srv = Server(ex)
    bad = [srv.submit(0, b"x") for _ in range(2)]
    srv.step()                          # first launch fails
    good = [srv.submit(1, b"y") for _ in range(2)]
    empty = srv.submit(0, b"")
    srv.drain()
    assert all(r.status == "error" and "injected" in r.error for r in bad)
    assert all(r.status == "done" for r in good)
    assert empty.status == "error"
    with pytest.raises(TimeoutError):
        stuck = Server(FakeExecutor(texts, nslots=1, delay=10**9))
        stuck.submit(0, b"a")
        stuck.drain(timeout=0.05)


def test_reports_share_one_batch():
    """Reporting requests admitted together go to the device as one batched report."""
    texts = make_texts()
    ex = FakeExecutor(texts, nslots=1, delay=1)
    srv = Server(ex)
    g = np.random.default_rng(3)
    reqs = [srv.submit(k % len(texts), synth.substring_pattern(texts[k % len(texts)], 3, g)[0], report=True)
            for k in range(10)]
    srv.drain()
    assert all(r.status == "done" for r in reqs)
    assert ex.report_batches == [10]
    for r in reqs:
        assert np.array_equal(np.asarray(r.positions, dtype=np.uint64), oracle.report(r.pattern, texts[r.text_id]))


def test_prefix_reaches_the_cheaper_bitmap_mode():
    """On a 1 GiB binary text 21 byte-tile queries already exceed 10 ms, while 32 or more share a
    bitmap pass for about 3 ms: the batch takes the longest prefix that fits, past the bump."""
    from paper_1612_01506_amd.serve import CostModel
    texts = make_texts()
    ex = CostedExecutor(texts, gib=[1.0] * 4, cls=2, nslots=1, delay=0)
    srv = Server(ex, batch_budget_us=10_000.0, adaptive=False)
    reqs = [srv.submit(3, b"AC") for _ in range(400)]
    srv.step()
    m = CostModel()
    k = max(k for k in range(1, 401) if m.text_cost(1.0, 2, k) <= 10_000.0)
    assert k >= 100 and m.text_cost(1.0, 2, 21) > 10_000.0
    assert srv.batch_sizes == [k] and srv.batch_costs_us[0] <= 10_000.0
    srv.drain()
    assert all(r.status == "done" and r.count == oracle.count(b"AC", texts[3]) for r in reqs)


def test_adaptive_budget_grows_with_the_wait():
    """With adaptive admission a batch may take as much modelled device time as its oldest request
    has waited: fresh requests get the budget, a backlog that waited 50 ms gets about 50 ms."""
    texts = make_texts()
    now = [0.0]
    ex = CostedExecutor(texts, gib=[1.0] * 4, nslots=1, delay=0)
    srv = Server(ex, batch_budget_us=10_000.0, clock=lambda: now[0])
    fresh = [srv.submit(k % 4, b"ab") for k in range(400)]
    srv.step()
    assert srv.batch_costs_us[-1] <= 10_000.0
    srv.drain()
    late = [srv.submit(k % 4, b"ab", t_submit=0.0) for k in range(4000)]
    now[0] = 0.05                                     # the backlog has waited 50 ms
    srv.step()
    assert 10_000.0 < srv.batch_costs_us[-1] <= 50_000.0
    srv.drain()
    assert all(r.status == "done" for r in fresh + late)
