"""The allocation-free report (sm_patterns_report_noalloc) against the allocating one.

sm_patterns_report_noalloc keeps its scratch in a fixed device array that every
call on the device reuses, so each test makes calls in a row with shrinking
inputs: stale per-vector counts of a longer earlier text must never leak into a
later, shorter report.  Every position list and total is compared element by
element with sm_patterns_report_async (the allocating entry point sharing its
kernels) and with the oracle.  Calls go through the C ABI.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

sm = pytest.importorskip("paper_1612_01506_amd")
from paper_1612_01506_amd import _lib  # noqa: E402

MAX_STARTS = (2**20 + 1024) * 1024 - 15      # the documented limit on n - m + 1


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def patterns(pats):
    return sm.Patterns([bytes(p) for p in pats])


def call(name, ps, i, t, cap, stream=0):
    """Runs one of the two report entry points through the C ABI; returns (rc, positions, total)."""
    lib = _lib.load()
    pos = torch.full((max(cap, 1),), -1, dtype=torch.int64, device=t.device)
    tot = torch.full((1,), -1, dtype=torch.int64, device=t.device)
    rc = getattr(lib, name)(ps._h, i, t.data_ptr(), t.numel(), None, pos.data_ptr() if cap else None, cap,
                            tot.data_ptr(), ctypes.c_void_p(stream))
    torch.cuda.synchronize()
    return rc, pos[:cap].cpu().numpy(), int(tot.item())


def check_pair(ps, i, t, t_host, p, cap):
    rc_a, pos_a, tot_a = call("sm_patterns_report_async", ps, i, t, cap)
    rc_n, pos_n, tot_n = call("sm_patterns_report_noalloc", ps, i, t, cap)
    assert rc_a == 0 and rc_n == 0, _lib.load().sm_last_error()
    assert tot_n == tot_a
    k = min(cap, tot_a)
    assert np.array_equal(pos_n[:k], pos_a[:k])
    assert (pos_n[k:] == -1).all()                         # nothing written past min(total, cap)
    if t_host is not None:
        want = oracle.report(p, t_host)
        assert tot_n == want.size
        assert np.array_equal(pos_n[:k].astype(np.uint64), want[:k])
    return tot_n


def test_two_calls_second_smaller(dev):
    g = np.random.default_rng(5150)
    big = synth.zipf_text(5_000_003, 4, 1.0, family=12, stream=1)
    small = big[:200_001].copy()
    p = bytes(big[777:777 + 6])
    ps = patterns([p, b"A", big[4_000_000:4_000_300]])
    tb = torch.from_numpy(big).to(dev)
    ts = torch.from_numpy(small).to(dev)
    # the long text leaves nonzero per-vector counts over ~4900 vectors; the short one uses ~200
    n_big = check_pair(ps, 0, tb, big, p, cap=1 << 20)
    n_small = check_pair(ps, 0, ts, small, p, cap=1 << 20)
    assert n_big > n_small > 0
    # dense matches, a cap, then a long pattern on the short text, then the long text again
    check_pair(ps, 1, tb, big, b"A", cap=12_345)
    check_pair(ps, 1, ts, small, b"A", cap=1 << 18)
    check_pair(ps, 2, ts, small, bytes(big[4_000_000:4_000_300]), cap=8)
    check_pair(ps, 2, tb, big, bytes(big[4_000_000:4_000_300]), cap=8)
    # misaligned views and counts only (cap 0)
    for off in (1, 7, 15):
        v = tb[off:off + 300_000]
        check_pair(ps, 0, v, big[off:off + 300_000], p, cap=1000)
        rc, _, tot = call("sm_patterns_report_noalloc", ps, 0, v, 0)
        assert rc == 0 and tot == oracle.count(p, big[off:off + 300_000])
    # m > n and n == 0
    rc, _, tot = call("sm_patterns_report_noalloc", ps, 2, ts[:100], 4)
    assert rc == 0 and tot == 0
    rc, _, tot = call("sm_patterns_report_noalloc", ps, 0, ts[:0], 4)
    assert rc == 0 and tot == 0
    ps.close()


def test_limit_and_errors(dev):
    """n - m + 1 == the limit is served (a 1 GiB-class text, planted matches); one more is rejected."""
    n = MAX_STARTS + 1                                    # m = 2
    buf = torch.zeros(n + 64, dtype=torch.uint8, device=dev)
    planted = [0, 1_000, (1 << 30) - 5, n - 2]            # the last one is the last valid start
    for s in planted:
        buf[s] = ord("a")
        buf[s + 1] = ord("b")
    ps = patterns([b"ab", b"abc"])
    t = buf[:n]
    rc_n, pos_n, tot_n = call("sm_patterns_report_noalloc", ps, 0, t, 16)
    assert rc_n == 0, _lib.load().sm_last_error()
    assert tot_n == len(planted) and pos_n[:tot_n].tolist() == planted
    rc_a, pos_a, tot_a = call("sm_patterns_report_async", ps, 0, t, 16)
    assert rc_a == 0 and tot_a == tot_n and pos_a[:tot_a].tolist() == planted
    # a second call right after, on a much shorter text
    rc, pos, tot = call("sm_patterns_report_noalloc", ps, 0, buf[:5000], 16)
    assert rc == 0 and tot == 2 and pos[:2].tolist() == [0, 1000]
    # one start more than the limit
    rc, _, _ = call("sm_patterns_report_noalloc", ps, 0, buf[:n + 1], 16)
    assert rc == _lib.SM_EINVAL
    assert "allocation-free" in _lib.load().sm_last_error().decode()
    # m = 3 on the same n has one start fewer than the limit: served
    rc, pos, tot = call("sm_patterns_report_noalloc", ps, 1, t, 16)
    assert rc == 0 and tot == 0
    # bad arguments
    lib = _lib.load()
    tot_d = torch.zeros(1, dtype=torch.int64, device=dev)
    assert lib.sm_patterns_report_noalloc(ps._h, 5, t.data_ptr(), 100, None, None, 0, tot_d.data_ptr(),
                                          None) == _lib.SM_EINVAL
    assert lib.sm_patterns_report_noalloc(ps._h, 0, t.data_ptr(), 100, None, None, 4, tot_d.data_ptr(),
                                          None) == _lib.SM_EINVAL
    assert lib.sm_patterns_report_noalloc(ps._h, 0, t.data_ptr(), 100, None, None, 0, None,
                                          None) == _lib.SM_EINVAL
    ps.close()
    del buf
    torch.cuda.empty_cache()


def test_graph_replays(dev):
    """Captured in a graph and replayed with eager work and rewritten texts between the replays."""
    g = np.random.default_rng(5151)
    n = 1_500_007
    host = [synth.zipf_text(n, 20, 1.0, family=12, stream=k) for k in range(3)]
    t = torch.from_numpy(host[0]).to(dev)
    p = bytes(host[0][1234:1234 + 3])
    ps = patterns([p])
    cap = 100_000
    pos = torch.full((cap,), -1, dtype=torch.int64, device=dev)
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ps.report_noalloc(0, t, pos, tot)                  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ps.report_noalloc(0, t, pos, tot)
    for rep in range(4):
        th = host[rep % 3]
        t.copy_(torch.from_numpy(th))
        pos.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        want = oracle.report(p, th)
        assert int(tot.item()) == want.size, rep
        k = min(cap, want.size)
        assert np.array_equal(pos[:k].cpu().numpy().astype(np.uint64), want[:k]), rep
        # eager work between replays, including an allocation-free call on a shorter text
        short = th[: 10_000 + 1000 * rep]
        rc, sp, st = call("sm_patterns_report_noalloc", ps, 0, torch.from_numpy(short).to(dev), 1000)
        assert rc == 0 and st == oracle.count(p, short)
    ps.close()
