"""Parity at the benchmark workloads' full sizes, in the launch configurations bench.py times.

Outputs the oracle can compute one by one are compared with it: every count of the
1 GiB Zipf step and 50 of its lists, 100 batched queries spanning the length range
on the 2 GiB text, every count of the 4,096-text batch, and a sample of served
counts and lists at the serving workload's size.  The rest are checked through
properties that hold at any size (batched == single searches, count == report
length, closed forms, order and peel invariance).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

sm = pytest.importorskip("paper_1612_01506_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_single_count_8mib(dev):
    """8 MiB uniform ACGT, m = 16 substring, both compare orders."""
    t, p = synth.single_count_workload()
    td = sm.Text(torch.from_numpy(t).to(dev))
    want = oracle.count(p, t)
    assert sm.count(td, p, order="ltr") == want
    assert sm.count(td, p, order="freq") == want
    assert sm.report(td, p).cpu().numpy().astype(np.uint64).tolist() == oracle.report(p, t).tolist()


def test_zipf_1gib_bench_configuration(dev):
    """1 GiB Zipf text, 100 substrings per m in {2..1024}: prepared frequency-ordered patterns counted
    and reported asynchronously through the resident Text (the tuning table's launch parameters and
    streaming tile loads), exactly as the benchmark step does."""
    t, pats = synth.zipf_workload(n=1 << 30, per_m=100)
    td = torch.from_numpy(t).to(dev)
    text = sm.Text(td)
    hist = text.hist
    assert hist.tolist() == oracle.hist(t).tolist()
    patterns = [p for p, _ in pats]
    ps = sm.Patterns(patterns, "freq", hist)
    counts = torch.zeros(len(patterns), dtype=torch.int64, device=dev)
    for i in range(len(patterns)):
        ps.count_async(i, text, counts[i:i + 1])
    rep = [i for i, (_, r) in enumerate(pats) if r]
    cap = 4096
    pos = torch.empty((len(rep), cap), dtype=torch.int64, device=dev)
    tot = torch.empty(len(rep), dtype=torch.int64, device=dev)
    for k, i in enumerate(rep):
        ps.report_async(i, text, pos[k], tot[k:k + 1])
    torch.cuda.synchronize()
    counts = counts.cpu().numpy()
    tot = tot.cpu().numpy()
    assert (counts >= 1).all()                      # every pattern is a substring of the text
    for k, i in enumerate(rep):
        assert tot[k] == counts[i]
    want_all = [oracle.count(p, t) for p in patterns]   # every count against the oracle (~1 min of host time)
    bad = [(len(patterns[i]), counts[i], want_all[i]) for i in range(len(patterns)) if counts[i] != want_all[i]]
    assert not bad, bad[:5]
    # the default launch (no tuning table: 8 KiB tiles, 6 workgroups per CU) gives the same counts
    plain = torch.zeros(len(patterns), dtype=torch.int64, device=dev)
    for i in range(len(patterns)):
        ps.count_async(i, td, plain[i:i + 1])
    torch.cuda.synchronize()
    assert plain.cpu().numpy().tolist() == counts.tolist()
    for k in range(0, len(rep), 10):                 # 50 reported lists (10 per length) against the oracle
        want = oracle.report(patterns[rep[k]], t)
        got = pos[k, :min(int(tot[k]), cap)].cpu().numpy().astype(np.uint64)
        assert got.tolist() == want[:cap].tolist(), len(patterns[rep[k]])
    ps.close()


def test_batched_one_text_2gib(dev):
    """10,000 patterns on a 2 GiB Zipf text in one launch (bitmap mode): 200 counts against single
    searches, and 100 against the oracle -- 10 per decade-spaced length band over [2, 1024], each
    band half substrings (even indices) and half random patterns (odd)."""
    t, pats = synth.batched_one_text_workload()
    text = sm.Text(torch.from_numpy(t).to(dev))
    got = sm.count_batch([text], [(0, p) for p in pats]).cpu().numpy()
    g = np.random.default_rng(5)
    for i in g.choice(len(pats), size=200, replace=False):   # batched == single searches
        assert got[i] == sm.count(text, pats[i]), i
    edges = np.geomspace(2, 1025, 11)
    picked = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        band = [i for i in range(len(pats)) if lo <= len(pats[i]) < hi]
        for parity in (0, 1):
            idx = [i for i in band if i % 2 == parity]
            picked += list(g.choice(idx, size=min(5, len(idx)), replace=False))
    assert len(picked) >= 100 and min(len(pats[i]) for i in picked) <= 3 and max(len(pats[i]) for i in picked) >= 700
    for i in picked:
        assert got[i] == oracle.count(pats[i], t), (i, len(pats[i]))


def test_batched_many_texts(dev):
    """4,096 texts (4 KiB..4 MiB) with one pattern each, packed in one buffer with histograms;
    every count against the oracle."""
    texts_h, pats = synth.batched_many_texts_workload()
    total = sum(x.size for x in texts_h)
    big = torch.empty(total + 16 * len(texts_h), dtype=torch.uint8, device=dev)
    offs, off = [], 0
    for i, th in enumerate(texts_h):
        off += i % 16
        big[off:off + th.size].copy_(torch.from_numpy(th))
        offs.append(off)
        off += th.size
    views = [big[o:o + th.size] for o, th in zip(offs, texts_h)]
    hists = torch.stack([sm.histogram(v) for v in views]).cpu().numpy().view(np.uint64)
    packed = sm.PackedTexts(big, offs, [x.size for x in texts_h], hists)
    got = sm.count_batch(packed, list(enumerate(pats))).cpu().tolist()
    assert got == [oracle.count(p, th) for p, th in zip(pats, texts_h)]


@pytest.mark.parametrize("sigma", [2, 4])
def test_small_alphabets_1gib(dev, sigma):
    """1 GiB uniform texts over 2 and 4 symbols, m in {8, 64, 512, 4096}: every count in the tuned
    launch (the bitmap compares in most cells, as the benchmark runs it) against the oracle; byte
    compares at peels 2 and 5 and the bitmap compares with 8 KiB tiles give the same counts."""
    t, pats = synth.small_alphabet_workload(n=1 << 30, sigma=sigma)
    text = sm.Text(torch.from_numpy(t).to(dev))
    for p in pats:
        a = sm.count(text, p, order="freq")
        assert a == oracle.count(p, t), (sigma, len(p))
        assert a == sm.count(text, p, order="freq", peel=5, bitmap=False)
        assert a == sm.count(text, p, order="freq", peel=2, bitmap=False)
        assert a == sm.count(text, p, order="freq", tile_kib=8, bitmap=True), (sigma, len(p))


def test_periodic_256mib_closed_forms(dev):
    n = 256 << 20
    td = torch.full((n,), ord("a"), dtype=torch.uint8, device=dev)
    for k in (16, 256):
        for order in ("ltr", "freq"):
            assert sm.count(td, b"a" * k, order=order) == n - k + 1
            assert sm.count(td, b"a" * (k - 1) + b"b", order=order) == 0


def test_text_beyond_4gib(dev):
    """64-bit coordinates: a 4.5 GiB text, patterns planted past 2^32; counts, positions and the
    histogram against the oracle."""
    n = (9 << 30) // 2
    t = synth.uniform_text(n, 4, family=6, stream=3)
    planted = [(1 << 32) + 12_345, n - 40, (3 << 30) + 7]
    p = b"GATTACAGATTACAGG"
    for o in planted:
        t[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    td = torch.from_numpy(t).to(dev)
    text = sm.Text(td)
    assert text.hist.tolist() == oracle.hist(t).tolist()
    want = oracle.report(p, t)
    assert set(planted) <= set(want.tolist())
    assert sm.count(text, p, order="freq", bitmap=True) == want.size
    assert sm.count(text, p, order="freq", bitmap=False) == want.size
    assert sm.report(text, p).cpu().numpy().astype(np.uint64).tolist() == want.tolist()
    q = b"ACGTA"
    wq = oracle.count(q, t)
    assert sm.count(text, q, bitmap=True) == wq and sm.count(text, q, bitmap=False) == wq
    assert sm.count_batch([text], [(0, p), (0, q)]).cpu().tolist() == [want.size, oracle.count(q, t)]


def test_report_batch_over_512mib(dev):
    """A reporting batch whose texts total more than 512 MiB (streaming tile loads in the byte-tile
    kernel's reporting instance): every list and total against the oracle."""
    n = 600 << 20
    t = synth.zipf_text(n, 95, 1.0, family=15, stream=1)
    text = sm.Text(torch.from_numpy(t).to(dev))          # no histogram: byte-tile mode for every query
    g = np.random.default_rng(600)
    pats = [synth.substring_pattern(t, m, g)[0] for m in (3, 8, 8, 32, 200, 1000)]
    caps = [50_000, 100, 7, 1000, 10, 1]
    pos, totals = sm.report_batch([text.t], [(0, p) for p in pats], caps)
    pos = pos.cpu().numpy().astype(np.uint64)
    totals = totals.cpu().tolist()
    off = 0
    for i, (p, cap) in enumerate(zip(pats, caps)):
        total, want = oracle.report_full(p, t, cap)
        assert totals[i] == total, (i, len(p))
        assert pos[off:off + min(total, cap)].tolist() == want.tolist(), (i, len(p))
        off += cap


def test_serving_8_texts_of_1gib_against_oracle(dev):
    """The serving workload's shape (8 resident 1 GiB texts of 2-95 symbols, m log-uniform in
    [2, 512], half substrings, 5% reports): requests submitted in bursts while batches are in
    flight; a sample of the served counts and every served list of moderate length against the
    oracle."""
    from paper_1612_01506_amd.serve import GpuExecutor, Server
    n = 1 << 30
    mixes = [("uniform", 2), ("uniform", 4), ("zipf", 4), ("uniform", 20), ("zipf", 20), ("uniform", 95),
             ("zipf", 95), ("zipf", 95)]
    texts_h = [synth.zipf_text(n, s_, 1.0, family=5, stream=i) if kind == "zipf" else
               synth.uniform_text(n, s_, family=5, stream=i) for i, (kind, s_) in enumerate(mixes)]
    ex = GpuExecutor([torch.from_numpy(x).to(dev) for x in texts_h], nstreams=2)
    seen = {}

    def consume(r):
        if r.report and r.count <= 100_000:
            pos = r.positions.cpu().numpy() if isinstance(r.positions, torch.Tensor) else np.asarray(r.positions)
            seen[r.rid] = pos.astype(np.uint64)

    srv = Server(ex, hbm_budget=1 << 28, on_done=consume)
    g = synth.rng(5, 777)
    alphabets = [bytes(np.unique(x[:1 << 20])) for x in texts_h]
    reqs = []
    for k in range(600):
        ti = int(g.integers(0, 8))
        m = int(synth.loguniform_ints(2, 512, 1, g)[0])
        p = synth.substring_pattern(texts_h[ti], m, g)[0] if k % 2 else synth.random_pattern(alphabets[ti], m, g)
        reqs.append(srv.submit(ti, p, report=bool(g.random() < 0.05)))
        if k % 37 == 0:
            srv.step()
    srv.drain()
    assert all(r.status in ("done", "rejected") for r in reqs)
    done = [r for r in reqs if r.status == "done"]
    assert len(done) >= 590
    for r in done[::10]:
        assert r.count == oracle.count(r.pattern, texts_h[r.text_id]), (r.text_id, len(r.pattern))
    assert len(seen) >= 5
    for rid, pos in seen.items():
        r = reqs[rid]
        assert pos.tolist() == oracle.report(r.pattern, texts_h[r.text_id]).tolist(), (r.text_id, len(r.pattern))
    del ex
    torch.cuda.empty_cache()
