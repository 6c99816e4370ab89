"""Parity at the benchmark workloads' full sizes, in the launch configurations bench.py times.

Outputs the oracle can compute one by one are sampled (a pattern per length, a few
batch queries); the rest are checked through properties that hold at any size
(batched == single searches, count == report length, closed forms, order and
peel invariance).
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
    for i in range(0, len(patterns), 100):          # one pattern per length against the oracle
        assert counts[i] == oracle.count(patterns[i], t), len(patterns[i])
    # the default launch (no tuning table: 8 KiB tiles, 6 workgroups per CU) gives the same counts
    plain = torch.zeros(len(patterns), dtype=torch.int64, device=dev)
    for i in range(len(patterns)):
        ps.count_async(i, td, plain[i:i + 1])
    torch.cuda.synchronize()
    assert plain.cpu().numpy().tolist() == counts.tolist()
    for k in range(0, len(rep), 100):                # one reported list per length against the oracle
        want = oracle.report(patterns[rep[k]], t)
        got = pos[k, :min(int(tot[k]), cap)].cpu().numpy().astype(np.uint64)
        assert got.tolist() == want[:cap].tolist(), len(patterns[rep[k]])
    ps.close()


def test_batched_one_text_2gib(dev):
    """10,000 patterns on a 2 GiB Zipf text in one launch (bitmap mode)."""
    t, pats = synth.batched_one_text_workload()
    text = sm.Text(torch.from_numpy(t).to(dev))
    got = sm.count_batch([text], [(0, p) for p in pats]).cpu().numpy()
    g = np.random.default_rng(5)
    for i in g.choice(len(pats), size=200, replace=False):   # batched == single searches
        assert got[i] == sm.count(text, pats[i]), i
    for i in g.choice(len(pats), size=4, replace=False):     # and the oracle on a few
        assert got[i] == oracle.count(pats[i], t), i


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
    t, pats = synth.small_alphabet_workload(n=1 << 30, sigma=sigma)
    text = sm.Text(torch.from_numpy(t).to(dev))
    seen = set()
    for p in pats:
        a = sm.count(text, p, order="freq", peel=5)
        assert a == sm.count(text, p, order="freq", peel=2)
        if len(p) not in seen:
            seen.add(len(p))
            assert a == oracle.count(p, t), (sigma, len(p))


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
    assert sm.count(text, p, order="freq") == want.size
    assert sm.report(text, p).cpu().numpy().astype(np.uint64).tolist() == want.tolist()
    q = b"ACGTA"
    assert sm.count(text, q) == oracle.count(q, t)
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
