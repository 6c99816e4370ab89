"""GPU parity: every C-ABI entry point against the CPU oracle, element by element, bit exact.

Sizes span several 4/8/16 KiB tiles and 1024-start wave vectors with ragged
tails; text pointers are deliberately misaligned; patterns cover the peel
factors, the compare orders, LDS-staged and global (long) kernels.
"""
import itertools

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


def to_dev(a: np.ndarray, dev, offset: int = 0) -> torch.Tensor:
    """Device copy of a whose data pointer is `offset` bytes past a 256-byte boundary."""
    buf = torch.empty(a.size + offset + 64, dtype=torch.uint8, device=dev)
    v = buf[offset:offset + a.size]
    if a.size:
        v.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return v


def rand_text(n, sigma, seed):
    g = np.random.default_rng(seed)
    if sigma == 256:
        return g.integers(0, 256, size=n, dtype=np.uint8)
    alpha = np.frombuffer(synth.ALPHABETS[sigma], dtype=np.uint8)
    return alpha[g.integers(0, sigma, size=n)]


def pick_pattern(t, m, g, planted=True):
    if planted and t.size >= m:
        o = int(g.integers(0, t.size - m + 1))
        return bytes(t[o:o + m])
    return bytes(g.integers(0, 256, size=m, dtype=np.uint8))


# ------------------------------------------------------------------ worked example
def test_fig1_prefix(dev):
    t = to_dev(np.frombuffer(b"aabcd", dtype=np.uint8), dev)
    assert sm.count(t, b"abcd") == 1
    assert sm.count(t, b"abcd", order="freq") == 1
    assert sm.report(t, b"abcd").tolist() == [1]
    assert sm.report(t, b"a").tolist() == [0, 1]


# ------------------------------------------------------------------ tiny exhaustive
def test_exhaustive_binary_via_batch(dev):
    """All {a,b} texts with n <= 8 against all patterns with m <= 4, as one batch."""
    texts_h = [bytes(x) for n in range(1, 9) for x in itertools.product(b"ab", repeat=n)]
    pats = [bytes(x) for m in range(1, 5) for x in itertools.product(b"ab", repeat=m)]
    texts = [to_dev(np.frombuffer(t, dtype=np.uint8), dev, offset=i % 16) for i, t in enumerate(texts_h)]
    queries = [(i, p) for i in range(len(texts_h)) for p in pats]
    got = sm.count_batch(texts, queries).cpu().numpy()
    want = [sum(1 for s in range(len(texts_h[i]) - len(p) + 1) if texts_h[i][s:s + len(p)] == p)
            for i, p in queries]
    assert got.tolist() == want
    # a sample through the single-search path too
    for i in range(0, len(queries), 97):
        ti, p = queries[i]
        assert sm.count(texts[ti], p) == want[i]


# ------------------------------------------------------------ single search sweep
SIZES = [1, 15, 16, 17, 1000, 1023, 1024, 1025, 4095, 4096, 4097, 16383, 16384, 16385,
         3 * 16384 + 777, 200_003]
MS = [1, 2, 3, 4, 5, 7, 8, 16, 31, 64, 100, 257, 1000]


@pytest.mark.parametrize("sigma", [2, 4, 95, 256])
def test_count_sweep(dev, sigma):
    g = np.random.default_rng(1000 + sigma)
    for n in SIZES:
        t = rand_text(n, sigma, n * 7 + sigma)
        off = int(g.integers(0, 16))
        td = to_dev(t, dev, off)
        for m in MS:
            if m > n + 1:
                continue
            p = pick_pattern(t, m, g, planted=(m <= n and g.random() < 0.8))
            want = oracle.count(p, t)
            for order in ("ltr", "freq", "h"):
                got = sm.count(td, p, order=order, peel=int(g.integers(1, 9)))
                assert got == want, (sigma, n, off, m, order, got, want)


@pytest.mark.parametrize("tile_kib", [4, 8, 16])
@pytest.mark.parametrize("peel", [1, 2, 3, 5, 8])
def test_count_tiles_and_peels(dev, tile_kib, peel):
    g = np.random.default_rng(tile_kib * 10 + peel)
    t = rand_text(300_001, 4, 99)
    td = to_dev(t, dev, 5)
    for m in (1, 2, 6, 12, 33, 300, 5000):
        p = pick_pattern(t, m, g)
        want = oracle.count(p, t)
        perm = g.permutation(m).astype(np.int32)
        assert sm.count(td, p, order=perm, peel=peel, tile_kib=tile_kib) == want
        assert sm.count(td, p, order="freq", peel=peel, tile_kib=tile_kib, wgs_per_cu=1) == want


@pytest.mark.parametrize("offset", range(16))
def test_misaligned_text(dev, offset):
    t = rand_text(70_000 + offset * 13, 2, offset)
    td = to_dev(t, dev, offset)
    g = np.random.default_rng(offset)
    for m in (1, 4, 9, 17, 40):
        p = pick_pattern(t, m, g)
        assert sm.count(td, p) == oracle.count(p, t)
    # matches at the very first and very last start
    p0, pl = bytes(t[:11]), bytes(t[-11:])
    assert sm.report(td, p0)[:1].tolist() == [0]
    assert sm.report(td, pl)[-1:].tolist() == [t.size - 11]


def test_extreme_bytes(dev):
    g = np.random.default_rng(5)
    t = np.array([0x00, 0x7F, 0x80, 0xFF, 0x01, 0xFE], dtype=np.uint8)[g.integers(0, 6, size=50_000)]
    td = to_dev(t, dev, 3)
    for m in (1, 2, 3, 5, 8, 13):
        for _ in range(3):
            p = pick_pattern(t, m, g)
            assert sm.count(td, p, order="freq") == oracle.count(p, t)
            assert np.array_equal(sm.report(td, p).cpu().numpy().astype(np.uint64), oracle.report(p, t))


# --------------------------------------------------------------------- degenerate
def test_degenerate(dev):
    t = to_dev(np.frombuffer(b"abcabc", dtype=np.uint8), dev)
    assert sm.count(t, b"abcabca") == 0                       # m > n
    assert sm.count(t, b"abcabc") == 1                        # m == n
    assert sm.count(t[:0], b"a") == 0                         # n == 0
    assert sm.report(t, b"abcabca").numel() == 0
    with pytest.raises(sm.SmError):
        sm.count(t, b"")
    with pytest.raises(sm.SmError):
        sm.count(t, b"abc", order=[0, 0, 1])


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("n", [1, 1000, 65_536, 1_000_003])
def test_unary_closed_forms(dev, n):
    td = torch.full((n,), ord("a"), dtype=torch.uint8, device=dev)
    for k in (1, 2, 16, 256, 4096):
        want = max(0, n - k + 1)
        for order in ("ltr", "freq"):
            assert sm.count(td, b"a" * k, order=order) == want
            assert sm.count(td, b"a" * (k - 1) + b"b", order=order) == 0


@pytest.mark.parametrize("tile_kib", [4, 8, 16])
def test_unary_tile_and_vector_edges(dev, tile_kib):
    """On a^n every start of p = a^k matches, so a start masked wrongly at a tile or vector edge
    changes the count: the last valid start is placed just before, on and after vector and tile
    boundaries (coordinates from the 16-byte-aligned base), for misaligned text pointers."""
    T = tile_kib * 1024
    for offset in (0, 1, 15):
        first = offset % 16
        for last in (0, 1, 15, 1022, 1023, 1024, 1025, T - 2, T - 1, T, T + 1, 2 * T + 1023, 3 * T - 1):
            if last < first:
                continue
            for k in (1, 2, 3, 17):
                n = last - first + k
                td = to_dev(np.full(n, ord("a"), dtype=np.uint8), dev, offset)
                for peel in (1, 2, min(k, 8)):
                    assert sm.count(td, b"a" * k, tile_kib=tile_kib, peel=peel) == n - k + 1, (offset, last, k, peel)
                    assert sm.count(td, b"a" * (k - 1) + b"b", tile_kib=tile_kib, peel=peel) == 0
                if k == 2:
                    pos = sm.report(td, b"aa", tile_kib=tile_kib).cpu().numpy()
                    assert pos.tolist() == list(range(n - 1)), (offset, last)


@pytest.mark.parametrize("unit", [b"ab", b"abc", b"aab", b"GATTACA", b"abcabd"])
def test_periodic_closed_forms(dev, unit):
    n = 123_457
    L = len(unit)
    td = to_dev(synth.periodic_text(n, unit), dev, 7)
    for o in range(L):
        for m in (L, L + 1, 3 * L + 2, 40 * L):
            p = (unit * (m // L + 3))[o:o + m]
            want = (n - m - o) // L + 1 if n >= m + o else 0
            assert sm.count(td, p, order="freq") == want


# ------------------------------------------------------------------------ report
@pytest.mark.parametrize("sigma", [2, 4, 95])
def test_report_parity(dev, sigma):
    g = np.random.default_rng(sigma)
    for n in (17, 1025, 16385, 100_000, 1_048_583):
        t = rand_text(n, sigma, n + sigma)
        td = to_dev(t, dev, n % 16)
        for m in (1, 2, 5, 12, 64, 700):
            if m > n:
                continue
            p = pick_pattern(t, m, g)
            want = oracle.report(p, t)
            got = sm.report(td, p, order="freq").cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, want), (sigma, n, m)


def test_report_dense_and_cap(dev):
    n = 300_000
    td = torch.full((n,), ord("a"), dtype=torch.uint8, device=dev)
    pos, total = sm.report(td, b"aa", return_count=True)
    assert total == n - 1
    assert torch.equal(pos.cpu(), torch.arange(n - 1, dtype=torch.int64))
    head, total = sm.report(td, b"aaa", cap=1000, return_count=True)
    assert total == n - 2 and head.tolist() == list(range(1000))


def test_report_long_pattern(dev):
    n = 400_000
    t = rand_text(n, 2, 3)
    p = bytes(t[1000:1000 + 70_000])  # halo beyond LDS: global kernels
    td = to_dev(t, dev, 1)
    assert sm.count(td, p) == oracle.count(p, t)
    assert np.array_equal(sm.report(td, p).cpu().numpy().astype(np.uint64), oracle.report(p, t))
    u = torch.full((n,), 7, dtype=torch.uint8, device=dev)
    assert sm.count(u, bytes([7]) * 70_000) == n - 70_000 + 1


# --------------------------------------------------------------------- histogram
@pytest.mark.parametrize("n", [0, 1, 2, 15, 16, 17, 31, 33, 4096, 100_001, 5_000_000])
@pytest.mark.parametrize("offset", [0, 1, 7, 15])
def test_histogram(dev, n, offset):
    t = rand_text(n, 256, n)
    td = to_dev(t, dev, offset)
    h = sm.histogram(td).cpu().numpy()
    assert h.tolist() == np.bincount(t, minlength=256).tolist()


def test_histogram_skewed_and_large(dev):
    """One symbol only (every lane hits the same bin), a Zipf text, and a text spanning many workgroups."""
    for t in (np.full(3_000_017, 0xFF, dtype=np.uint8),
              synth.zipf_text(40_000_001, 95, 1.0, family=9, stream=77),
              rand_text(70_000_003, 4, 5)):
        td = to_dev(t, dev, 9)
        assert sm.histogram(td).cpu().numpy().tolist() == np.bincount(t, minlength=256).tolist()


# ------------------------------------------------------------------------ batch
def test_batch_mixed(dev):
    g = np.random.default_rng(77)
    texts_h = [rand_text(n, s, i) for i, (n, s) in enumerate(
        [(50_000, 4), (1_000_003, 95), (17, 2), (300_000, 256), (70_001, 20)])]
    texts = [sm.Text(to_dev(t, dev, i * 3 % 16)) for i, t in enumerate(texts_h)]
    queries, want = [], []
    for k in range(600):
        ti = int(g.integers(0, len(texts_h)))
        t = texts_h[ti]
        m = int(synth.loguniform_ints(1, 2048, 1, g)[0])
        p = pick_pattern(t, m, g, planted=g.random() < 0.7)
        order = [None, "ltr", "freq", "h"][k % 4]
        queries.append((ti, p, order))
        want.append(oracle.count(p, t))
    # a few long ones (global kernel) and empty-result ones
    queries.append((1, bytes(texts_h[1][10:10 + 60_000]), None))
    want.append(oracle.count(queries[-1][1], texts_h[1]))
    queries.append((2, b"x" * 100, None))
    want.append(0)
    got = sm.count_batch(texts, queries).cpu().numpy().tolist()
    assert got == want
    got2 = sm.count_batch(texts, queries, tile_kib=4, peel=3).cpu().numpy().tolist()
    assert got2 == want
    single = [sm.count(texts[q[0]], q[1]) for q in queries[:50]]
    assert single == want[:50]


def test_batch_validation(dev):
    td = to_dev(np.frombuffer(b"abc", dtype=np.uint8), dev)
    with pytest.raises(sm.SmError, match="query 1"):
        sm.count_batch([td], [(0, b"a"), (1, b"b")])
    with pytest.raises(sm.SmError, match="query 0"):
        sm.count_batch([td], [(0, b"")])


def test_count_async_accumulates(dev):
    t = rand_text(500_000, 4, 1)
    td = to_dev(t, dev)
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    pats = [bytes(t[i * 1000:i * 1000 + 8]) for i in range(10)]
    for p in pats:
        sm.count_async(td, p, out, order="freq")
    torch.cuda.synchronize()
    assert int(out.item()) == sum(oracle.count(p, t) for p in pats)


def test_deterministic(dev):
    t = rand_text(2_000_000, 2, 11)
    td = to_dev(t, dev)
    p = bytes(t[5:25])
    a = sm.report(td, p, order="freq").cpu()
    b = sm.report(td, p, order="freq").cpu()
    assert torch.equal(a, b)
    assert bool((a[1:] > a[:-1]).all())


# ------------------------------------------------------------- prepared patterns
def test_prepared_patterns(dev):
    g = np.random.default_rng(31)
    t = rand_text(1_500_007, 95, 4)
    td = to_dev(t, dev, 9)
    h = oracle.hist(t)
    pats = [pick_pattern(t, int(m), g, planted=g.random() < 0.8)
            for m in synth.loguniform_ints(1, 3000, 120, g)] + [bytes(t[5:5 + 70_000])]
    orders = [oracle.order_freq(p, h) if i % 2 else None for i, p in enumerate(pats)]
    ps = sm.Patterns(pats, orders)
    out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
    for i in range(len(pats)):
        ps.count_async(i, td, out[i:i + 1], peel=1 + i % 8)
    torch.cuda.synchronize()
    want = [oracle.count(p, t) for p in pats]
    assert out.cpu().tolist() == want
    buf = torch.empty(4096, dtype=torch.int64, device=dev)
    for i in range(0, len(pats), 7):
        tot = ps.report(i, td, buf)
        assert tot == want[i]
        if tot <= buf.numel():
            assert np.array_equal(buf[:tot].cpu().numpy().astype(np.uint64), oracle.report(pats[i], t))
    ps.close()
    with pytest.raises(sm.SmError):
        sm.Patterns([b"ab", b""])


def test_pattern_set_larger_than_half_the_upload_ring(dev):
    """Step tables over 32 MiB (half the 64 MiB pinned ring) go up through a dedicated staging buffer;
    a small set created right after reuses the ring.  Counts against the oracle."""
    g = np.random.default_rng(77)
    t = rand_text(3_000_000, 20, 21)
    td = to_dev(t, dev, 3)
    # 5 patterns of 1 MB: 5 x (1 MB + 8) step entries x 8 B = 40 MB of tables
    big = [bytes(t[o:o + 1_000_000]) for o in g.integers(0, t.size - 1_000_000, size=4)] + \
          [bytes(rand_text(1_000_000, 20, 22))]
    ps = sm.Patterns(big)
    small = sm.Patterns([bytes(t[10:20]), b"zz"])
    out = torch.zeros(len(big) + 2, dtype=torch.int64, device=dev)
    for i in range(len(big)):
        ps.count_async(i, td, out[i:i + 1])
    for i in range(2):
        small.count_async(i, td, out[len(big) + i:len(big) + i + 1])
    torch.cuda.synchronize()
    want = [oracle.count(p, t) for p in big] + [oracle.count(bytes(t[10:20]), t), oracle.count(b"zz", t)]
    assert out.cpu().tolist() == want
    assert min(want[:4]) >= 1
    ps.close()
    small.close()


def test_report_async_two_streams(dev):
    """Async reports on two streams share the library's report scratch; results must be exact."""
    g = np.random.default_rng(8)
    t = rand_text(3_000_017, 4, 12)
    td = to_dev(t, dev, 6)
    pats = [pick_pattern(t, int(m), g) for m in (6, 7, 8, 9, 10, 11, 12, 14, 16, 20, 64, 200)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cap = 8192
    outs = torch.full((len(pats), cap), -1, dtype=torch.int64, device=dev)
    tots = torch.zeros(len(pats), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    for i, p in enumerate(pats):
        sm.report_async(td, p, outs[i], tots[i:i + 1], order="freq" if i % 2 else None,
                        stream=s1 if i % 2 else s2)
    torch.cuda.synchronize()
    for i, p in enumerate(pats):
        want = oracle.report(p, t)
        assert int(tots[i]) == want.size
        k = min(want.size, cap)
        assert np.array_equal(outs[i, :k].cpu().numpy().astype(np.uint64), want[:k])
    # prepared patterns, async, plus the m > n case (total 0)
    ps = sm.Patterns(pats + [b"A" * (t.size + 1)])
    tot = torch.full((len(pats) + 1,), -1, dtype=torch.int64, device=dev)
    for i in range(len(pats) + 1):
        ps.report_async(i, td, outs[i % len(pats)], tot[i:i + 1])
    torch.cuda.synchronize()
    assert tot.cpu().tolist() == [oracle.count(p, t) for p in pats] + [0]


def test_patterns_create_ordered(dev):
    g = np.random.default_rng(21)
    t = rand_text(400_009, 95, 7)
    td = to_dev(t, dev, 2)
    h = oracle.hist(t)
    pats = [pick_pattern(t, int(m), g) for m in synth.loguniform_ints(1, 600, 40, g)]
    want = [oracle.count(p, t) for p in pats]
    for kind in ("ltr", "freq", "h", "hs"):
        ps = sm.Patterns(pats, kind, h if kind == "freq" else None)
        out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
        for i in range(len(pats)):
            ps.count_async(i, td, out[i:i + 1])
        torch.cuda.synchronize()
        assert out.cpu().tolist() == want, kind
    with pytest.raises(sm.SmError):
        sm.Patterns(pats, "freq")  # needs a histogram


@pytest.mark.parametrize("sigma", [2, 4, 20, 95])
def test_batch_bitmap_mode(dev, sigma):
    """Texts with histograms and >= 32 queries each run in the bitmap mode."""
    g = np.random.default_rng(300 + sigma)
    sizes = [5_000, 8_192, 8_193, 70_001, 1_234_567]
    texts_h = [rand_text(n, sigma, 50 + i) if sigma != 95 else
               synth.zipf_text(n, 95, 1.0, family=9, stream=i) for i, n in enumerate(sizes)]
    texts = [sm.Text(to_dev(t, dev, (7 * i) % 16)) for i, t in enumerate(texts_h)]
    queries, want = [], []
    for ti, t in enumerate(texts_h):
        for k in range(150):
            m = int(synth.loguniform_ints(1, 4096, 1, g)[0])
            if k % 3 == 0:
                p = bytes(g.integers(0, 256, size=min(m, 16), dtype=np.uint8))   # mostly absent symbols
            elif k % 3 == 1:
                p = pick_pattern(t, min(m, t.size), g)
            else:
                alpha = np.unique(t)
                p = bytes(alpha[g.integers(0, alpha.size, size=m)])
            queries.append((ti, p))
            want.append(oracle.count(p, t))
    queries.append((0, bytes(texts_h[0]) + b"x"))     # m > n
    want.append(0)
    got = sm.count_batch(texts, queries).cpu().numpy().tolist()
    assert got == want
    got = sm.count_batch(texts, queries, peel=4).cpu().numpy().tolist()
    assert got == want


def test_batch_bitmap_unary_closed_form(dev):
    n = 100_003
    td = sm.Text(torch.full((n,), ord("a"), dtype=torch.uint8, device=dev))
    ks = list(range(1, 60)) + [100, 1000, 4096]
    queries = [(0, b"a" * k) for k in ks] + [(0, b"a" * (k - 1) + b"b") for k in ks]
    got = sm.count_batch([td], queries).cpu().tolist()
    assert got == [n - k + 1 for k in ks] + [0] * len(ks)


def test_packed_texts_batch(dev):
    g = np.random.default_rng(44)
    lens = [int(x) for x in synth.loguniform_ints(1, 300_000, 200, g)]
    texts_h = [rand_text(n, (4, 20, 95)[i % 3], 900 + i) for i, n in enumerate(lens)]
    offs, pos = [], 0
    for i, th in enumerate(texts_h):
        pos += i % 16
        offs.append(pos)
        pos += th.size
    buf = torch.zeros(pos, dtype=torch.uint8, device=dev)
    for o, th in zip(offs, texts_h):
        buf[o:o + th.size].copy_(torch.from_numpy(th))
    hists = np.stack([oracle.hist(th) for th in texts_h])
    queries, want = [], []
    for i, th in enumerate(texts_h):
        for k in range(2):
            p = pick_pattern(th, int(synth.loguniform_ints(1, 64, 1, g)[0]), g)
            queries.append((i, p))
            want.append(oracle.count(p, th))
    for h in (None, hists):
        got = sm.count_batch(sm.PackedTexts(buf, offs, lens, h), queries).cpu().tolist()
        assert got == want


def test_text_past_allocation_rejected(dev):
    td = torch.zeros(1 << 20, dtype=torch.uint8, device=dev)
    lib = sm._lib.load()
    p = np.frombuffer(b"ab", dtype=np.uint8)
    rc = lib.sm_count(p.ctypes.data, 2, td.data_ptr(), 1 << 40, None)
    assert rc == sm._lib.SM_EINVAL
    assert "past the end" in lib.sm_last_error().decode()


def test_serving_alone_equals_mix(dev):
    from paper_1612_01506_amd.serve import GpuExecutor, Server
    texts_h = [synth.zipf_text(3_000_000, 95, 1.0, family=5, stream=1),
               rand_text(2_000_003, 4, 77), synth.zipf_text(1_500_000, 20, 1.0, family=5, stream=2)]
    ex = GpuExecutor([to_dev(t, dev, 3 * i) for i, t in enumerate(texts_h)], nstreams=2)
    srv = Server(ex, max_batch=96, hbm_budget=1 << 24)
    g = np.random.default_rng(12)
    reqs = []
    for k in range(400):
        ti = int(g.integers(0, 3))
        m = int(synth.loguniform_ints(2, 512, 1, g)[0])
        p = (synth.substring_pattern(texts_h[ti], m, g)[0] if k % 2 else
             synth.random_pattern(bytes(np.unique(texts_h[ti])), m, g))
        reqs.append(srv.submit(ti, p, report=(k % 20 == 0)))
        if g.random() < 0.3:
            srv.step()
    srv.drain()
    assert srv.batches > 2
    for k, r in enumerate(reqs):
        assert r.status == "done", (r.status, r.error)
        alone = sm.count(ex.texts[r.text_id], r.pattern)
        assert r.count == alone
        if k % 10 == 0 or r.report:
            assert r.count == oracle.count(r.pattern, texts_h[r.text_id])
        if r.report:
            pos = r.positions.cpu().numpy() if hasattr(r.positions, "cpu") else r.positions
            assert np.array_equal(pos.astype(np.uint64), oracle.report(r.pattern, texts_h[r.text_id]))


def test_serving_lone_requests(dev):
    """Requests served one at a time take the single-search count and report paths."""
    from paper_1612_01506_amd.serve import GpuExecutor, Server
    texts_h = [synth.zipf_text(2_000_000, 95, 1.0, family=5, stream=3), rand_text(1_000_001, 4, 78)]
    ex = GpuExecutor([to_dev(t, dev, 5 + i) for i, t in enumerate(texts_h)], nstreams=2)
    srv = Server(ex, hbm_budget=1 << 24)
    g = np.random.default_rng(13)
    for k in range(12):
        ti = k % 2
        p = synth.substring_pattern(texts_h[ti], int(g.integers(2, 40)), g)[0]
        r = srv.submit(ti, p, report=(k % 3 == 0))
        srv.drain()
        assert r.status == "done", (r.status, r.error)
        assert r.count == oracle.count(p, texts_h[ti])
        if r.report:
            pos = r.positions.cpu().numpy() if hasattr(r.positions, "cpu") else r.positions
            assert np.array_equal(pos.astype(np.uint64), oracle.report(p, texts_h[ti]))
    assert srv.batches >= 12


def test_batch_plan_graph_replay(dev):
    """A planned batch equals the one-shot batch and the oracle, eagerly and replayed from a graph.

    Between replays the program runs its own eager searches and rewrites the
    texts (same lengths, same alphabets); every replay is checked against the
    oracle on the texts as they are then.
    """
    g = np.random.default_rng(4242)
    spec = [(60_000, 4, True), (700_001, 95, True), (33, 2, False), (250_000, 256, False), (90_001, 20, True)]
    texts_h = [rand_text(n, s, 10 + i) for i, (n, s, _) in enumerate(spec)]
    bufs = [to_dev(t, dev, (5 * i) % 16) for i, t in enumerate(texts_h)]
    texts = [sm.Text(b) if hist else b for b, (_, _, hist) in zip(bufs, spec)]
    queries = []
    for k in range(500):
        ti = int(g.integers(0, len(spec)))
        m = int(synth.loguniform_ints(1, 3000, 1, g)[0])
        queries.append((ti, pick_pattern(texts_h[ti], m, g, planted=g.random() < 0.7)))
    queries.append((3, bytes(texts_h[3][100:100 + 40_000])))   # long: global kernel
    queries.append((2, b"0" * 40))                              # m > n
    want = [oracle.count(p, texts_h[ti]) for ti, p in queries]

    plan = sm.BatchPlan(texts, queries)
    out = torch.full((len(queries) + 3,), -7, dtype=torch.int64, device=dev)
    assert plan.run(out).cpu().tolist() == want
    assert out[len(queries):].cpu().tolist() == [-7] * 3      # only nq entries written
    assert sm.count_batch(texts, queries).cpu().tolist() == want

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(out)                                           # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(out)
    for rep in range(4):
        if rep >= 2:                                            # new contents, same lengths and alphabets
            for i, (n, sg, _) in enumerate(spec):
                texts_h[i] = rand_text(n, sg, 1000 * rep + i)
                bufs[i].copy_(torch.from_numpy(texts_h[i]))
            want = [oracle.count(p, texts_h[ti]) for ti, p in queries]
        out.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert out[:len(queries)].cpu().tolist() == want, f"replay {rep}"
        # the program's own eager work between replays
        ti, p = queries[rep]
        assert sm.count(bufs[ti], p) == want[rep]
        assert sm.count_batch(texts, queries[:40]).cpu().tolist() == want[:40]
    plan.close()
    plan.close()
    with pytest.raises(ValueError):
        plan.run(out)


def test_batch_plan_empty_and_errors(dev):
    td = to_dev(np.frombuffer(b"abcabc", dtype=np.uint8), dev)
    plan = sm.BatchPlan([td], [])
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    assert plan.run(out).numel() == 0
    plan.close()
    with pytest.raises(sm.SmError, match="query 1"):
        sm.BatchPlan([td], [(0, b"a"), (2, b"b")])
    with sm.BatchPlan([td], [(0, b"abc"), (0, b"c"), (0, b"abcabcx")]) as plan:
        assert plan.run().cpu().tolist() == [2, 2, 0]
        with pytest.raises(ValueError):
            plan.run(torch.zeros(2, dtype=torch.int64, device=dev))


# ------------------------------------------------------------ non-overlapping mode
@pytest.mark.parametrize("sigma", [1, 2, 4, 256])
def test_nonoverlap_parity(dev, sigma):
    """Disjoint occurrences (greedy leftmost) against the oracle: counts, positions, cap, misalignment."""
    g = np.random.default_rng(700 + sigma)
    for n in (1, 17, 1023, 1024, 4097, 65_537, 1_000_003):
        t = (np.full(n, ord("a"), dtype=np.uint8) if sigma == 1 else rand_text(n, min(sigma, 256), n + sigma))
        td = to_dev(t, dev, n % 16)
        for m in (1, 2, 3, 5, 8, 31, 100):
            if sigma == 1:
                p = b"a" * m
            else:
                p = pick_pattern(t, m, g, planted=g.random() < 0.8)
            want = oracle.report_nonoverlap(p, t)
            want_n = int(want.size)
            assert sm.count(td, p, overlap=False) == want_n, (n, m)
            pos, total = sm.report(td, p, overlap=False, return_count=True)
            assert total == want_n
            assert pos.cpu().numpy().astype(np.uint64).tolist() == want.tolist(), (n, m)
            if want_n > 3:
                pos, total = sm.report(td, p, overlap=False, cap=3, return_count=True)
                assert total == want_n and pos.cpu().tolist() == want[:3].tolist()
            # the overlapping count is unchanged by the mode of earlier calls
            assert sm.count(td, p) == oracle.count(p, t)


def test_nonoverlap_closed_forms_large(dev):
    """a^n with p = a^k takes floor(n/k) starts 0, k, 2k, ...; (ab)^q with (ab)^j: floor(q/j)."""
    n = 48_000_011
    td = torch.full((n,), ord("a"), dtype=torch.uint8, device=dev)
    for k in (1, 2, 3, 16, 255):
        assert sm.count(td, b"a" * k, overlap=False) == n // k
    pos, total = sm.report(td, b"a" * 7, overlap=False, cap=1000, return_count=True)
    assert total == n // 7 and pos.cpu().tolist() == list(range(0, 7000, 7))
    q = 3_000_001
    t2 = to_dev(np.frombuffer(b"ab" * q, dtype=np.uint8), dev, 5)
    for j in (1, 2, 5):
        assert sm.count(t2, b"ab" * j, overlap=False) == q // j
    assert sm.count(t2, b"ba", overlap=False) == q - 1


def test_nonoverlap_patterns_and_rejections(dev):
    t = rand_text(300_000, 2, 9)
    td = to_dev(t, dev, 3)
    pats = [b"0", b"01", b"0101", b"11011", bytes(t[1000:1040])]
    ps = sm.Patterns(pats)
    out = torch.empty(200_000, dtype=torch.int64, device=dev)
    for i, p in enumerate(pats):
        want_n, want = oracle.report_nonoverlap_full(p, t, out.numel())
        got = ps.report(i, td, out, overlap=False)
        assert got == want_n
        assert out[:min(got, out.numel())].cpu().numpy().astype(np.uint64).tolist() == want.tolist()
    ps.close()
    c = torch.zeros(1, dtype=torch.int64, device=dev)
    lib = sm._lib.load()
    no = sm._lib.sm_params(0, 0, 0, sm._lib.SM_NONOVERLAP)
    import ctypes
    p = np.frombuffer(b"01", dtype=np.uint8)
    rc = lib.sm_count_async(p.ctypes.data, 2, td.data_ptr(), td.numel(), None, ctypes.byref(no), c.data_ptr(), None)
    assert rc == sm._lib.SM_EINVAL and "synchronous" in lib.sm_last_error().decode()
    torch.cuda.synchronize()
    assert int(c.item()) == 0


# ------------------------------------------------------------- bigram statistics
@pytest.mark.parametrize("n", [0, 1, 2, 3, 15, 16, 17, 31, 33, 4096, 100_003, 3_000_001])
@pytest.mark.parametrize("offset", [0, 5, 15])
def test_bigram_counts(dev, n, offset):
    t = rand_text(n, 256, 31 * n + offset)
    td = to_dev(t, dev, offset)
    assert sm.bigram(td).cpu().numpy().astype(np.uint64).tolist() == oracle.bigram(t).tolist()


def test_bigram_counts_skewed_and_one_half(dev):
    """Zipf text over printable bytes (one pass skipped through the histogram), high bytes only,
    a single repeated byte, and a text spanning many workgroups."""
    for t in (synth.zipf_text(20_000_003, 95, 1.0, family=9, stream=5),
              (rand_text(1_000_001, 256, 4) | np.uint8(0x80)),
              np.full(2_000_001, 0xC3, dtype=np.uint8),
              rand_text(50_000_017, 4, 8)):
        td = sm.Text(to_dev(t, dev, 7))
        want = oracle.bigram(t)
        assert td.bigram.tolist() == want.tolist()
        assert sm.bigram(td.t).cpu().numpy().astype(np.uint64).tolist() == want.tolist()


def test_bigram_order_searches(dev):
    """Counts and reports with the bigram order equal the oracle's (the order changes only speed)."""
    g = np.random.default_rng(91)
    t = synth.zipf_text(3_000_000, 95, 1.0, family=9, stream=6)
    text = sm.Text(to_dev(t, dev, 3))
    for m in (1, 2, 3, 5, 8, 16, 64, 300):
        for _ in range(3):
            p = pick_pattern(t, m, g)
            o = sm.order("bigram", p, text.hist, text.bigram)
            assert o.tolist() == oracle.order_bigram(p, oracle.hist(t), oracle.bigram(t)).tolist()
            want = oracle.count(p, t)
            assert sm.count(text, p, order="bigram") == want
            assert sm.report(text, p, order="bigram").cpu().numpy().astype(np.uint64).tolist() == \
                oracle.report(p, t).tolist()


# ------------------------------------------------------------- randomized sweep
def test_random_sweep_all_entry_points(dev):
    """Seeded random cases across alphabets, lengths, alignments, orders, peels and tile sizes, through
    the synchronous, asynchronous, prepared-pattern and batched entry points, all against the oracle."""
    g = np.random.default_rng(2024)
    texts, hosts = [], []
    for k in range(6):
        n = int(synth.loguniform_ints(1, 3_000_000, 1, g)[0])
        sigma = int(g.choice([1, 2, 3, 4, 20, 95, 256]))
        t = (np.full(n, 0x41, dtype=np.uint8) if sigma == 1 else rand_text(n, sigma, 5000 + k))
        hosts.append(t)
        texts.append(sm.Text(to_dev(t, dev, int(g.integers(0, 16)))))
    queries, want = [], []
    for k in range(240):
        ti = int(g.integers(0, len(hosts)))
        t = hosts[ti]
        m = int(synth.loguniform_ints(1, 5000, 1, g)[0])
        p = pick_pattern(t, m, g, planted=g.random() < 0.75) if t.size else bytes([65] * m)
        order = [None, "ltr", "freq", "h", "hs", "bigram"][k % 6]
        peel = int(g.choice([1, 2, 3, 5, 8]))
        tile = int(g.choice([4, 8, 16]))
        c = oracle.count(p, t)
        if k % 4 == 0:
            assert sm.count(texts[ti], p, order=order, peel=peel, tile_kib=tile) == c, (k, ti, m)
        elif k % 4 == 1:
            out = torch.zeros(1, dtype=torch.int64, device=dev)
            sm.count_async(texts[ti], p, out, order=order, peel=peel, tile_kib=tile)
            assert int(out.item()) == c, (k, ti, m)
        elif k % 4 == 2:
            cap = int(g.integers(0, 50))
            pos, total = sm.report(texts[ti], p, order=order, cap=cap, peel=peel, return_count=True)
            assert total == c and pos.cpu().numpy().astype(np.uint64).tolist() == oracle.report(p, t, cap).tolist()
        else:
            assert sm.count(texts[ti], p, overlap=False) == oracle.count_nonoverlap(p, t), (k, ti, m)
        queries.append((ti, p))
        want.append(c)
    assert sm.count_batch(texts, queries).cpu().tolist() == want
    with sm.BatchPlan(texts, queries, peel=3, tile_kib=4) as plan:
        assert plan.run().cpu().tolist() == want


# ------------------------------------------------------------- batched reports
def test_report_batch_parity(dev):
    """Ordered positions of many queries from one reporting batch: every list, total and cap against
    the oracle; texts with histograms and many queries stay in byte-tile mode; long patterns use the
    global kernel."""
    g = np.random.default_rng(4321)
    sizes = [(200_003, 2), (1_500_000, 95), (70_001, 4), (33, 20), (400_000, 256)]
    hosts = [rand_text(n, s, 77 + i) for i, (n, s) in enumerate(sizes)]
    texts = [sm.Text(to_dev(t, dev, (3 * i) % 16)) for i, t in enumerate(hosts)]
    queries, caps = [], []
    for k in range(300):
        ti = int(g.integers(0, len(hosts)))
        t = hosts[ti]
        m = int(synth.loguniform_ints(1, 3000, 1, g)[0])
        p = pick_pattern(t, m, g, planted=g.random() < 0.8)
        queries.append((ti, p, [None, "freq", "h"][k % 3]))
        caps.append(int(g.choice([0, 1, 5, 1000, 100_000])))
    queries.append((1, bytes(hosts[1][500:500 + 40_000]), None))   # long: global kernel
    caps.append(3)
    queries.append((3, b"x" * 100, None))                             # m > n
    caps.append(10)
    pos, totals = sm.report_batch(texts, queries, caps)
    pos = pos.cpu().numpy().astype(np.uint64)
    totals = totals.cpu().tolist()
    off = 0
    for i, ((ti, p, _), cap) in enumerate(zip(queries, caps)):
        total, want = oracle.report_full(p, hosts[ti], cap)
        assert totals[i] == total, i
        assert pos[off:off + min(total, cap)].tolist() == want.tolist(), i
        off += cap
    assert totals == sm.count_batch(texts, [(ti, p) for ti, p, _ in queries]).cpu().tolist()
    # a second batch reuses the shared scratch (it must start from zero again)
    pos2, totals2 = sm.report_batch(texts, queries[:50], caps[:50], peel=3)
    assert totals2.cpu().tolist() == totals[:50]
    pos2 = pos2.cpu().numpy().astype(np.uint64)
    off = 0
    for i in range(50):                       # only the written part of each segment is defined
        k = min(totals[i], caps[i])
        assert pos2[off:off + k].tolist() == pos[off:off + k].tolist(), i
        off += caps[i]
