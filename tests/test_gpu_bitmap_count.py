"""Bitmap-mode counts (SM_BITMAP) against the oracle.

The bitmap kernel turns Section 2.1's SIMDcompare of each distinct pattern
symbol into one bit per text byte per tile, and each compare into a shift and
AND of those bits, with Algorithm 4's peel and zero tests.  These cases cover
every distinct-symbol count it takes (1 to 4) and the fallback past 4, the
three tile sizes and the automatic tile growth for long patterns, texts from
empty to several tiles with ragged tails and every start alignment, the first
and last start of a text, compare chains past 64 (periodic text), lone
candidates verified across lanes, and the prepared-pattern and asynchronous
entry points.
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


def over(alpha: bytes, n: int, seed: int) -> np.ndarray:
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[np.random.default_rng(seed).integers(0, a.size, size=n)]


def distinct(p: bytes) -> int:
    return len(set(p))


def patterns_for(t: np.ndarray, g, lengths) -> list[bytes]:
    """Substrings (whose distinct symbols follow the text) and random patterns of 1..5 symbols."""
    out = []
    syms = np.unique(t) if t.size else np.frombuffer(b"ab", dtype=np.uint8)
    for m in lengths:
        if m <= t.size:
            o = int(g.integers(0, t.size - m + 1))
            out.append(bytes(t[o:o + m]))
        for k in (1, 2, 3, 4, 5):
            pick = syms[g.integers(0, syms.size, size=k)]
            out.append(bytes(pick[g.integers(0, pick.size, size=m)]))
    return out


def test_ragged_texts_every_alignment(dev):
    """Texts of 0 to about four 32 KiB tiles at start offsets 0..15, small and large alphabets."""
    g = np.random.default_rng(9100)
    base = torch.zeros(300_064, dtype=torch.uint8, device=dev)
    cases = 0
    for sigma_alpha, seed in ((b"ab", 1), (b"abc", 2), (b"ACGT", 3), (bytes(range(65, 65 + 20)), 4)):
        for n in (0, 1, 5, 31, 32, 33, 100, 8_159, 8_192, 8_193, 16_400, 65_537, 131_101, 299_999):
            off = int(g.integers(0, 16))
            t = over(sigma_alpha, n, seed + n)
            base[off:off + n].copy_(torch.from_numpy(t))
            view = base[off:off + n]
            pats = patterns_for(t, g, (1, 2, 3, 7, 31, 32, 33, 64, 100) if n < 10_000 else (2, 8, 33, 257, 1000))
            for p in pats:
                want = oracle.count(p, t)
                for tile in (8, 16, 32):
                    got = sm.count(view, p, bitmap=True, tile_kib=tile, peel=int(g.integers(1, 9)))
                    assert got == want, (sigma_alpha, n, off, len(p), distinct(p), tile, got, want)
                    cases += 1
    assert cases > 1000


def test_zipf_and_binary_multi_tile(dev):
    """Half-MiB texts (dozens of tiles per workgroup round) with lengths up to 4096: long patterns
    grow the tile (halo of up to 129 words) or fall back to byte compares."""
    g = np.random.default_rng(9101)
    texts = [synth.uniform_text(524_288 + 13, 2, family=3, stream=1),
             synth.uniform_text(524_288 + 77, 4, family=3, stream=2),
             synth.zipf_text(524_288 + 5, 95, 1.0, family=3, stream=3)]
    for t in texts:
        td = torch.from_numpy(t).to(dev)
        for p in patterns_for(t, g, (2, 5, 16, 63, 128, 512, 1024, 2049, 4096)):
            want = oracle.count(p, t)
            for tile in (8, 32):
                assert sm.count(td, p, bitmap=True, tile_kib=tile) == want, (len(p), distinct(p), tile)
            assert sm.count(td, p, bitmap=False) == want


def test_first_and_last_starts(dev):
    """Matches exactly at the text's first and last start, in texts ending at every residue of 32."""
    g = np.random.default_rng(9102)
    for n in range(40_000, 40_064):
        t = over(b"ab", n, n)
        p = bytes(t[:9])
        t[n - 9:] = t[:9]
        td = torch.from_numpy(t).to(dev)
        want = oracle.count(p, t)
        assert want >= 2
        assert sm.count(td, p, bitmap=True, tile_kib=8, peel=int(g.integers(1, 4))) == want, n


def test_periodic_text_long_compare_chains(dev):
    """a^n with a^k and a^(k-1)b: every start survives k compares (chains past 64 entries)."""
    n = 3_000_017
    td = torch.full((n,), ord("a"), dtype=torch.uint8, device=dev)
    for k in (1, 63, 64, 65, 200, 1000):
        for peel in (1, 2, 8):
            assert sm.count(td, b"a" * k, bitmap=True, peel=peel) == n - k + 1, (k, peel)
            assert sm.count(td, b"a" * (k - 1) + b"b", bitmap=True, peel=peel, order="ltr") == 0, (k, peel)


def test_prepared_and_async_paths(dev):
    """sm_patterns_count and sm_count_async take the bitmap kernel too (frequency order from the
    text's histogram); a pattern of five or more symbols takes the byte compares."""
    g = np.random.default_rng(9103)
    t = synth.uniform_text(1_000_003, 4, family=3, stream=7)
    text = sm.Text(torch.from_numpy(t).to(dev))
    pats = patterns_for(t, g, (3, 12, 40, 300))
    pats.append(bytes(range(65, 70)) * 3)
    want = [oracle.count(p, t) for p in pats]
    ps = sm.Patterns(pats, "freq", text.hist)
    out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
    for i in range(len(pats)):
        ps.count_async(i, text, out[i:i + 1], bitmap=True, tile_kib=16)
    assert out.cpu().tolist() == want
    out.zero_()
    for i, p in enumerate(pats):
        sm.count_async(text, p, out[i:i + 1], order="freq", bitmap=True)
    assert out.cpu().tolist() == want
    ps.close()


def test_bitmap_flag_ignored_by_reports(dev):
    """Reports (and the non-overlapping mode) run the byte path whatever the flag says."""
    t = over(b"ab", 100_001, 77)
    td = torch.from_numpy(t).to(dev)
    for p in (b"ab", b"abba", b"a" * 9):
        pos = sm.report(td, p)
        assert pos.cpu().numpy().astype(np.uint64).tolist() == oracle.report(p, t).tolist()
        assert sm.count(td, p, bitmap=True, overlap=False) == sm.count(td, p, overlap=False)


def test_lone_candidates_verified_across_lanes(dev):
    """Long patterns planted a few times close together (several candidates in one wave) and
    near misses differing in one byte at varying depths: the starts left after the grouped
    compares are verified one at a time, and a single mismatch anywhere ends a start."""
    g = np.random.default_rng(9104)
    for m in (80, 700, 3000):
        for tile in (8, 32):
            t = over(b"ab", 400_000, m + tile)
            p = bytes(over(b"ab", m, m * 7 + 1))
            # copies side by side (two or three in one wave's starts for the shorter m), apart, last
            at = [1_000, 1_000 + m, 1_003 + 2 * m, 9_000 + 10 * m, 70_123 + 10 * m, 399_999 - m]
            for o in at:
                t[o:o + m] = np.frombuffer(p, dtype=np.uint8)
            for o in (150_000, 220_000, 300_000):        # near misses: one byte flipped
                t[o:o + m] = np.frombuffer(p, dtype=np.uint8)
                k = int(g.integers(0, m))
                t[o + k] = ord("a") if p[k] == ord("b") else ord("b")
            td = torch.from_numpy(t).to(dev)
            want = oracle.count(p, t)
            assert want >= len(at)
            for order in ("ltr", "freq"):
                for peel in (1, 4):
                    got = sm.count(td, p, order=order, bitmap=True, tile_kib=tile, peel=peel)
                    assert got == want, (m, tile, order, peel, got, want)


def test_batch_single_search_launches_on_small_alphabet_texts(dev):
    """Inside a batch, a text of 64 MiB or more with one or two queries runs them as single searches,
    with the bitmap compares when its histogram shows at most 4 symbols.  Counts equal the oracle
    under the text's own histogram, a histogram claiming 2 symbols for a 95-letter text (patterns of
    5 or more distinct symbols fall back to byte compares), and no histogram."""
    g = np.random.default_rng(9105)
    texts_h = [synth.uniform_text((72 << 20) + 5, 2, family=3, stream=11),
               synth.uniform_text((72 << 20) + 77, 4, family=3, stream=12),
               synth.zipf_text((76 << 20) + 3, 95, 1.0, family=3, stream=13)]
    texts_d = [torch.from_numpy(t).to(dev) for t in texts_h]
    queries = [(ti, synth.substring_pattern(texts_h[ti], m, g)[0]) for ti in (0, 1) for m in (7, 300)]
    queries.append((2, synth.substring_pattern(texts_h[2], 40, g)[0]))
    queries.append((2, b"eeee"))                    # at most 4 distinct symbols on the 95-letter text
    want = [oracle.count(p, texts_h[ti]) for ti, p in queries]
    own = [oracle.hist(t) for t in texts_h]
    claims_two = np.zeros(256, dtype=np.uint64)
    claims_two[[ord("e"), ord("t")]] = 1
    for hists in (own, [own[0], own[1], claims_two], None):
        offs, pos = [], 0
        buf = torch.zeros(sum(t.size for t in texts_h) + 64, dtype=torch.uint8, device=dev)
        for t in texts_h:
            pos += 7
            offs.append(pos)
            buf[pos:pos + t.size].copy_(torch.from_numpy(t))
            pos += t.size
        pt = sm.PackedTexts(buf, offs, [t.size for t in texts_h],
                            None if hists is None else np.stack(hists))
        assert sm.count_batch(pt, queries).cpu().tolist() == want
        del buf, pt
