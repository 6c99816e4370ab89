"""Lone queries on small-alphabet texts inside a batch (bitmap deals) against the oracle.

A text holding one count query, whose histogram shows at most 4 symbols and whose pattern has at
most 4 distinct symbols and m <= 8192, runs as runs of 16 KiB bitmap tiles: Section 2.1's
SIMDcompare of each distinct pattern symbol becomes one bit per text byte and tile, each compare a
shift and AND of those bits, with Algorithm 4's peel and zero tests.  These cases cover texts from
one byte to several tiles at every start alignment, patterns of 1 to 4 distinct symbols (and 5,
which take the byte deals), the longest pattern the bitmap tiles take and the next one, patterns
longer than their text or holding symbols their text lacks, histograms that understate a text's
alphabet (counts must not depend on them), and plans replayed in a graph after their texts were
rewritten with symbols unseen at planning.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

sm = pytest.importorskip("paper_1612_01506_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def over(alpha: bytes, n: int, g) -> np.ndarray:
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[g.integers(0, a.size, size=n)]


def pack(dev, texts):
    """Texts back to back at start offsets 0..15 past a 16-byte boundary."""
    offs, pos = [], 0
    for i, t in enumerate(texts):
        pos = (pos + 15) // 16 * 16 + i % 16
        offs.append(pos)
        pos += t.size
    buf = torch.zeros(pos + 64, dtype=torch.uint8, device=dev)
    for o, t in zip(offs, texts):
        if t.size:
            buf[o:o + t.size].copy_(torch.from_numpy(t))
    return buf, offs


def pattern_for(t: np.ndarray, k: int, g) -> bytes:
    """Kinds 0..6: a substring, random patterns over 1..4 of the text's symbols, 5 symbols (byte
    deals), a symbol the text lacks; lengths from 1 to 4097."""
    m = int(np.exp(g.uniform(0, np.log(4097)))) if k != 6 else int(g.integers(1, 40))
    syms = np.unique(t) if t.size else np.frombuffer(b"ab", dtype=np.uint8)
    if k == 0 and 0 < t.size:
        m = min(m, t.size)
        o = int(g.integers(0, t.size - m + 1))
        return bytes(t[o:o + m])
    if k in (1, 2, 3, 4):
        pick = syms[g.integers(0, syms.size, size=min(k, syms.size))]
        return bytes(pick[g.integers(0, pick.size, size=m)])
    if k == 5:
        return bytes(over(b"ACGTN", m, g))
    return bytes(over(b"ab", m, g)) + b"Z"     # 'Z' is in no text


def test_ragged_texts_one_query_each(dev):
    g = np.random.default_rng(9200)
    sizes = [0, 1, 2, 7, 31, 32, 33, 255, 4095, 4096, 4097, 8159, 8192, 8193, 16_383, 32_768, 32_769,
             65_537, 131_101, 262_145, 1_000_003]
    alphas = [b"ab", b"ACGT", b"xyz", b"a"]
    texts, queries = [], []
    for n in sizes:
        for a in alphas:
            for k in range(7):
                t = over(a, n, g)
                texts.append(t)
                queries.append((len(texts) - 1, pattern_for(t, k, g)))
    # the longest pattern the bitmap tiles take (a halo of 256 words) and the next one
    for m in (4096, 8191, 8192, 8193, 9000):
        t = over(b"ab", 300_000, g)
        o = int(g.integers(0, 100_000))
        t[o + 100_000:o + 100_000 + m] = t[o:o + m]
        texts.append(t)
        queries.append((len(texts) - 1, bytes(t[o:o + m])))
    buf, offs = pack(dev, texts)
    hists = np.stack([oracle.hist(t) for t in texts])
    pt = sm.PackedTexts(buf, offs, [t.size for t in texts], hists)
    want = [oracle.count(p, texts[ti]) for ti, p in queries]
    got = sm.count_batch(pt, queries).cpu().tolist()
    bad = [(i, len(queries[i][1]), texts[queries[i][0]].size, got[i], want[i]) for i in range(len(want))
           if got[i] != want[i]]
    assert not bad, bad[:10]
    assert sum(want) > 1000


def test_understated_histograms(dev):
    """95-letter and 20-letter texts whose histograms claim 2 or 4 symbols: the planner takes the
    bitmap deals, and every text byte outside the pattern's symbols sets no bit."""
    g = np.random.default_rng(9201)
    texts, queries, hists = [], [], []
    for i in range(60):
        sigma = 95 if i % 2 else 20
        n = int(g.integers(1, 400_000))
        t = (32 + g.integers(0, sigma, size=n)).astype(np.uint8)
        texts.append(t)
        syms = np.unique(t)
        claim = np.zeros(256, dtype=np.uint64)
        few = syms[g.integers(0, syms.size, size=2 + (i % 3))]
        claim[few] = g.integers(1, 1000, size=few.size).astype(np.uint64)
        hists.append(claim)
        if i % 3 == 0:                        # a substring: matches exist
            m = int(g.integers(1, min(n, 12) + 1))
            o = int(g.integers(0, n - m + 1))
            p = bytes(t[o:o + m])
        else:                                 # over the claimed symbols only
            m = int(g.integers(1, 6))
            p = bytes(few[g.integers(0, few.size, size=m)])
        queries.append((i, p))
    buf, offs = pack(dev, texts)
    pt = sm.PackedTexts(buf, offs, [t.size for t in texts], np.stack(hists))
    want = [oracle.count(p, texts[ti]) for ti, p in queries]
    assert sm.count_batch(pt, queries).cpu().tolist() == want
    assert sum(want) > 100


def test_plan_replays_after_texts_gain_symbols(dev):
    """A plan built while the texts held 2-4 symbols, replayed in a graph after they were rewritten
    with 95-letter bytes (and the patterns planted): counts follow the new contents."""
    g = np.random.default_rng(9202)
    n_texts = 40
    texts = [over((b"ab", b"ACGT", b"xyz")[i % 3], int(g.integers(10, 200_000)), g) for i in range(n_texts)]
    queries = [(i, pattern_for(texts[i], 1 + i % 4, g)) for i in range(n_texts)]
    buf, offs = pack(dev, texts)
    pt = sm.PackedTexts(buf, offs, [t.size for t in texts], np.stack([oracle.hist(t) for t in texts]))
    plan = sm.BatchPlan(pt, queries)
    out = torch.full((n_texts,), -1, dtype=torch.int64, device=dev)
    plan.run(out)
    assert out.cpu().tolist() == [oracle.count(p, texts[ti]) for ti, p in queries]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(out)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(out)
    for rnd in range(3):
        new = []
        for (ti, p), t in zip(queries, texts):
            u = (32 + g.integers(0, 95, size=t.size)).astype(np.uint8)
            if rnd and len(p) <= u.size:      # plant the pattern a few times
                for _ in range(3):
                    o = int(g.integers(0, u.size - len(p) + 1))
                    u[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
            new.append(u)
        for o, u in zip(offs, new):
            buf[o:o + u.size].copy_(torch.from_numpy(u))
        out.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        want = [oracle.count(p, new[ti]) for ti, p in queries]
        assert out.cpu().tolist() == want, rnd
    del graph
    plan.close()
