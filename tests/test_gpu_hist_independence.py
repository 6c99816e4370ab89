"""Counts never depend on the symbol frequencies a caller supplies.

Section 2.2 takes the frequencies that order the compares from some corpus of
the same kind, and Algorithm 4's count is the same under every compare order
(Section 2.3): frequencies are a speed input only.  These tests hand the batch
entry points and the pair-count pass histograms that are understated, foreign
or all zero, with enough queries per text that the bitmap mode is taken, and
compare every result with the oracle on the bytes actually searched.
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


def alphabet_text(n, alpha: bytes, seed):
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[np.random.default_rng(seed).integers(0, a.size, size=n)]


def packed(texts_h, dev, hists):
    offs, pos = [], 0
    for i, th in enumerate(texts_h):
        pos += 3 + i % 13                          # misaligned starts
        offs.append(pos)
        pos += th.size
    buf = torch.zeros(pos + 16, dtype=torch.uint8, device=dev)
    for o, th in zip(offs, texts_h):
        buf[o:o + th.size].copy_(torch.from_numpy(th))
    return buf, offs, [th.size for th in texts_h], sm.PackedTexts(buf, offs, [th.size for th in texts_h], hists)


def mixed_queries(texts_h, per_text, g, extra_alpha=b""):
    """Substrings, random patterns over each text's alphabet (plus extra_alpha), and single symbols."""
    queries = []
    for ti, t in enumerate(texts_h):
        alpha = np.unique(np.concatenate([t[:4096], np.frombuffer(extra_alpha or b"\0", dtype=np.uint8)]))
        for k in range(per_text):
            m = int(synth.loguniform_ints(1, 600, 1, g)[0])
            if k % 3 == 0 and t.size >= m:
                o = int(g.integers(0, t.size - m + 1))
                p = bytes(t[o:o + m])
            elif k % 3 == 1:
                p = bytes(alpha[g.integers(0, alpha.size, size=min(m, 6))])
            else:
                p = bytes([int(t[int(g.integers(0, t.size))])])
            queries.append((ti, p))
    return queries


def understated(h):
    """Keeps only the three rarest present symbols: every other present symbol looks absent."""
    out = np.zeros(256, dtype=np.uint64)
    present = np.flatnonzero(h)
    keep = present[np.argsort(h[present], kind="stable")[:3]]
    out[keep] = h[keep]
    return out


def test_batch_counts_with_inexact_histograms(dev):
    """Bitmap-mode batches (histogram given, >= 32 queries per text) under understated, foreign and
    all-zero histograms equal the oracle, and equal the batch run with each text's own histogram."""
    g = np.random.default_rng(7001)
    texts_h = [synth.zipf_text(400_003, 95, 1.0, family=11, stream=1),
               alphabet_text(123_457, synth.ALPHABETS[4], 2),
               alphabet_text(70_001, synth.ALPHABETS[20], 3),
               alphabet_text(9_000, synth.ALPHABETS[2], 4),
               synth.zipf_text(1_000_000, 95, 1.0, family=11, stream=5)]
    queries = mixed_queries(texts_h, 60, g)
    want = [oracle.count(p, texts_h[ti]) for ti, p in queries]
    own = np.stack([oracle.hist(t) for t in texts_h])
    foreign = np.stack([oracle.hist(texts_h[(i + 1) % len(texts_h)]) for i in range(len(texts_h))])
    variants = {
        "own": own,
        "understated": np.stack([understated(h) for h in own]),
        "foreign": foreign,
        "zero": np.zeros_like(own),
        "uniform": np.ones_like(own),
    }
    _, _, _, none_pt = packed(texts_h, dev, None)
    assert sm.count_batch(none_pt, queries).cpu().tolist() == want
    for name, hists in variants.items():
        _, _, _, pt = packed(texts_h, dev, hists)
        got = sm.count_batch(pt, queries).cpu().tolist()
        bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b][:5]
        assert not bad, (name, [(queries[i][0], queries[i][1][:12], got[i], want[i]) for i in bad])
        assert sm.count_batch(pt, queries, peel=3).cpu().tolist() == want, name


def test_text_object_with_foreign_histogram(dev):
    """A Text whose histogram was taken from another kind of text (ACGT against a 95-letter text)."""
    g = np.random.default_rng(7002)
    t = synth.zipf_text(2_000_003, 95, 1.0, family=11, stream=9)
    text = sm.Text(torch.from_numpy(t).to(dev))
    text._hist = oracle.hist(alphabet_text(100_000, synth.ALPHABETS[4], 9))   # frequencies from elsewhere
    queries = mixed_queries([t], 200, g)
    want = [oracle.count(p, t) for _, p in queries]
    assert sm.count_batch([text], queries).cpu().tolist() == want
    assert all(sm.count(text, p) == w for (_, p), w in list(zip(queries, want))[:20])


def test_plan_replays_after_texts_gain_new_symbols(dev):
    """A plan made on ACGT texts (with their histograms) and replayed from a graph after the texts are
    rewritten over other alphabets, symbols never seen at plan time included."""
    g = np.random.default_rng(7003)
    lens = [150_001, 64_000, 333_333]
    first = [alphabet_text(n, synth.ALPHABETS[4], 20 + i) for i, n in enumerate(lens)]
    later_alpha = b"acgtxyz0123456789ACGT.,;"
    later = [alphabet_text(n, later_alpha, 30 + i) for i, n in enumerate(lens)]
    hists = np.stack([oracle.hist(t) for t in first])
    buf, offs, _, pt = packed(first, dev, hists)
    queries = mixed_queries(first, 40, g) + mixed_queries(later, 40, g, extra_alpha=later_alpha)
    plan = sm.BatchPlan(pt, queries)
    out = torch.full((len(queries),), -1, dtype=torch.int64, device=dev)
    assert plan.run(out).cpu().tolist() == [oracle.count(p, first[ti]) for ti, p in queries]

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(out)
    for rep, texts_h in enumerate((first, later, later, first)):
        for o, th in zip(offs, texts_h):
            buf[o:o + th.size].copy_(torch.from_numpy(th))
        want = [oracle.count(p, texts_h[ti]) for ti, p in queries]
        out.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert out.cpu().tolist() == want, f"replay {rep}"
        ti, p = queries[-1 - rep]
        assert sm.count(buf[offs[ti]:offs[ti] + lens[ti]], p) == want[-1 - rep]
    plan.close()


def test_bigram_ignores_understated_histogram(dev):
    """Pair counts are exact when the caller's histogram hides the high or the low byte half."""
    t = np.random.default_rng(7004).integers(0, 256, size=3_000_017, dtype=np.uint8)
    td = torch.from_numpy(t).to(dev)
    want = oracle.bigram(t).tolist()
    h = oracle.hist(t)
    low_only = h.copy()
    low_only[128:] = 0
    high_only = h.copy()
    high_only[:128] = 0
    for hint in (low_only, high_only, np.zeros(256, dtype=np.uint64), None):
        got = sm.bigram(td, hint).cpu().numpy().astype(np.uint64).tolist()
        assert got == want
