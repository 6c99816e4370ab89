"""One-shot count batches of many queries over many texts, which the library plans in two parts
(split by text id, so that the GPU runs the first while the host plans the second), against the
oracle and against the same batch planned whole (BatchPlan).  The queries arrive shuffled, texts
take every launch mode (bitmap mode, byte tiles shared by several queries, lone queries as byte or
bitmap deals), and batches whose queries all sit on the first or the last text are not split."""
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


def make_texts(g, n_texts=600):
    texts = []
    for i in range(n_texts):
        n = int(np.exp(g.uniform(np.log(16), np.log(300_000))))
        if i % 3 == 0:
            a = np.frombuffer(b"ACGT", dtype=np.uint8)
            texts.append(a[g.integers(0, 4, size=n)])
        elif i % 3 == 1:
            texts.append((65 + g.integers(0, 20, size=n)).astype(np.uint8))
        else:
            ranks = np.minimum(g.zipf(1.3, size=n), 95) - 1
            texts.append((32 + ranks).astype(np.uint8))
    return texts


def queries_for(texts, g):
    q = []
    for ti, t in enumerate(texts):
        k = 40 if ti % 25 == 7 else 1 + ti % 4      # every 25th text takes the bitmap mode
        for _ in range(k):
            m = int(np.exp(g.uniform(0, np.log(300))))
            if t.size >= m and g.random() < 0.7:
                o = int(g.integers(0, t.size - m + 1))
                q.append((ti, bytes(t[o:o + m])))
            else:
                q.append((ti, bytes(t[g.integers(0, t.size, size=m)]) if t.size else b"A" * m))
    order = g.permutation(len(q))
    return [q[i] for i in order]


def pack(dev, texts):
    offs, pos = [], 0
    for i, t in enumerate(texts):
        pos += i % 16
        offs.append(pos)
        pos += t.size
    buf = torch.zeros(pos + 64, dtype=torch.uint8, device=dev)
    for o, t in zip(offs, texts):
        buf[o:o + t.size].copy_(torch.from_numpy(t))
    return buf, offs


def test_split_batch_equals_oracle_and_whole_plan(dev):
    g = np.random.default_rng(9300)
    texts = make_texts(g)
    queries = queries_for(texts, g)
    assert len(queries) >= 2048 and len(texts) >= 512       # the split applies
    buf, offs = pack(dev, texts)
    pt = sm.PackedTexts(buf, offs, [t.size for t in texts], np.stack([oracle.hist(t) for t in texts]))
    want = [oracle.count(p, texts[ti]) for ti, p in queries]
    got = sm.count_batch(pt, queries).cpu().tolist()
    bad = [(i, queries[i][0], len(queries[i][1]), got[i], want[i]) for i in range(len(want)) if got[i] != want[i]]
    assert not bad, bad[:10]
    plan = sm.BatchPlan(pt, queries)
    out = torch.full((len(queries),), -1, dtype=torch.int64, device=dev)
    plan.run(out)
    assert out.cpu().tolist() == want
    plan.close()
    # twice in a row on one stream, then with stale counts in the output: every slot is rewritten
    out2 = sm.count_batch(pt, queries)
    out3 = sm.count_batch(pt, queries)
    assert out2.cpu().tolist() == want and out3.cpu().tolist() == want
    assert sum(want) > 10_000


@pytest.mark.parametrize("where", ["first", "last"])
def test_batches_on_one_text_are_not_split(dev, where):
    g = np.random.default_rng(9301)
    texts = make_texts(g)
    ti = 0 if where == "first" else len(texts) - 1
    t = texts[ti]
    queries = []
    for _ in range(2100):
        m = int(g.integers(1, 12))
        o = int(g.integers(0, max(t.size - m, 0) + 1))
        queries.append((ti, bytes(t[o:o + m]) if t.size >= m else b"A" * m))
    buf, offs = pack(dev, texts)
    pt = sm.PackedTexts(buf, offs, [x.size for x in texts], np.stack([oracle.hist(x) for x in texts]))
    want = [oracle.count(p, texts[ti]) for ti, p in queries]
    assert sm.count_batch(pt, queries).cpu().tolist() == want
