"""The seeded generators: bulk C path equals the numpy definition, determinism, symbol laws."""
import numpy as np

import synth


def test_bulk_equals_numpy_definition():
    for sigma in (2, 4, 20, 95):
        syms = synth.rank_permutation(synth.ALPHABETS[sigma], 9, sigma)
        for thr in (synth.uniform_thresholds(sigma), synth.zipf_thresholds(sigma, 1.0)):
            key = synth.stream_key(9, sigma)
            a = synth.iid_text(100_003, syms, thr, key)
            b = synth.iid_text_numpy(100_003, syms, thr, key)
            assert np.array_equal(a, b)
            # any slice can be recomputed on its own (counter-based)
            assert np.array_equal(a[70_000:70_100], synth.iid_text_numpy(100, syms, thr, key, start=70_000))


def test_deterministic_and_alphabet():
    a = synth.zipf_text(50_000, 95, 1.0, family=2, stream=0)
    b = synth.zipf_text(50_000, 95, 1.0, family=2, stream=0)
    assert np.array_equal(a, b)
    assert set(np.unique(a).tolist()) <= set(synth.ALPHABETS[95])
    c = synth.uniform_text(50_000, 4, family=1, stream=0)
    assert set(np.unique(c).tolist()) == set(b"ACGT")


def test_zipf_frequencies_match_law():
    n = 2_000_000
    t = synth.zipf_text(n, 95, 1.0, family=2, stream=3)
    ranks = synth.rank_permutation(synth.ALPHABETS[95], 2, 3)
    k = np.arange(1, 96, dtype=np.float64)
    p = (1.0 / k) / (1.0 / k).sum()
    h = np.bincount(t, minlength=256)
    emp = np.array([h[c] for c in ranks]) / n
    assert abs(p[0] - 0.1947) < 1e-3            # 1 / H_95
    assert np.max(np.abs(emp - p) / np.sqrt(p * (1 - p) / n)) < 6.0


def test_uniform_thresholds_even():
    thr = synth.uniform_thresholds(4).astype(np.uint64)
    assert thr.tolist() == [1 << 30, 2 << 30, 3 << 30]


def test_pattern_helpers():
    g = synth.rng(1, 1)
    t = synth.uniform_text(10_000, 4)
    p, o = synth.substring_pattern(t, 16, g)
    assert p == bytes(t[o:o + 16])
    ms = synth.loguniform_ints(2, 1024, 5000, g)
    assert ms.min() >= 2 and ms.max() <= 1024
    assert 30 < np.median(ms) < 60            # log-uniform median ~ sqrt(2*1024) = 45
    q = synth.random_pattern(synth.ALPHABETS[95], 33, g)
    assert len(q) == 33 and set(q) <= set(synth.ALPHABETS[95])
    assert synth.periodic_text(7, b"ab").tobytes() == b"abababa"


def test_markov_text_matches_reference_and_is_correlated():
    a = synth.markov_text(20_000, family=8, stream=3)
    assert a.tolist() == synth.markov_text_numpy(20_000, family=8, stream=3).tolist()
    assert set(np.unique(a).tolist()) <= set(synth.LETTERS)
    assert synth.markov_text(5000, stream=1).tolist() != synth.markov_text(5000, stream=2).tolist()
    # adjacent symbols are far from independent: the most likely successor of the most frequent
    # symbol is much likelier than that symbol's overall frequency
    big = synth.markov_text(400_000, stream=0)
    x = int(np.bincount(big).argmax())
    nxt = big[1:][big[:-1] == x]
    top = np.bincount(nxt, minlength=256).max() / nxt.size
    assert top > 2 * np.bincount(big, minlength=256).max() / big.size
