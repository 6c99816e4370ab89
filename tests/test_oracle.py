"""Pins for the CPU oracle: brute force, the Figure 1 worked example, closed forms, invariants.

None of these checks retypes the oracle's own loop: the references are Python
slicing, the stdlib ``re`` engine (lookahead finds overlapping matches, plain
``finditer`` disjoint ones), ``bytes.count`` (disjoint, leftmost first), numpy's bincount, closed-form counts of periodic texts and algebraic
invariants (reversal, thread split, compare order and peel factor).
"""
import itertools
import json
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_positions(p: bytes, t: bytes):
    m = len(p)
    return [s for s in range(len(t) - m + 1) if t[s:s + m] == p]


def re_positions(p: bytes, t: bytes):
    return [mt.start() for mt in re.finditer(b"(?=" + re.escape(p) + b")", t)]


# --------------------------------------------------------------------------- Figure 1
def test_fig1_prefix_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "fig1_prefix.json")))
    t, p = g["text"].encode(), g["pattern"].encode()
    assert oracle.count(p, t, 1) == g["count"]
    assert oracle.report(p, t).tolist() == g["positions_0based"]
    # The Algorithm 4 emulation (r = m: every compare peeled) reaches the same count.
    for r in range(1, len(p) + 1):
        assert oracle.alg4_count(p, t, None, r) == g["count"]
    # found after each left-to-right compare (bit k = start k), from the caption's alignment.
    valid = len(t) - len(p) + 1
    found = set(range(valid))
    for j, expect in enumerate(g["found_after_each_compare_ltr"]):
        found = {k for k in found if t[k + j] == p[j]}
        assert sorted(found) == expect
    # A prefix of the pattern shows up at both a-positions.
    assert oracle.report(b"a", t).tolist() == [0, 1]


# --------------------------------------------------------------------- brute force
def test_exhaustive_binary_small():
    """Every text over {a,b} with n <= 9 against every pattern with 1 <= m <= 4."""
    pats = [bytes(x) for m in range(1, 5) for x in itertools.product(b"ab", repeat=m)]
    for n in range(0, 10):
        for tx in itertools.product(b"ab", repeat=n):
            t = bytes(tx)
            for p in pats:
                want = brute_positions(p, t)
                assert oracle.count(p, t, 1) == len(want), (p, t)
                assert oracle.report(p, t).tolist() == want, (p, t)


@settings(max_examples=300, deadline=None)
@given(t=st.binary(min_size=0, max_size=600), m=st.integers(1, 8), data=st.data())
def test_random_bytes_vs_re(t, m, data):
    if len(t) >= m and data.draw(st.booleans()):
        o = data.draw(st.integers(0, len(t) - m))
        p = t[o:o + m]
    else:
        p = data.draw(st.binary(min_size=m, max_size=m))
    want = re_positions(p, t)
    assert want == brute_positions(p, t)
    assert oracle.count(p, t, 2) == len(want)
    assert oracle.report(p, t).tolist() == want


@pytest.mark.parametrize("b", [0x00, 0x01, 0x7F, 0x80, 0xFE, 0xFF])
def test_extreme_byte_values(b):
    g = np.random.default_rng(b)
    t = g.choice(np.array([b, b ^ 0x80, 0x00, 0xFF], dtype=np.uint8), size=3000)
    tb = t.tobytes()
    for m in (1, 2, 3, 5, 9):
        o = int(g.integers(0, len(tb) - m))
        p = tb[o:o + m]
        assert oracle.count(p, tb, 3) == len(re_positions(p, tb))


def test_degenerate_lengths():
    assert oracle.count(b"abc", b"ab") == 0          # m > n
    assert oracle.count(b"a", b"") == 0              # n == 0
    assert oracle.count(b"abc", b"abc") == 1         # m == n
    assert oracle.count(b"abd", b"abc") == 0
    with pytest.raises(ValueError):
        oracle.count(b"", b"abc")                    # m == 0 is rejected
    with pytest.raises(ValueError):
        oracle.alg4_count(b"", b"abc")


# --------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,k", [(1, 1), (100, 1), (100, 7), (4096, 16), (5000, 256), (300, 300), (299, 300)])
def test_unary_text_closed_form(n, k):
    t = b"a" * n
    assert oracle.count(b"a" * k, t) == max(0, n - k + 1)
    assert oracle.count(b"a" * (k - 1) + b"b", t) == 0
    assert oracle.alg4_count(b"a" * k, t, None, 2) == max(0, n - k + 1)


@pytest.mark.parametrize("unit", [b"ab", b"abc", b"aab", b"aaab", b"abcabd", b"GATTACA"])
@pytest.mark.parametrize("n", [0, 1, 17, 64, 65, 1000, 4099])
def test_periodic_closed_form(unit, n):
    """t = u^q (u primitive, |u| = L); p = factor of u^inf at phase o with m >= L.

    A primitive word occurs in u^inf only at phases = o (mod L), hence
    count = floor((n - m - o) / L) + 1 if n >= m + o, else 0.
    """
    L = len(unit)
    t = (unit * (n // L + 2))[:n]
    for o in range(L):
        for m in (L, L + 1, 2 * L + 3, 5 * L):
            p = (unit * (m // L + 3))[o:o + m]
            want = (n - m - o) // L + 1 if n >= m + o else 0
            assert oracle.count(p, t) == want, (unit, n, o, m)


# ------------------------------------------------------------------------ invariants
def test_reverse_invariance_and_thread_split():
    g = np.random.default_rng(7)
    t = g.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=200_000).tobytes()
    for m in (1, 3, 6, 9):
        o = int(g.integers(0, len(t) - m))
        p = t[o:o + m]
        c = oracle.count(p, t, 1)
        assert c >= 1
        assert c <= len(t) - m + 1
        assert oracle.count(p[::-1], t[::-1], 1) == c
        for th in (2, 3, 7, 8):
            assert oracle.count(p, t, th) == c
        pos = oracle.report(p, t)
        assert len(pos) == c
        assert np.all(np.diff(pos.astype(np.int64)) > 0)
        for s in pos[:200]:
            assert t[int(s):int(s) + m] == p


def test_report_cap_truncation():
    t = b"abababababab"
    full = oracle.report(b"ab", t).tolist()
    assert full == [0, 2, 4, 6, 8, 10]
    n, head = oracle.report_full(b"ab", t, 4)
    assert n == 6 and head.tolist() == [0, 2, 4, 6]
    n, head = oracle.report_full(b"ab", t, 0)
    assert n == 6 and head.size == 0


# ------------------------------------------------------------------------ histogram
def test_hist_vs_bincount():
    g = np.random.default_rng(3)
    for n in (0, 1, 255, 10_000):
        t = g.integers(0, 256, size=n, dtype=np.uint8)
        h = oracle.hist(t)
        assert h.tolist() == np.bincount(t, minlength=256).tolist()
        assert int(h.sum()) == n


# ---------------------------------------------------------------------------- orders
def _check_freq_order(p: bytes, h, o):
    m = len(p)
    assert sorted(o.tolist()) == list(range(m))
    keys = [int(h[p[j]]) for j in o]
    assert keys == sorted(keys)
    for a, b in zip(o[:-1], o[1:]):        # ties keep increasing position
        if h[p[a]] == h[p[b]]:
            assert a < b


def test_order_freq_properties():
    g = np.random.default_rng(11)
    h = g.integers(0, 50, size=256).astype(np.uint64)
    for m in (1, 2, 5, 64, 1000):
        p = g.integers(0, 256, size=m, dtype=np.uint8).tobytes()
        _check_freq_order(p, h, oracle.order_freq(p, h))
    # equal frequencies -> left to right
    assert oracle.order_freq(b"hello", np.ones(256, np.uint64)).tolist() == [0, 1, 2, 3, 4]
    # worked case: rare symbols first
    h2 = np.zeros(256, np.uint64)
    for ch, f in zip(b"qui", (1, 50, 40)):
        h2[ch] = f
    assert oracle.order_freq(b"qui", h2).tolist() == [0, 2, 1]


def test_order_h_enumeration():
    # Section 2.4 listing, 1-based: p[1], p[m], p[4], p[7], ..., p[3], p[6], ..., p[2], p[5], ...
    assert (oracle.order_h(10) + 1).tolist() == [1, 10, 4, 7, 3, 6, 9, 2, 5, 8]
    assert (oracle.order_h(9) + 1).tolist() == [1, 9, 4, 7, 3, 6, 2, 5, 8]
    assert (oracle.order_h(8) + 1).tolist() == [1, 8, 4, 7, 3, 6, 2, 5]
    assert (oracle.order_h(1) + 1).tolist() == [1]
    assert (oracle.order_h(2) + 1).tolist() == [1, 2]
    for m in range(1, 300):
        assert sorted(oracle.order_h(m).tolist()) == list(range(m))


def test_order_hs_spaces_last():
    p = b"to be or not"
    o = oracle.order_hs(p)
    assert sorted(o.tolist()) == list(range(len(p)))
    sp = [j for j in o if p[j] == 0x20]
    assert o.tolist()[-len(sp):] == sp
    h = oracle.order_h(len(p)).tolist()
    assert [j for j in o if p[j] != 0x20] == [j for j in h if p[j] != 0x20]


# ------------------------------------------------- Algorithm 4: order / peel invariance
def test_alg4_all_orders_all_peels():
    g = np.random.default_rng(5)
    t = g.choice(np.frombuffer(b"ab", dtype=np.uint8), size=700).tobytes()
    for m in (1, 2, 3, 4):
        for _ in range(3):
            o = int(g.integers(0, len(t) - m))
            p = t[o:o + m]
            want = len(brute_positions(p, t))
            for perm in itertools.permutations(range(m)):
                for r in range(1, m + 2):
                    assert oracle.alg4_count(p, t, perm, r) == want


@settings(max_examples=150, deadline=None)
@given(t=st.binary(min_size=1, max_size=400), m=st.integers(1, 12), r=st.integers(1, 8), data=st.data())
def test_alg4_random(t, m, r, data):
    if len(t) >= m:
        o = data.draw(st.integers(0, len(t) - m))
        p = t[o:o + m]
    else:
        p = data.draw(st.binary(min_size=m, max_size=m))
    perm = data.draw(st.permutations(list(range(m))))
    want = len(re_positions(p, t))
    assert oracle.alg4_count(p, t, perm, r) == want
    h = oracle.hist(t)
    assert oracle.alg4_count(p, t, oracle.order_freq(p, h), r) == want
    assert oracle.alg4_count(p, t, oracle.order_h(m), r) == want


def test_alg4_block_boundaries():
    """Texts whose start count straddles the 64-start blocks of the emulation."""
    for n in (63, 64, 65, 127, 128, 129, 200):
        t = b"a" * n
        for k in (1, 2, 5):
            assert oracle.alg4_count(b"a" * k, t, None, 3) == max(0, n - k + 1)


# ------------------------------------------------------------ non-overlapping mode
# Pinned against two independent definitions of "disjoint occurrences, leftmost first":
# Python's bytes.count (documented as non-overlapping) and re.finditer without lookahead.
def test_nonoverlap_exhaustive_binary_small():
    pats = [bytes(x) for m in range(1, 5) for x in itertools.product(b"ab", repeat=m)]
    for n in range(0, 10):
        for tx in itertools.product(b"ab", repeat=n):
            t = bytes(tx)
            for p in pats:
                want = [mt.start() for mt in re.finditer(re.escape(p), t)]
                assert oracle.count_nonoverlap(p, t) == t.count(p) == len(want), (p, t)
                assert oracle.report_nonoverlap(p, t).tolist() == want, (p, t)


@settings(max_examples=300, deadline=None)
@given(t=st.binary(min_size=0, max_size=600), m=st.integers(1, 8), data=st.data())
def test_nonoverlap_random_vs_bytes_count(t, m, data):
    alpha = data.draw(st.sampled_from([b"a", b"ab", b"abc", bytes(range(256))]))
    t = bytes(alpha[b % len(alpha)] for b in t)
    p = bytes(alpha[b % len(alpha)] for b in data.draw(st.binary(min_size=m, max_size=m)))
    assert oracle.count_nonoverlap(p, t) == t.count(p)
    assert oracle.report_nonoverlap(p, t).tolist() == [mt.start() for mt in re.finditer(re.escape(p), t)]
    # disjoint occurrences are a subset of all occurrences
    assert set(oracle.report_nonoverlap(p, t).tolist()) <= set(oracle.report(p, t).tolist())


@pytest.mark.parametrize("n,k", [(1, 1), (100, 1), (100, 7), (4096, 16), (5000, 256), (300, 300), (299, 300)])
def test_nonoverlap_unary_closed_form(n, k):
    """a^n with p = a^k: the greedy takes starts 0, k, 2k, ..., floor(n/k) of them."""
    t, p = b"a" * n, b"a" * k
    assert oracle.count_nonoverlap(p, t) == n // k
    assert oracle.report_nonoverlap(p, t).tolist() == list(range(0, (n // k) * k, k))


def test_nonoverlap_periodic_and_cap():
    # (ab)^q with p = (ab)^j: disjoint occurrences every 2j bytes
    for q in (1, 5, 64, 1001):
        for j in (1, 2, 3):
            t, p = b"ab" * q, b"ab" * j
            assert oracle.count_nonoverlap(p, t) == q // j
    # "aaa" in "aaaaaaa": starts 0 and 3 (not 0, 1, ..., 4)
    assert oracle.report_nonoverlap(b"aaa", b"aaaaaaa").tolist() == [0, 3]
    total, first = oracle.report_nonoverlap_full(b"a", b"a" * 50, 7)
    assert total == 50 and first.tolist() == list(range(7))
    assert oracle.count_nonoverlap(b"abc", b"ab") == 0
    with pytest.raises(ValueError):
        oracle.count_nonoverlap(b"", b"abc")


# ------------------------------------------------------------- bigram-aware order
def test_bigram_counts_vs_bincount():
    g = np.random.default_rng(3)
    for n in (0, 1, 2, 3, 1000, 65_537):
        t = g.integers(0, 256, size=n, dtype=np.uint8)
        want = np.bincount(t[:-1].astype(np.int64) * 256 + t[1:], minlength=65536) if n > 1 else np.zeros(65536)
        assert oracle.bigram(t).reshape(-1).tolist() == want.astype(np.uint64).tolist()
    t = np.frombuffer(b"abab", dtype=np.uint8)
    b = oracle.bigram(t)
    assert b[ord("a"), ord("b")] == 2 and b[ord("b"), ord("a")] == 1 and int(b.sum()) == 3


def test_bigram_order_qui_example():
    """Section 2.2's example: u nearly always follows q, so q, i, u beats frequency order q, u, i."""
    t = b"qui " * 10 + b"ii " * 20 + b"xu " * 5
    h, bg = oracle.hist(t), oracle.bigram(t)
    assert h[ord("q")] < h[ord("u")] < h[ord("i")]
    assert oracle.order_freq(b"qui", h).tolist() == [0, 1, 2]
    assert oracle.order_bigram(b"qui", h, bg).tolist() == [0, 2, 1]


def test_bigram_order_reduces_to_frequency_under_independence():
    """With bigram[a][b] = h_a h_b and hist = h * sum(h), every conditional estimate equals the
    unconditional one, so the order is the frequency order (ties by position)."""
    g = np.random.default_rng(11)
    for trial in range(40):
        hs = np.zeros(256, dtype=np.uint64)
        syms = g.choice(256, size=int(g.integers(2, 12)), replace=False)
        hs[syms] = g.integers(1, 50, size=syms.size).astype(np.uint64)
        S = int(hs.sum())
        bg = np.outer(hs, hs).astype(np.uint64)
        h = hs * np.uint64(S)
        m = int(g.integers(1, 40))
        p = bytes(g.choice(syms, size=m).astype(np.uint8))
        assert oracle.order_bigram(p, h, bg).tolist() == oracle.order_freq(p, h).tolist(), trial


def _tables(pairs, hist):
    bg = np.zeros((256, 256), dtype=np.uint64)
    for (a, b), v in pairs.items():
        bg[ord(a), ord(b)] = v
    h = np.zeros(256, dtype=np.uint64)
    for a, v in hist.items():
        h[ord(a)] = v
    return h, bg


def test_bigram_order_backward_conditional_uses_column_sums():
    # p = "xab": b is rarest; then a (right neighbour b compared) has e = bg[a][b] / col(b) = 5/10,
    # x has e = hist[x] / total = 30/100, so x comes before a.  With row(a) = 100 instead of
    # col(b) a would come first.
    h, bg = _tables({("a", "b"): 5, ("z", "b"): 5, ("a", "z"): 95}, {"x": 30, "a": 60, "b": 10})
    assert oracle.order_bigram(b"xab", h, bg).tolist() == [2, 0, 1]


def test_bigram_order_both_neighbours_take_the_smaller_estimate():
    # p = "uvwxy": w (rarest) first, then u; then v has both neighbours compared:
    # min(bg[u][v]/row(u), bg[v][w]/col(w)) = min(0.9, 0.1) = 0.1, which beats x at bg[w][x]/row(w)
    # = 0.2 and y at 0.5.
    h, bg = _tables({("u", "v"): 9, ("u", "q"): 1, ("v", "w"): 1, ("q", "w"): 9, ("w", "x"): 2,
                     ("w", "q"): 8},
                    {"u": 1, "v": 40, "w": 0, "x": 40, "y": 50})
    assert oracle.order_bigram(b"uvwxy", h, bg).tolist() == [2, 0, 1, 3, 4]


def test_bigram_order_is_a_permutation_and_result_invariant():
    g = np.random.default_rng(5)
    t = g.integers(0, 6, size=5000, dtype=np.uint8)
    h, bg = oracle.hist(t), oracle.bigram(t)
    for m in (1, 2, 7, 40):
        p = bytes(t[100:100 + m])
        o = oracle.order_bigram(p, h, bg)
        assert sorted(o.tolist()) == list(range(m))
        for r in (1, 2, min(m, 5)):
            assert oracle.alg4_count(p, t, o, r) == oracle.count(p, t)
    with pytest.raises(ValueError):
        oracle.order_bigram(b"", h, bg)
