"""The AVX2 Algorithm-4 CPU baseline counts exactly what the oracle counts (it is timed in
bench.py, so its results are checked here: every peel, order, tail length and thread count)."""
import numpy as np
import pytest

import cpu_alg4
import oracle
import synth

pytestmark = pytest.mark.skipif(not cpu_alg4.available(), reason="host has no AVX2")


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 63, 64, 65, 1000, 4099, 70_001])
def test_counts_equal_oracle(n):
    g = np.random.default_rng(n + 5)
    for sigma in (2, 4, 95):
        t = synth.uniform_text(n, sigma, family=21, stream=n) if n else np.zeros(0, dtype=np.uint8)
        h = oracle.hist(t)
        for m in (1, 2, 3, 5, 31, 32, 33, 100):
            if n and m <= n and g.random() < 0.7:
                o = int(g.integers(0, n - m + 1))
                p = bytes(t[o:o + m])
            else:
                p = bytes(synth.ALPHABETS[sigma][int(g.integers(0, sigma))] for _ in range(m))
            want = oracle.count(p, t)
            for r in sorted({1, 2, min(5, m), m}):
                for order in (None, cpu_alg4.freq_order(p, h), np.random.default_rng(m).permutation(m)):
                    for th in (1, 4):
                        assert cpu_alg4.count(p, t, order, r, th) == want, (n, sigma, m, r, th)


def test_unary_and_extreme_bytes():
    t = np.full(10_007, 0xFF, dtype=np.uint8)
    assert cpu_alg4.count(b"\xff" * 7, t, r=3, nthreads=3) == 10_007 - 6
    assert cpu_alg4.count(b"\xff" * 6 + b"\x00", t, r=1) == 0
    t[5000] = 0x80
    assert cpu_alg4.count(b"\xff\x80\xff", t) == oracle.count(b"\xff\x80\xff", t) == 1


def test_rejects_empty_pattern():
    with pytest.raises(ValueError):
        cpu_alg4.count(b"", np.zeros(10, dtype=np.uint8))
