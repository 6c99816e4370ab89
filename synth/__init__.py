"""Seeded synthetic inputs for exact string matching: texts, patterns, workloads.

This module only draws bytes.  It holds none of the matching arithmetic, so both
the GPU path's tests/benchmarks and the CPU oracle's tests can take their inputs
from here without sharing any search code.

Workload shapes follow the paper's experiments (Section 3): natural-language
texts with large alphabets (|Sigma| = 63 and 117), DNA (|Sigma| = 4) and protein
(|Sigma| = 19), searched with patterns picked at random from the text
(Section 2.3).  The corpus files themselves are replaced by order-0 i.i.d.
sources with matching alphabet sizes:

* sigma = 95: printable bytes 0x20..0x7E with Zipf(s) rank probabilities under a
  seeded rank -> symbol permutation (stand-in for the natural-language files);
* sigma = 4: ACGT uniform (stand-in for E.coli);
* sigma = 20: the 20 one-letter amino-acid codes (stand-in for the protein file);
* sigma = 2: {'0', '1'} uniform (adversarial small alphabet);
* periodic texts u^q (closed-form counts, long partial matches);
* an order-1 Markov text over 26 letters and space whose rows are Zipf laws
  over seeded permutations (adjacent symbols strongly correlated, as in
  natural language; used to measure the bigram-aware compare order).

Bytes are produced by a counter-based splitmix64 hash (Steele, Lea and Flood,
OOPSLA 2014): byte i depends only on (key, i), so a GiB-scale text can be made
in parallel by the C helper ``synth.c`` and any slice of it recomputed here in
numpy.  Keys come from ``numpy.random.SeedSequence([SEED, family, stream])``, where
a family number separates the workloads and a stream number the texts and draws within one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

SEED = 161201506
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

ALPHABETS = {
    2: b"01",
    4: b"ACGT",
    20: b"ACDEFGHIKLMNPQRSTVWY",
    95: bytes(range(0x20, 0x7F)),
}

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


# ----------------------------------------------------------------------------- seeds
def stream_key(family: int, stream: int) -> int:
    """64-bit generator key for (family, stream) under the master seed."""
    ss = np.random.SeedSequence([SEED, int(family), int(stream)])
    return int(ss.generate_state(1, dtype=np.uint64)[0])


def rng(family: int, stream: int) -> np.random.Generator:
    """numpy Generator for the small draws (offsets, lengths, patterns)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, int(family), int(stream)])))


# ------------------------------------------------------------------------ symbol laws
def zipf_thresholds(sigma: int, s: float = 1.0) -> np.ndarray:
    """Inverse-CDF thresholds (sigma-1 entries, 2^32 scale) for Zipf(s) over ranks 1..sigma.

    Rank k has probability k^-s / H(sigma, s).  The quantisation to 2^32 changes
    each probability by < 2^-32.
    """
    k = np.arange(1, sigma + 1, dtype=np.float64)
    p = k ** (-float(s))
    p /= p.sum()
    c = np.cumsum(p)[:-1]
    thr = np.minimum(np.rint(c * 2.0**32), 2.0**32 - 1).astype(np.uint64)
    return thr.astype(np.uint32)


def uniform_thresholds(sigma: int) -> np.ndarray:
    k = np.arange(1, sigma, dtype=np.uint64)
    return ((k << np.uint64(32)) // np.uint64(sigma)).astype(np.uint32)


def rank_permutation(alphabet: bytes, family: int, stream: int) -> bytes:
    """Seeded rank -> symbol map (rank 0 is the most probable symbol)."""
    perm = rng(family, 10_000 + stream).permutation(len(alphabet))
    return bytes(alphabet[i] for i in perm)


# ----------------------------------------------------------------------------- texts
def _lib():
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.synth_text.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_char_p,
                               ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.synth_text.restype = None
    lib.synth_markov.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_char_p,
                                 ctypes.c_void_p, ctypes.c_int]
    lib.synth_markov.restype = None
    return lib


def build() -> None:
    """Compile the bulk generator (gcc, OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src], check=True)
    os.replace(tmp, _LIB_PATH)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def iid_text_numpy(n: int, symbols: bytes, thr: np.ndarray, key: int, start: int = 0) -> np.ndarray:
    """Reference (numpy) form of the generator: bytes [start, start+n) of the text."""
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(32)).astype(np.uint32)
    idx = np.searchsorted(thr, u, side="right")
    return np.frombuffer(symbols, dtype=np.uint8)[idx]


def iid_text(n: int, symbols: bytes, thr: np.ndarray, key: int) -> np.ndarray:
    """i.i.d. text of n bytes (bulk C path)."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    assert len(thr) == len(symbols) - 1
    out = np.empty(n, dtype=np.uint8)
    if n:
        _lib().synth_text(out.ctypes.data, n, key & (2**64 - 1), symbols, thr.ctypes.data, len(thr), _threads())
    return out


def zipf_text(n: int, sigma: int = 95, s: float = 1.0, family: int = 2, stream: int = 0) -> np.ndarray:
    """Order-0 Zipf(s) text over ALPHABETS[sigma] under a seeded rank permutation."""
    syms = rank_permutation(ALPHABETS[sigma], family, stream)
    return iid_text(n, syms, zipf_thresholds(sigma, s), stream_key(family, stream))


def uniform_text(n: int, sigma: int = 4, family: int = 1, stream: int = 0) -> np.ndarray:
    return iid_text(n, ALPHABETS[sigma], uniform_thresholds(sigma), stream_key(family, stream))


def periodic_text(n: int, unit: bytes) -> np.ndarray:
    """u^q truncated to n bytes."""
    u = np.frombuffer(unit, dtype=np.uint8)
    reps = -(-n // len(u)) if n else 0
    return np.tile(u, reps)[:n].copy()


LETTERS = b"abcdefghijklmnopqrstuvwxyz "


def markov_thresholds(sigma: int = 27, s: float = 1.3, family: int = 8, stream: int = 0) -> np.ndarray:
    """(sigma, sigma-1) uint32 inverse-CDF rows: row a is Zipf(s) over a seeded permutation of the
    successors, so each symbol has a few likely followers."""
    g = rng(family, 20_000 + stream)
    k = np.arange(1, sigma + 1, dtype=np.float64)
    rows = []
    for _ in range(sigma):
        pk = k ** (-float(s))
        pk /= pk.sum()
        probs = np.empty(sigma)
        probs[g.permutation(sigma)] = pk           # rank r -> a seeded successor
        c = np.cumsum(probs)[:-1]
        rows.append(np.minimum(np.rint(c * 2.0**32), 2.0**32 - 1).astype(np.uint64).astype(np.uint32))
    return np.stack(rows)


def markov_text(n: int, family: int = 8, stream: int = 0, s: float = 1.3) -> np.ndarray:
    """Order-1 Markov text over LETTERS (bulk C path; sequential)."""
    thr = np.ascontiguousarray(markov_thresholds(len(LETTERS), s, family, stream))
    out = np.empty(n, dtype=np.uint8)
    if n:
        _lib().synth_markov(out.ctypes.data, n, stream_key(family, stream) & (2**64 - 1), LETTERS,
                            thr.ctypes.data, len(LETTERS))
    return out


def markov_text_numpy(n: int, family: int = 8, stream: int = 0, s: float = 1.3) -> np.ndarray:
    """Reference (Python loop) form of markov_text, for small n."""
    thr = markov_thresholds(len(LETTERS), s, family, stream)
    key = np.uint64(stream_key(family, stream))
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(32)).astype(np.uint32)
    sym = np.frombuffer(LETTERS, dtype=np.uint8)
    out = np.empty(n, dtype=np.uint8)
    x = 0
    for j in range(n):
        x = int(np.searchsorted(thr[x], u[j], side="right"))
        out[j] = sym[x]
    return out


# -------------------------------------------------------------------------- patterns
def loguniform_ints(lo: int, hi: int, count: int, g: np.random.Generator) -> np.ndarray:
    """round(2^U(log2 lo, log2 hi)), clipped to [lo, hi]."""
    x = np.exp2(g.uniform(np.log2(lo), np.log2(hi), size=count))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def substring_pattern(t: np.ndarray, m: int, g: np.random.Generator) -> tuple[bytes, int]:
    """Pattern picked at random from the text (Section 2.3): t[o:o+m], o uniform in [0, n-m]."""
    o = int(g.integers(0, len(t) - m + 1))
    return bytes(t[o:o + m]), o


def random_pattern(symbols: bytes, m: int, g: np.random.Generator) -> bytes:
    idx = g.integers(0, len(symbols), size=m)
    return bytes(np.frombuffer(symbols, dtype=np.uint8)[idx])


# ------------------------------------------------------------------------- workloads
@dataclass
class Query:
    text_id: int
    pattern: bytes
    report: bool = False


def single_count_workload(n: int = 8 << 20, m: int = 16):
    """Single count search: uniform ACGT text, one substring pattern at a seeded offset."""
    t = uniform_text(n, 4, family=1, stream=0)
    p, _ = substring_pattern(t, m, rng(1, 1))
    return t, p


def zipf_workload(n: int = 1 << 30, per_m: int = 100,
                  ms=(2, 4, 8, 16, 32, 64, 128, 256, 512, 1024), report_min_m: int = 64):
    """Skewed large alphabet: Zipf(1.0) sigma=95 text and per_m substring patterns for each m.

    Returns (text, list of (pattern, report_flag)).  Report mode is requested for m >= report_min_m.
    """
    t = zipf_text(n, 95, 1.0, family=2, stream=0)
    g = rng(2, 1)
    pats = []
    for m in ms:
        for _ in range(per_m):
            if m <= n:
                p, _ = substring_pattern(t, m, g)
                pats.append((p, m >= report_min_m))
    return t, pats


def small_alphabet_workload(n: int = 1 << 30, sigma: int = 2, ms=(8, 64, 512, 4096), per_m: int = 10):
    t = uniform_text(n, sigma, family=3, stream=sigma)
    g = rng(3, 100 + sigma)
    pats = []
    for m in ms:
        if m > n:
            continue
        for _ in range(per_m):
            pats.append(substring_pattern(t, m, g)[0])
        pats.append(random_pattern(ALPHABETS[sigma], m, g))
    return t, pats


def batched_one_text_workload(n: int = 2 << 30, nq: int = 10_000, lo: int = 2, hi: int = 1024):
    """One Zipf sigma=95 text, nq patterns with m log-uniform in [lo, hi]; half substrings, half random."""
    t = zipf_text(n, 95, 1.0, family=4, stream=0)
    g = rng(4, 1)
    ms = loguniform_ints(lo, hi, nq, g)
    pats = []
    for i, m in enumerate(ms):
        m = int(min(m, n))
        if i % 2 == 0:
            pats.append(substring_pattern(t, m, g)[0])
        else:
            pats.append(random_pattern(ALPHABETS[95], m, g))
    return t, pats


def batched_many_texts_workload(ntexts: int = 4096, lo: int = 4 << 10, hi: int = 4 << 20,
                                mlo: int = 4, mhi: int = 256):
    """ntexts texts with lengths log-uniform in [lo, hi], sigma in {4, 20, 95} round-robin, one pattern each."""
    g = rng(4, 2)
    lens = loguniform_ints(lo, hi, ntexts, g)
    ms = loguniform_ints(mlo, mhi, ntexts, g)
    texts, pats = [], []
    for i in range(ntexts):
        sigma = (4, 20, 95)[i % 3]
        if sigma == 95:
            t = zipf_text(int(lens[i]), 95, 1.0, family=4, stream=100 + i)
        else:
            t = uniform_text(int(lens[i]), sigma, family=4, stream=100 + i)
        m = int(min(ms[i], len(t)))
        texts.append(t)
        pats.append(substring_pattern(t, m, g)[0])
    return texts, pats
