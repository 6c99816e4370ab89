/*
 * Seeded synthetic text generator (bulk path for GiB-scale texts).
 *
 * This file draws symbols; it holds none of the string-matching arithmetic and
 * is shared by the GPU tests, the benchmark and the oracle tests only as a
 * source of input bytes.
 *
 * Generator: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used as a counter-based hash: the value for
 * text index i is the splitmix64 output function applied to
 * key + (i + 1) * 0x9E3779B97F4A7C15.  The top 32 bits u select a symbol by
 * inverse CDF: the symbol index is the number of thresholds thr[k] <= u
 * (thr has nthr = sigma - 1 non-decreasing entries, scaled to 2^32).
 * synth/__init__.py holds a numpy implementation of the same definition; the
 * tests check that both agree byte for byte.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void synth_text(uint8_t *out, uint64_t n, uint64_t key, const uint8_t *symbols,
                const uint32_t *thr, int nthr, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t z = key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
        uint32_t u = (uint32_t)(mix64(z) >> 32);
        int lo = 0, hi = nthr; /* count thresholds <= u by binary search */
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (thr[mid] <= u)
                lo = mid + 1;
            else
                hi = mid;
        }
        out[i] = symbols[lo];
    }
}

/* Order-1 Markov text: byte i is symbols[x_i], where x_i is drawn by inverse
 * CDF from row x_{i-1} of a transition table (x_{-1} = 0) with the same
 * counter-based uniform u_i as above.  thr holds nsym rows of nsym - 1
 * non-decreasing thresholds.  Sequential: each byte depends on the previous. */
void synth_markov(uint8_t *out, uint64_t n, uint64_t key, const uint8_t *symbols, const uint32_t *thr, int nsym)
{
    /* guide table: for each row and each value of the top 12 bits of u, the
     * number of thresholds below that 2^20-wide bucket; the exact count then
     * needs a short forward scan (the same result as a binary search) */
    enum { GB = 12 };
    const int nthr = nsym - 1;
    uint8_t *guide = (uint8_t *)malloc((size_t)nsym << GB);
    if (!guide)
        return;
    for (int r = 0; r < nsym; ++r) {
        const uint32_t *row = thr + (size_t)r * (size_t)nthr;
        int k = 0;
        for (uint32_t b = 0; b < (1u << GB); ++b) {
            const uint32_t lo = b << (32 - GB);
            while (k < nthr && row[k] < lo)
                ++k;
            guide[((size_t)r << GB) + b] = (uint8_t)k;
        }
    }
    int x = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t z = key + (i + 1) * 0x9E3779B97F4A7C15ULL;
        uint32_t u = (uint32_t)(mix64(z) >> 32);
        const uint32_t *row = thr + (size_t)x * (size_t)nthr;
        int k = guide[((size_t)x << GB) + (u >> (32 - GB))];
        while (k < nthr && row[k] <= u)
            ++k;
        x = k;
        out[i] = symbols[x];
    }
    free(guide);
}
