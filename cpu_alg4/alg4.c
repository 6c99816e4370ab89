/* The paper's fast naive search (Algorithm 4, Sections 2.1-2.3) on the host CPU with
 * AVX2: the CPU baseline the benchmark reports beside the GPU path.
 *
 * Blocks of alpha = 32 consecutive starts.  For a block starting at i, the found
 * mask has bit k set while start i+k is still a candidate.  A compare of pattern
 * position j (SIMDcompare, Section 2.1) loads the 32 text bytes t[i+j .. i+j+31],
 * compares each with p[j] and keeps the bits of the equal ones.  Positions are
 * taken in the compare order pi (Section 2.2); the first r compares run without a
 * test (loop peeling, Section 2.3), each later one only while found is nonzero;
 * the block adds popcount(found).
 *
 * No load reads past t[n-1]: blocks whose loads would are run on a zero-padded
 * copy of the text's end, with the starts past n-m cleared from found, so padding
 * never decides a count.  Blocks are split over OpenMP threads.
 *
 * Not part of the GPU path; nothing there links or calls it. */
#include <immintrin.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t blocks(const uint8_t *t, uint64_t i0, uint64_t i1, uint64_t last, const int32_t *order,
                      const __m256i *rep, uint64_t m, uint32_t r)
{
    /* starts [i0, i1) in blocks of 32; starts past `last` are dead */
    int64_t total = 0;
    for (uint64_t i = i0; i < i1; i += 32) {
        uint32_t found = last >= i + 31 ? 0xFFFFFFFFu : (uint32_t)((1ull << (last - i + 1)) - 1u);
        uint64_t l = 0;
        for (; l < r; ++l) {
            const __m256i w = _mm256_loadu_si256((const __m256i *)(t + i + (uint64_t)order[l]));
            found &= (uint32_t)_mm256_movemask_epi8(_mm256_cmpeq_epi8(w, rep[l]));
        }
        for (; l < m && found; ++l) {
            const __m256i w = _mm256_loadu_si256((const __m256i *)(t + i + (uint64_t)order[l]));
            found &= (uint32_t)_mm256_movemask_epi8(_mm256_cmpeq_epi8(w, rep[l]));
        }
        total += __builtin_popcount(found);
    }
    return total;
}

/* Count of the m-byte pattern p in the n-byte text t (overlapping), comparing positions in
 * `order` (a permutation of 0..m-1) with the first r (1..m) compares peeled.  Returns -1 on
 * bad arguments or memory exhaustion. */
int64_t alg4_avx2_count(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                        uint32_t r, int nthreads)
{
    if (m == 0 || r == 0 || r > m)
        return -1;
    if (m > n)
        return 0;
    __m256i *rep = (__m256i *)aligned_alloc(32, ((m * sizeof(__m256i) + 31) / 32) * 32);
    if (!rep)
        return -1;
    for (uint64_t l = 0; l < m; ++l)
        rep[l] = _mm256_set1_epi8((char)p[order[l]]);
    const uint64_t last = n - m;               /* the last valid start */
    /* blocks whose every load stays inside t: i + 31 + (m - 1) <= n - 1 */
    const uint64_t nsafe = n >= m + 31 ? (n - m - 31) / 32 + 1 : 0;
    int64_t total = 0;
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static) reduction(+ : total)
    for (int64_t b = 0; b < (int64_t)nsafe; b += 256) {
        const uint64_t i0 = (uint64_t)b * 32, i1 = ((uint64_t)b + 256 < nsafe ? (uint64_t)b + 256 : nsafe) * 32;
        total += blocks(t, i0, i1, last, order, rep, m, r);
    }
    /* the remaining starts, on a zero-padded copy of the text's end */
    const uint64_t s0 = nsafe * 32;
    if (s0 <= last) {
        const uint64_t len = n - s0, cap = len + 64;
        uint8_t *tail = (uint8_t *)calloc(cap, 1);
        if (!tail) {
            free(rep);
            return -1;
        }
        memcpy(tail, t + s0, len);
        total += blocks(tail, 0, last - s0 + 1, last - s0, order, rep, m, r);
        free(tail);
    }
    free(rep);
    return total;
}
