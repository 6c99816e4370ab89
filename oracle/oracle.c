/*
 * CPU oracle for exact string matching (Tarhio, Holub and Giaquinta,
 * "Technology Beats Algorithms (in Exact String Matching)", arXiv 1612.01506).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * Conventions: positions are 0-based (the paper is 1-based), every byte value
 * 0..255 is a symbol, counts are 64-bit and include overlapping occurrences.
 *
 * Plain and slow on purpose: each function follows a definition or an
 * algorithm of the paper step by step, with no blocking or reordering beyond
 * what that definition states.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Match test at one start s: Algorithm 1 (Section 2.1).  The inner loop ANDs
 * t[s+j] == p[j] for j = 0..m-1 and leaves at the first mismatch.
 * ---------------------------------------------------------------------- */
static int occurs_at(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t s)
{
    for (uint64_t j = 0; j < m; ++j)
        if (t[s + j] != p[j])
            return 0;
    return 1;
}

/* Count (Section 1 problem statement; Algorithm 1): the number of starts
 * s in [0, n-m] with t[s..s+m-1] == p.  m == 0 is rejected (-1); m > n gives 0
 * because the loop over starts is empty.  The loop over starts is split over
 * nthreads OpenMP threads; each start is tested independently, so the sum is
 * the same for any split. */
int64_t oracle_count(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, int nthreads)
{
    if (m == 0)
        return -1;
    if (m > n)
        return 0;
    if (nthreads < 1)
        nthreads = 1;
    const int64_t last = (int64_t)(n - m);
    uint64_t count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count) num_threads(nthreads)
    for (int64_t s = 0; s <= last; ++s)
        count += (uint64_t)occurs_at(p, m, t, (uint64_t)s);
    return (int64_t)count;
}

/* Report (Section 2.1: the reporting version prints position i where the
 * counting version increments count).  Writes the first min(count, cap)
 * starts in increasing order to pos and returns the full count. */
int64_t oracle_report(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n,
                      uint64_t *pos, uint64_t cap)
{
    if (m == 0)
        return -1;
    if (m > n)
        return 0;
    uint64_t count = 0;
    for (uint64_t s = 0; s + m <= n; ++s) {
        if (occurs_at(p, m, t, s)) {
            if (count < cap)
                pos[count] = s;
            ++count;
        }
    }
    return (int64_t)count;
}

/* Non-overlapping occurrences.  The paper counts every start (Algorithm 1
 * tests each s); a mode that counts only disjoint occurrences is not defined
 * there.  The reading taken: the greedy leftmost selection.  The scan starts
 * at s = 0; an occurrence at s is taken and the scan resumes at s + m,
 * otherwise at s + 1.  Writes the first min(count, cap) taken starts in
 * increasing order and returns the full count. */
int64_t oracle_report_nonoverlap(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n,
                                 uint64_t *pos, uint64_t cap)
{
    if (m == 0)
        return -1;
    if (m > n)
        return 0;
    uint64_t count = 0;
    uint64_t s = 0;
    while (s + m <= n) {
        if (occurs_at(p, m, t, s)) {
            if (count < cap)
                pos[count] = s;
            ++count;
            s += m;
        } else {
            ++s;
        }
    }
    return (int64_t)count;
}

/* Symbol frequencies (Section 2.2): hist[b] = number of s with t[s] == b. */
void oracle_hist(const uint8_t *t, uint64_t n, uint64_t *hist)
{
    memset(hist, 0, 256 * sizeof(uint64_t));
    for (uint64_t s = 0; s < n; ++s)
        hist[t[s]]++;
}

/* Adjacent-pair frequencies: bigram[a * 256 + b] = number of s in [0, n-2]
 * with t[s] == a and t[s+1] == b.  The statistics behind the bigram-aware
 * compare order below. */
void oracle_bigram(const uint8_t *t, uint64_t n, uint64_t *bigram)
{
    memset(bigram, 0, 65536 * sizeof(uint64_t));
    for (uint64_t s = 0; s + 1 < n; ++s)
        bigram[(uint64_t)t[s] * 256 + t[s + 1]]++;
}

/* ------------------------------------------------------------------------
 * Frequency order pi (Section 2.2): pattern positions sorted by the text
 * frequency of their symbol, least frequent first.  The paper leaves ties
 * open; positions with equal frequency keep increasing position order, which
 * makes the key (hist[p[j]], j) unique, so an unstable library sort gives the
 * same permutation.
 * ---------------------------------------------------------------------- */
static const uint8_t *g_sort_p;
static const uint64_t *g_sort_hist;

static int cmp_freq(const void *a, const void *b)
{
    int32_t ja = *(const int32_t *)a, jb = *(const int32_t *)b;
    uint64_t fa = g_sort_hist[g_sort_p[ja]], fb = g_sort_hist[g_sort_p[jb]];
    if (fa != fb)
        return fa < fb ? -1 : 1;
    return ja < jb ? -1 : (ja > jb ? 1 : 0);
}

int oracle_order_freq(const uint8_t *p, uint64_t m, const uint64_t *hist, int32_t *order)
{
    if (m == 0 || m > 0x7fffffffULL)
        return -1;
    for (uint64_t j = 0; j < m; ++j)
        order[j] = (int32_t)j;
    g_sort_p = p;
    g_sort_hist = hist;
    qsort(order, (size_t)m, sizeof(int32_t), cmp_freq);
    return 0;
}

/* Fixed heuristic order pi_h (Section 2.4), written 1-based in the paper as
 * p[1], p[m], p[4], p[7], ..., p[3], p[6], ..., p[2], p[5], ...
 * Reading used here (each position exactly once): first 1, then m, then the
 * positions j = 1 (mod 3) from 4 upward, then j = 0 (mod 3) from 3 upward,
 * then j = 2 (mod 3) from 2 upward, skipping 1 and m everywhere.  Output is
 * 0-based. */
int oracle_order_h(uint64_t m, int32_t *order)
{
    if (m == 0 || m > 0x7fffffffULL)
        return -1;
    uint64_t k = 0;
    order[k++] = 0;
    if (m > 1)
        order[k++] = (int32_t)(m - 1);
    const uint64_t starts[3] = {4, 3, 2};
    for (int c = 0; c < 3; ++c)
        for (uint64_t j = starts[c]; j <= m; j += 3)
            if (j != 1 && j != m)
                order[k++] = (int32_t)(j - 1);
    return k == m ? 0 : -1;
}

/* pi_hs (Section 2.4): the non-space positions in pi_h order, then the space
 * positions (byte 0x20) in pi_h order. */
int oracle_order_hs(const uint8_t *p, uint64_t m, int32_t *order)
{
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    if (!h || oracle_order_h(m, h) != 0) {
        free(h);
        return -1;
    }
    uint64_t k = 0;
    for (uint64_t i = 0; i < m; ++i)
        if (p[h[i]] != 0x20)
            order[k++] = h[i];
    for (uint64_t i = 0; i < m; ++i)
        if (p[h[i]] == 0x20)
            order[k++] = h[i];
    free(h);
    return 0;
}

/* ------------------------------------------------------------------------
 * Bigram-aware compare order.  Section 2.2 notes that ordering by symbol
 * frequency alone compares 'qui' as q, u, i although q, i, u is better, since
 * u nearly always follows q, and points to strategies that compare next the
 * position least likely to match given the positions already compared.  The
 * reading taken, restricted to adjacent pairs: repeatedly pick the position j
 * not yet compared whose estimated match probability e(j) is smallest (ties by
 * position), where
 *   e(j) = bigram[p[j-1]][p[j]] / row(p[j-1])   if only j-1 is compared,
 *          bigram[p[j]][p[j+1]] / col(p[j+1])   if only j+1 is compared,
 *          the smaller of the two                  if both are,
 *          hist[p[j]] / (sum of hist)            if neither is;
 * row(a) and col(b) are the row and column sums of the bigram table, and a
 * zero denominator gives e = 0.  Fractions are compared exactly.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t num, den;
} frac_t;

static int frac_less(frac_t x, frac_t y)
{
    return (unsigned __int128)x.num * y.den < (unsigned __int128)y.num * x.den;
}

static frac_t frac_of(uint64_t num, uint64_t den)
{
    frac_t f = {den ? num : 0, den ? den : 1};
    return f;
}

int oracle_order_bigram(const uint8_t *p, uint64_t m, const uint64_t *hist, const uint64_t *bigram,
                        int32_t *order)
{
    if (m == 0 || m > 0x7fffffffULL)
        return -1;
    uint64_t total = 0, row[256] = {0}, col[256] = {0};
    for (int a = 0; a < 256; ++a)
        total += hist[a];
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) {
            row[a] += bigram[a * 256 + b];
            col[b] += bigram[a * 256 + b];
        }
    unsigned char *done = (unsigned char *)calloc((size_t)m, 1);
    if (!done)
        return -1;
    for (uint64_t k = 0; k < m; ++k) {
        uint64_t best = m;
        frac_t best_e = {0, 1};
        for (uint64_t j = 0; j < m; ++j) {
            if (done[j])
                continue;
            const int left = j > 0 && done[j - 1], right = j + 1 < m && done[j + 1];
            frac_t e;
            if (left || right) {
                frac_t el = {0, 1}, er = {0, 1};
                if (left)
                    el = frac_of(bigram[(uint64_t)p[j - 1] * 256 + p[j]], row[p[j - 1]]);
                if (right)
                    er = frac_of(bigram[(uint64_t)p[j] * 256 + p[j + 1]], col[p[j + 1]]);
                e = !right ? el : !left ? er : (frac_less(er, el) ? er : el);
            } else {
                e = frac_of(hist[p[j]], total);
            }
            if (best == m || frac_less(e, best_e)) {
                best = j;
                best_e = e;
            }
        }
        order[k] = (int32_t)best;
        done[best] = 1;
    }
    free(done);
    return 0;
}

/* ------------------------------------------------------------------------
 * Algorithm 4 (Section 2.3, LP-Freq-SIMD-Naive-search) emulated with a 64-bit
 * found word (alpha = 64), used to check that the compare order pi and the
 * peel factor r leave the result unchanged.
 *
 * SIMDcompare (Section 2.1) for pattern position j at block start i returns
 * the alpha-bit word whose bit k says whether t[i+k+j] == p[j].  Readings for
 * the points the paper leaves open:
 *  - the last block holds fewer than alpha valid starts; bits of starts past
 *    n-m are never set and no byte past t[n-1] is read;
 *  - the first r compares run unconditionally and the first zero test follows
 *    them (r is clamped to m); afterwards found is tested after every compare;
 *  - order == NULL means left to right (Algorithm 2).
 * ---------------------------------------------------------------------- */
static uint64_t simd_compare(const uint8_t *t, uint64_t i, uint64_t nvalid, const uint8_t *p, uint64_t j)
{
    uint64_t mask = 0;
    for (uint64_t k = 0; k < nvalid; ++k)
        if (t[i + k + j] == p[j])
            mask |= 1ULL << k;
    return mask;
}

int64_t oracle_alg4_count(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n,
                          const int32_t *order, uint64_t r)
{
    if (m == 0)
        return -1;
    if (m > n)
        return 0;
    if (r < 1)
        r = 1;
    if (r > m)
        r = m;
    const uint64_t alpha = 64, nstarts = n - m + 1;
    uint64_t count = 0;
    for (uint64_t i = 0; i < nstarts; i += alpha) {
        uint64_t nvalid = nstarts - i < alpha ? nstarts - i : alpha;
        uint64_t found = nvalid == 64 ? ~0ULL : ((1ULL << nvalid) - 1);
        uint64_t l;
        for (l = 0; l < r; ++l) {
            uint64_t j = order ? (uint64_t)order[l] : l;
            found &= simd_compare(t, i, nvalid, p, j);
        }
        if (found == 0)
            continue;
        for (; l < m; ++l) {
            uint64_t j = order ? (uint64_t)order[l] : l;
            found &= simd_compare(t, i, nvalid, p, j);
            if (found == 0)
                break;
        }
        count += (uint64_t)__builtin_popcountll(found);
    }
    return (int64_t)count;
}
