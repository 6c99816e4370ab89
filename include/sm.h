/*
 * sm.h -- C ABI of libsm, exact string matching on AMD Instinct MI355X (gfx950).
 *
 * Method: Tarhio, Holub and Giaquinta, "Technology Beats Algorithms (in Exact
 * String Matching)", arXiv 1612.01506.  The library counts or reports every
 * occurrence (overlapping ones included) of a pattern p of length m in a text
 * t of length n (Section 1 problem statement), comparing pattern symbols in a
 * caller-chosen order pi (Section 2.2) with the first r compares peeled out of
 * the early-exit loop (Section 2.3, Algorithm 4).  The order and r change only
 * the speed: every compare is ANDed into the found mask, so the result is the
 * plain definition of Algorithm 1.
 *
 * Conventions for every call:
 *   - Bytes are uint8_t; every value 0..255 is a symbol; no NUL termination.
 *   - Positions are 0-based start offsets into t (the paper counts from 1).
 *   - Counts are uint64 and include overlapping occurrences ("aaaa"/"aa" = 3).
 *   - "device" pointers are HIP device memory of the current HIP device
 *     (hipMalloc or torch CUDA tensors); "host" pointers are ordinary memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *   - The caller owns every buffer.  The library keeps no caller pointer after
 *     a synchronous call returns, or after the stream work of an asynchronous
 *     call completes.  It owns and reuses its own scratch memory (an upload
 *     ring of pinned host + device memory and per-device scratch), freed by
 *     sm_shutdown().
 *   - Text reads: the kernels load whole 16-byte aligned chunks that overlap
 *     [t, t+n); bytes of such a chunk outside the text are read but never
 *     affect a result (an aligned 16-byte chunk never crosses a page).
 *   - Return values: >= 0 success (a count where stated), < 0 an error code;
 *     sm_last_error() then holds a message (thread-local).
 *
 * Error codes:
 *   SM_EINVAL  null pointer with nonzero length, m == 0, an order that is not
 *              a permutation of 0..m-1, a text pointer that is not device
 *              memory, bad text_id, unknown flag or order kind, m >= 2^32.
 *   SM_ENOMEM  library scratch could not be allocated.
 *   SM_EDEVICE a HIP runtime error (message has the HIP error string).
 * Not errors: n == 0 or m > n (count 0); cap == 0 with pos == NULL (count only).
 */
#ifndef SM_H
#define SM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SM_OK 0
#define SM_EINVAL (-1)
#define SM_ENOMEM (-2)
#define SM_EDEVICE (-3)

/* Compare-order kinds for sm_order(). */
#define SM_ORDER_LTR 0  /* left to right: Algorithm 2 (Section 2.1)                      */
#define SM_ORDER_FREQ 1 /* increasing text frequency, ties by position (Section 2.2)    */
#define SM_ORDER_H 2    /* fixed heuristic order pi_h (Section 2.4)                      */
#define SM_ORDER_HS 3   /* pi_h with space (0x20) positions moved last: pi_hs (Section 2.4) */

/* sm_params.flags: count and report only disjoint occurrences.  The paper
 * counts every start (Section 1, Algorithm 1); this optional mode is not
 * defined there and takes the greedy leftmost selection: the first
 * occurrence, then the first one starting at or after the previous taken
 * start + m, and so on (the convention of Python's bytes.count).  Supported by
 * the synchronous calls sm_count_ex, sm_report_ex and sm_patterns_report;
 * every other call rejects it with SM_EINVAL.  The occurrences are listed in
 * library scratch (about 17 bytes each), so a text with 2^32 - 1 or more
 * occurrences is rejected (SM_EINVAL) and scratch exhaustion gives SM_ENOMEM. */
#define SM_NONOVERLAP 1

/* Count calls (sm_count, sm_count_ex, sm_count_async, sm_patterns_count): compare through per-tile
 * symbol bitmaps when the pattern has at most 4 distinct symbols.  Section 2.1's SIMDcompare of a
 * symbol against every start of a tile is done once per tile and symbol, as one bit per text
 * byte, and each compare of pattern position j is then a shift of those bits by j and an AND over
 * 32 starts.  Faster where compares per start are many (texts over 2 or 3 symbols); the count is
 * the same.  Patterns with more distinct symbols, report calls and batched calls ignore the flag.
 * tile_kib then selects 8, 16 (default) or 32 KiB bitmap tiles; a pattern too long for the tile
 * (its halo of (m - 1) / 32 + 1 words over half the tile) takes the next larger, and above 32 KiB
 * the byte compares.  Also accepted by the calls that take SM_NONOVERLAP (there it is ignored). */
#define SM_BITMAP 2

/* Launch tuning and mode.  Any tuning field 0 selects the library default;
 * none of them changes a result. */
/* Launch tuning of batched calls, per alphabet class of a text: class 0 = at most 2 distinct
 * symbols in its histogram, 1 = at most 4, 2 = at most 32, 3 = more.  0 everywhere = the default.
 * None of these changes a result. */
typedef struct sm_batch_tune {
    int32_t bm_min[4];   /* queries of a text (with a histogram) from which it runs in bitmap mode; default 32 */
    int32_t bm_chunk[4]; /* queries per bitmap work item, 64..1024 (the LDS may hold fewer); default 1024 */
    int32_t peel[4];     /* peel r of batched queries, 1..8; default: from the frequency model */
    int32_t tile_kib;    /* byte-tile batches: 4, 8 or 16 KiB tiles; default 8                       */
    int32_t wgs_per_cu;  /* byte-tile batches, chunks of several queries: 1..32; default 8           */
    int32_t deal_wgs_per_cu; /* single-query chunks (byte and bitmap deals): 1..64; default 16      */
    int32_t pad;
} sm_batch_tune;

/* Launch parameters (NULL, or 0 in a field = the default).  Values outside the ranges below are
 * rejected with SM_EINVAL.  None of them changes a result. */
typedef struct sm_params {
    int32_t peel;       /* r: compares done before the first zero test, 1..8 (Section 2.3); default 2 */
    int32_t tile_kib;   /* text bytes staged per workgroup tile: 4, 8 or 16 KiB; default by n;
                           with SM_BITMAP 8, 16 or 32 KiB, default 16                             */
    int32_t wgs_per_cu; /* workgroups per compute unit the grid is sized for, 1..32; default 6 (8 for batched byte tiles) */
    int32_t flags;      /* SM_NONOVERLAP and/or SM_BITMAP; other bits are rejected (SM_EINVAL)    */
    const sm_batch_tune *batch; /* batched calls: per-class tuning, or NULL; peel, tile_kib and
                                   wgs_per_cu above, when given, take precedence over it         */
} sm_params;

/* ---------------------------------------------------------------- info */

/* Library ABI version (major*10000 + minor*100 + patch). */
int32_t sm_version(void);

/* Message for the last error returned on this thread ("" if none). */
const char *sm_last_error(void);

/* Number of compute units of the current device, or < 0 on error. */
int32_t sm_device_cus(void);

/* Frees the library's scratch and upload ring on every device it used.
 * The caller must make sure no library work is still running. */
int32_t sm_shutdown(void);

/* ------------------------------------------------------ preprocessing */

/* Symbol histogram (Section 2.2: symbol frequencies).  hist_dev: device,
 * 256 x uint64, overwritten with hist[b] = #{s : t[s] == b}.  Asynchronous
 * on `stream`.  t: device, n bytes. */
int32_t sm_histogram(const uint8_t *t, uint64_t n, uint64_t *hist_dev, void *stream);

/* Compare order pi as a permutation of 0..m-1 (host, synchronous).
 *   kind: SM_ORDER_LTR, SM_ORDER_FREQ (Section 2.2; ties keep increasing
 *   position), SM_ORDER_H or SM_ORDER_HS (Section 2.4; the 1-based listing
 *   1, m, 4, 7, ..., 3, 6, ..., 2, 5, ... read with each position once).
 *   p: host, m bytes.  hist_host: host 256 x uint64, required for FREQ only.
 *   order_out: host, m x int32. */
int32_t sm_order(int32_t kind, const uint8_t *p, uint64_t m, const uint64_t *hist_host, int32_t *order_out);

/* Adjacent-pair counts, the statistics of the bigram-aware order below.
 * bigram_dev: device, 65536 x uint64, overwritten with [a * 256 + b] =
 * #{s : t[s] == a, t[s+1] == b}, exactly, in two passes over t (one per
 * half of the first symbol's byte range).  hist_host is accepted for
 * compatibility and ignored: the table never depends on it.
 * Asynchronous on `stream`.  t: device, n bytes. */
int32_t sm_bigram(const uint8_t *t, uint64_t n, const uint64_t *hist_host, uint64_t *bigram_dev, void *stream);

/* Bigram-aware compare order (host, synchronous).  Section 2.2 observes that
 * frequency order compares 'qui' as q, u, i although q, i, u is better, since
 * u nearly always follows q, and mentions comparing next the position least
 * likely to match given those already compared.  On adjacent pairs: the next
 * position is the uncompared one with the smallest estimated match
 * probability -- bigram[a][b] / (row sum of a) from a compared left neighbour
 * a, bigram[a][b] / (column sum of b) from a compared right neighbour b, the
 * smaller of the two when both are compared, else hist[x] / (sum of hist); a
 * zero denominator counts as 0; fractions are compared exactly; ties keep
 * increasing position.  Only the speed depends on the order.
 *   p: host, m bytes.  hist_host: host 256 x uint64.  bigram_host: host
 *   65536 x uint64 as written by sm_bigram.  order_out: host, m x int32. */
int32_t sm_order_bigram(const uint8_t *p, uint64_t m, const uint64_t *hist_host, const uint64_t *bigram_host,
                        int32_t *order_out);

/* ------------------------------------------------------- single search */

/* Count (Section 1; Algorithm 4 of Section 2.3 with pi = order, r = default):
 * the number of s in [0, n-m] with t[s..s+m-1] == p.  Synchronous, null stream.
 *   p: host, m bytes.  t: device, n bytes.
 *   order: host, m x int32 permutation (compare order pi), or NULL = left to right.
 * Returns the count (>= 0) or an error code. */
int64_t sm_count(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order);

/* sm_count with tuning (params may be NULL) on `stream`; synchronous.  With
 * SM_NONOVERLAP in params->flags: the number of disjoint occurrences. */
int64_t sm_count_ex(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                    const sm_params *params, void *stream);

/* Asynchronous count: ADDS the count to *count_dev (device uint64, which the
 * caller zeroes first) on `stream` and returns SM_OK without waiting.  p and
 * order are copied before return. */
int32_t sm_count_async(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                       const sm_params *params, uint64_t *count_dev, void *stream);

/* Report (Section 2.1: the reporting version prints each start found).
 * Writes the min(count, cap) smallest start positions, strictly increasing,
 * to pos_dev (device, cap x uint64) and returns the full count, so a return
 * value > cap means the list was truncated.  Synchronous, null stream. */
int64_t sm_report(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                  uint64_t *pos_dev, uint64_t cap);

/* sm_report with tuning (params may be NULL) on `stream`; synchronous.  With
 * SM_NONOVERLAP: the starts of the disjoint occurrences, and their number. */
int64_t sm_report_ex(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                     const sm_params *params, uint64_t *pos_dev, uint64_t cap, void *stream);

/* Asynchronous report: as sm_report_ex, but the full count is written to
 * *total_dev (device uint64) and the call returns SM_OK without waiting.
 * Reports on one device share the library's report scratch; the library
 * orders them (a report's first kernel waits for the previous report's last
 * one, also across streams). */
int32_t sm_report_async(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                        const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev,
                        void *stream);

/* ---------------------------------------------------- prepared patterns */

/* A set of patterns whose step tables (pattern position and symbol per
 * compare, in compare order pi) are built and copied to the device once, so
 * that later searches issue no host-to-device copy (and can be captured in a
 * HIP graph).  Created and destroyed synchronously on the current device. */
typedef struct sm_patterns sm_patterns;

/* np patterns: p[i] (host, m[i] bytes) with compare order order[i] (host
 * permutation, or NULL = left to right; `order` itself may be NULL).  All
 * patterns are validated before anything is allocated. */
int32_t sm_patterns_create(uint64_t np, const uint8_t *const *p, const uint64_t *m,
                           const int32_t *const *order, sm_patterns **out);

/* As sm_patterns_create, with every compare order computed by the library:
 * kind is an SM_ORDER_* value; hist_host (host 256 x uint64) is required for
 * SM_ORDER_FREQ and ignored otherwise. */
int32_t sm_patterns_create_ordered(uint64_t np, const uint8_t *const *p, const uint64_t *m, int32_t kind,
                                   const uint64_t *hist_host, sm_patterns **out);

int32_t sm_patterns_destroy(sm_patterns *ps);

/* Count of pattern i of the set in t, ADDED to *count_dev (device uint64);
 * asynchronous on `stream`, no host-device copy. */
int32_t sm_patterns_count(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                          const sm_params *params, uint64_t *count_dev, void *stream);

/* Report of pattern i of the set (as sm_report_ex); synchronous on `stream`. */
int64_t sm_patterns_report(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                           const sm_params *params, uint64_t *pos_dev, uint64_t cap, void *stream);

/* Report of pattern i of the set (as sm_report_async); asynchronous, no host-device copy. */
int32_t sm_patterns_report_async(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                                 const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev,
                                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * report as sm_patterns_report_async -- the same kernels, the same positions
 * in pos_dev and full count in total_dev -- with its scratch (per-vector
 * counts, group sums and offsets) in a fixed array of the library's device
 * code instead of library-allocated memory.  The call allocates and frees
 * nothing and issues no host-device copy; it only launches kernels on
 * `stream` (a fill kernel clears the scratch first).  Limit: n - m + 1 <=
 * 1,074,790,385 starts (a 1 GiB text with any pattern); longer texts give
 * SM_EINVAL.  Each device holds its own 4 MiB copy of the array until the
 * process ends.  All calls on one device share that array: calls that
 * overlap on one device (different streams, or threads without ordering)
 * race and give wrong results; calls on one stream are ordered.  The pattern
 * set's creation must have initialised the device (SM_EINVAL after
 * sm_shutdown).  Errors as sm_patterns_report_async. */
int32_t sm_patterns_report_noalloc(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                                   const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev,
                                   void *stream);

/* -------------------------------------------------------------- batches */

typedef struct sm_text {
    const uint8_t *t;      /* device, n bytes                                                  */
    uint64_t n;
    const uint64_t *hist;  /* host 256 x uint64 symbol frequencies, or NULL.  Any values are
                              accepted -- the text's own histogram, one taken from another text
                              of the same kind (Section 2.2), or an estimate: they choose the
                              compare order, the peel and the kernel, never a count           */
} sm_text;

typedef struct sm_query {
    uint32_t text_id;      /* index into the texts array                                       */
    uint32_t flags;        /* must be 0                                                        */
    const uint8_t *p;      /* host, m bytes                                                    */
    uint64_t m;
    const int32_t *order;  /* host permutation, or NULL: frequency order when the text has a
                              histogram, else left to right                                    */
} sm_query;

/* Batched count: counts_dev[i] (device, nq x uint64) is overwritten with the
 * count of query i in its text, exactly as sm_count would return it, for any
 * histogram values (an understated, stale or foreign histogram only costs
 * speed).  The queries run in a few persistent launches, each text tile
 * staged once for all queries that share it: texts with a histogram and at
 * least bm_min queries through per-tile symbol bitmaps, the other queries
 * through byte tiles shared by a text's queries of one m-bucket.  A text's
 * lone query runs as deals (runs of tiles, one record each): of bitmap tiles
 * when the histogram shows at most 4 symbols and the pattern has at most 4
 * distinct symbols, else of byte tiles.  Texts of 64 MiB or more with one or
 * two such queries run them through the single-search kernel.  Validation is
 * all-or-nothing before anything is launched (the message names the first
 * bad query).  Asynchronous on `stream`: host inputs are consumed before
 * return. */
int32_t sm_count_batch(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt,
                       uint64_t *counts_dev, const sm_params *params, void *stream);

/* Batched report (Section 2.1: the reporting version) of many queries in one
 * pass per text and chunk: query i's min(total_i, caps[i]) smallest starts,
 * strictly increasing, go to pos_dev + caps[0] + ... + caps[i-1] (device,
 * caps[0] + ... + caps[nq-1] x uint64), and total_i, its full count, to
 * totals_dev[i] (device, nq x uint64).  The queries of a text share the
 * staged tiles of one launch, which also records each query's per-vector
 * counts; each query's vectors with matches are then searched again and
 * written in order, as in sm_report.  Queries, texts and orders as in
 * sm_count_batch (the bitmap mode is not used).  caps: host, nq x uint64.
 * Asynchronous on `stream`; host inputs are consumed before return.  Library
 * scratch of about 4 bytes per 1024 text bytes per query is shared by all
 * reporting batches on the device, which are ordered by an event. */
int32_t sm_report_batch(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt, const uint64_t *caps,
                        uint64_t *pos_dev, uint64_t *totals_dev, const sm_params *params, void *stream);

/* A planned batch (Section 1 problem statement, one count per query, as
 * sm_count_batch).  sm_batch_create validates and plans the batch exactly as
 * sm_count_batch does and uploads its tables (step tables, tile and query
 * lists) into one device buffer owned by the plan, synchronously on the null
 * stream.  The plan keeps the texts' device addresses and lengths, not their
 * contents: the texts must stay allocated, and may change contents between
 * runs, to any bytes: counts stay exact whatever symbols the texts hold then
 * (the histograms given at creation only chose the compare orders, peels and
 * kernels).  Host inputs (queries,
 * patterns, orders, histograms) are consumed before return.  nq = 0 gives a plan whose runs do nothing.  On error *out
 * is NULL.  The plan belongs to the device current at creation. */
typedef struct sm_batch sm_batch;

int32_t sm_batch_create(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt,
                        const sm_params *params, sm_batch **out);

/* Runs a plan: counts_dev[i] (device, nq x uint64) is overwritten with the
 * count of query i.  Launches kernels on `stream` only: no allocation, no
 * host-device copy and no synchronisation, so the call can be captured in a
 * HIP graph.  Runs of one plan may overlap on different streams only with
 * different counts_dev buffers.  SM_EINVAL if the current device is not the
 * plan's. */
int32_t sm_batch_run(const sm_batch *b, uint64_t *counts_dev, void *stream);

/* Frees the plan's device buffer (synchronous; no run may be pending). NULL is a no-op. */
int32_t sm_batch_destroy(sm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SM_H */
