// C-ABI host side of libsm: validation, compare orders, step tables, the
// upload ring, launch geometry, report scan plumbing and the batch planner.
// The declarations and their contracts are in include/sm.h.
#include "sm.h"
#include "sm_internal.h"

#include <algorithm>
#include <chrono>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <queue>
#include <thread>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

using namespace smk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(SM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define SM_TRY(expr)           \
    do {                       \
        int rc_ = (expr);      \
        if (rc_ < 0)           \
            return rc_;        \
    } while (0)

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t round_up(uint64_t a, uint64_t b) { return ceil_div(a, b) * b; }

// ------------------------------------------------------------------ devices

struct Seg {
    size_t begin, end;
    hipEvent_t ev;
};

// Per-device state.  `mu` serialises every call that touches the ring or the
// scratch buffers, so concurrent host threads are safe; overlapping device
// work on different streams is ordered by the ring's events.
struct Dev {
    int id = -1;
    int cus = 0;
    std::mutex mu;
    // upload ring: pinned host staging + device copy, reused in FIFO order
    uint8_t *rh = nullptr, *rd = nullptr;
    size_t rsize = 0, rhead = 0;
    std::deque<Seg> inflight;
    std::vector<hipEvent_t> evpool;
    // scratch for the synchronous calls
    unsigned long long *u64 = nullptr;  // [0] count, [1] report total
    unsigned long long *hpin = nullptr; // pinned host copy of u64
    uint32_t *bc = nullptr;
    size_t bc_cap = 0;
    unsigned long long *gs = nullptr, *go = nullptr;
    size_t g_cap = 0;
    hipEvent_t rep_ev = nullptr;  // recorded after each report's last kernel
    hipStream_t rep_stream = nullptr;  // ... on this stream
    bool rep_pending = false;
    // bc and gs must be zero when a report's count pass starts; the write pass
    // leaves them zero, so only fresh scratch or an unfinished report needs a fill
    bool rep_dirty = true;
    // non-overlapping mode (synchronous calls only): occurrence list, successor
    // indices, marks and chunk sums in one buffer
    uint8_t *no_buf = nullptr;
    size_t no_cap = 0;
    // reporting batches: per-query vector counts, group sums and offsets
    uint8_t *rb_buf = nullptr;
    size_t rb_cap = 0;
    hipEvent_t rb_ev = nullptr;  // recorded after each reporting batch's last kernel
    hipStream_t rb_stream = nullptr;  // ... on this stream
    bool rb_pending = false;
    // device address of this device's copy of `scratch` (the allocation-free report), or null if
    // the lookup failed at initialisation (that entry point then fails; the others are unaffected)
    uint8_t *na_scratch = nullptr;
};

// Scratch of the allocation-free report (sm_patterns_report_noalloc): the
// per-vector counts (uint32, one per 1024-start vector) of texts up to 1 GiB
// plus the group sums and offsets (uint64, one each per 1024 vectors).  Every
// device holds its own copy until the process ends.  Host code never uses the
// name itself as an address: it takes the device address from
// hipGetSymbolAddress once per device (get_dev) and passes that on.
constexpr uint64_t kNaMaxBlocks = (1ull << 20) + kGroupBlocks;  // 1 GiB text at any alignment, any m
constexpr uint64_t kNaMaxGroups = kNaMaxBlocks / kGroupBlocks;
constexpr uint64_t kNaMaxStarts = kNaMaxBlocks * kBlock - 15;
constexpr size_t kNaBcBytes = kNaMaxBlocks * sizeof(uint32_t);
constexpr size_t kNaBytes = kNaBcBytes + 2 * kNaMaxGroups * sizeof(unsigned long long);
static_assert(kNaBcBytes % 256 == 0, "group sums start 256-byte aligned");
__device__ __align__(256) uint8_t scratch[kNaBytes];

constexpr int kMaxDev = 64;
Dev *g_devs[kMaxDev];
std::mutex g_devs_mu;
constexpr size_t kRingBytes = 64u << 20;

int get_dev(Dev **out)
{
    int id = 0;
    HIP_TRY(hipGetDevice(&id));
    if (id < 0 || id >= kMaxDev)
        return fail(SM_EDEVICE, "device id out of range");
    std::lock_guard<std::mutex> lk(g_devs_mu);
    if (!g_devs[id]) {
        Dev *d = new Dev();
        d->id = id;
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, id);
        if (e == hipSuccess) {
            d->cus = prop.multiProcessorCount;
            d->rsize = kRingBytes;
            e = hipHostMalloc(reinterpret_cast<void **>(&d->rh), d->rsize, hipHostMallocDefault);
        }
        if (e == hipSuccess)  // touch every page once now: first writes to fresh pinned pages are slow
            std::memset(d->rh, 0, d->rsize);
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&d->rd), d->rsize);
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&d->u64), 2 * sizeof(unsigned long long));
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&d->hpin), 2 * sizeof(unsigned long long),
                              hipHostMallocDefault);
        if (e == hipSuccess)
            e = prime_kernel_attrs();
        if (e == hipSuccess) {  // this device's copy of the allocation-free report's scratch
            void *na = nullptr;
            if (hipGetSymbolAddress(&na, HIP_SYMBOL(scratch)) == hipSuccess)
                d->na_scratch = static_cast<uint8_t *>(na);
            else
                (void)hipGetLastError();  // only sm_patterns_report_noalloc depends on it
        }
        if (e != hipSuccess) {
            if (d->rh) (void)hipHostFree(d->rh);
            if (d->rd) (void)hipFree(d->rd);
            if (d->u64) (void)hipFree(d->u64);
            if (d->hpin) (void)hipHostFree(d->hpin);
            delete d;
            return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                        std::string("device init: ") + hipGetErrorString(e));
        }
        g_devs[id] = d;
    }
    *out = g_devs[id];
    return SM_OK;
}

// ------------------------------------------------------------- upload ring

struct Upload {
    uint8_t *host = nullptr;
    uint8_t *dev = nullptr;
    size_t begin = 0, end = 0;
    bool dedicated = false;
};

int release_event(Dev &d, Seg s)
{
    HIP_TRY(hipEventSynchronize(s.ev));
    d.evpool.push_back(s.ev);
    return SM_OK;
}

// Reserve `bytes` of staging.  The caller fills u.host, then calls
// ring_copy_commit after enqueuing every kernel that reads u.dev.
int ring_reserve(Dev &d, size_t bytes, Upload *u)
{
    bytes = round_up(std::max<size_t>(bytes, 1), 256);
    while (!d.inflight.empty() && hipEventQuery(d.inflight.front().ev) == hipSuccess) {
        d.evpool.push_back(d.inflight.front().ev);
        d.inflight.pop_front();
    }
    if (bytes > d.rsize / 2) {
        u->dedicated = true;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&u->host), bytes, hipHostMallocDefault));
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&u->dev), bytes);
        if (e != hipSuccess) {
            (void)hipHostFree(u->host);
            return fail(SM_ENOMEM, std::string("upload buffer: ") + hipGetErrorString(e));
        }
        return SM_OK;
    }
    size_t off = d.rhead;
    if (off + bytes > d.rsize)
        off = 0;
    auto overlaps = [&](const Seg &s) { return s.begin < off + bytes && off < s.end; };
    while (std::any_of(d.inflight.begin(), d.inflight.end(), overlaps)) {
        Seg s = d.inflight.front();
        d.inflight.pop_front();
        SM_TRY(release_event(d, s));
    }
    d.rhead = off + bytes;
    u->host = d.rh + off;
    u->dev = d.rd + off;
    u->begin = off;
    u->end = off + bytes;
    u->dedicated = false;
    return SM_OK;
}

int ring_copy(const Upload &u, size_t bytes, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(u.dev, u.host, bytes, hipMemcpyHostToDevice, s));
    return SM_OK;
}

int ring_commit(Dev &d, Upload &u, hipStream_t s)
{
    if (u.dedicated) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(u.dev));
        HIP_TRY(hipHostFree(u.host));
        u = Upload();
        return SM_OK;
    }
    hipEvent_t ev;
    if (d.evpool.empty()) {
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    } else {
        ev = d.evpool.back();
        d.evpool.pop_back();
    }
    HIP_TRY(hipEventRecord(ev, s));
    d.inflight.push_back({u.begin, u.end, ev});
    return SM_OK;
}

// ------------------------------------------------------------ validation

// The allocation the previous text of one call was found in: texts packed
// into one buffer are then validated without another runtime query.  Scoped
// to a single API call, so a freed and reused range is never trusted.
struct AllocCache {
    uintptr_t base = 0, end = 0;
};

int check_text(const uint8_t *t, uint64_t n, AllocCache *cache = nullptr)
{
    if (n == 0)
        return SM_OK;
    if (!t)
        return fail(SM_EINVAL, "t is NULL with n > 0");
    const uintptr_t a = reinterpret_cast<uintptr_t>(t);
    if (cache && a >= cache->base && a + n >= a && a + n <= cache->end)
        return SM_OK;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, t);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SM_EINVAL, "t is not device memory");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(SM_EINVAL, "t is not device memory");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, reinterpret_cast<hipDeviceptr_t>(const_cast<uint8_t *>(t)));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SM_EINVAL, "t is not inside a device allocation");
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base);
    if (a + n < a || a + n > b + size)
        return fail(SM_EINVAL, "[t, t + n) runs past the end of its device allocation");
    if (cache) {
        cache->base = b;
        cache->end = b + size;
    }
    return SM_OK;
}

int check_pattern(const uint8_t *p, uint64_t m, const int32_t *order)
{
    if (m == 0)
        return fail(SM_EINVAL, "pattern length m must be >= 1");
    if (m >= (1ull << 32))
        return fail(SM_EINVAL, "pattern length m must be < 2^32");
    if (!p)
        return fail(SM_EINVAL, "p is NULL");
    if (order) {
        std::vector<uint8_t> seen(m, 0);
        for (uint64_t l = 0; l < m; ++l) {
            const int64_t j = order[l];
            if (j < 0 || (uint64_t)j >= m || seen[j])
                return fail(SM_EINVAL, "order is not a permutation of 0..m-1");
            seen[j] = 1;
        }
    }
    return SM_OK;
}

// ----------------------------------------------------------------- orders

void order_ltr(uint64_t m, int32_t *o)
{
    for (uint64_t j = 0; j < m; ++j)
        o[j] = (int32_t)j;
}

// Section 2.2: increasing symbol frequency; equal frequencies keep position
// order.  A stable counting sort on frequency ranks: rank[b] orders the
// distinct frequencies (equal frequencies share a rank), so one FreqRanks
// serves every pattern planned against the same histogram.
struct FreqRanks {
    uint16_t rank[256];
    uint32_t nranks = 0;
    explicit FreqRanks(const uint64_t *hist)
    {
        std::vector<uint64_t> v(hist, hist + 256);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        nranks = (uint32_t)v.size();
        for (int b = 0; b < 256; ++b)
            rank[b] = (uint16_t)(std::lower_bound(v.begin(), v.end(), hist[b]) - v.begin());
    }
    void order(const uint8_t *p, uint64_t m, int32_t *o, std::vector<uint32_t> &cnt) const
    {
        cnt.assign(nranks + 1, 0);
        for (uint64_t j = 0; j < m; ++j)
            cnt[rank[p[j]] + 1]++;
        for (uint32_t r = 0; r < nranks; ++r)
            cnt[r + 1] += cnt[r];
        for (uint64_t j = 0; j < m; ++j)
            o[cnt[rank[p[j]]]++] = (int32_t)j;
    }
};

// The same order computed from the pattern's own symbols only: rank the
// distinct symbols of p by frequency (equal frequencies share a rank), then
// the same stable counting sort.  O(m + k log k) for k distinct symbols, so
// it is the cheaper choice when only a few patterns use a histogram.
void order_freq_sparse(const uint64_t *hist, const uint8_t *p, uint64_t m, int32_t *o)
{
    uint16_t rank[256];
    std::fill(rank, rank + 256, (uint16_t)0xFFFF);
    uint64_t key[256];  // frequency in the high bits, symbol in the low 8 when it fits
    uint8_t sym[256];
    uint32_t k = 0;
    uint64_t hmax = 0;
    for (uint64_t j = 0; j < m; ++j)
        if (rank[p[j]] == 0xFFFF) {
            rank[p[j]] = 0;
            sym[k++] = p[j];
            hmax = std::max(hmax, hist[p[j]]);
        }
    if (hmax < (1ull << 56)) {
        for (uint32_t i = 0; i < k; ++i)
            key[i] = (hist[sym[i]] << 8) | sym[i];
        std::sort(key, key + k);
        for (uint32_t i = 0; i < k; ++i)
            sym[i] = (uint8_t)(key[i] & 0xFFu);
    } else {
        std::sort(sym, sym + k, [&](uint8_t a, uint8_t b) { return hist[a] < hist[b]; });
    }
    uint32_t r = 0;
    for (uint32_t i = 0; i < k; ++i) {
        if (i > 0 && hist[sym[i]] != hist[sym[i - 1]])
            ++r;
        rank[sym[i]] = (uint16_t)r;
    }
    const uint32_t nr = k ? r + 1 : 0;
    uint32_t cnt[257];
    std::fill(cnt, cnt + nr + 1, 0u);
    for (uint64_t j = 0; j < m; ++j)
        cnt[rank[p[j]] + 1]++;
    for (uint32_t i = 0; i < nr; ++i)
        cnt[i + 1] += cnt[i];
    for (uint64_t j = 0; j < m; ++j)
        o[cnt[rank[p[j]]]++] = (int32_t)j;
}

// Patterns of at least this total length against one histogram share a FreqRanks.
constexpr uint64_t kRanksMinBytes = 1024;

// Bigram-aware order (the conditional-probability strategy Section 2.2
// discusses, on adjacent pairs): repeatedly compare next the position with
// the smallest estimated match probability given the compared positions --
// the forward conditional bigram[a][b] / row(a) from a compared left
// neighbour a, the backward one bigram[a][b] / col(b) from a compared right
// neighbour b, the smaller when both are compared, else hist[x] / total; a
// zero denominator gives 0.  Exact fraction comparisons, ties by position.
// A heap with per-position versions gives O(m log m).
struct Frac {
    uint64_t num, den;
};

bool frac_lt(Frac x, Frac y)
{
    return (unsigned __int128)x.num * y.den < (unsigned __int128)y.num * x.den;
}

Frac make_frac(uint64_t num, uint64_t den)
{
    return den ? Frac{num, den} : Frac{0, 1};
}

void order_bigram(const uint8_t *p, uint64_t m, const uint64_t *hist, const uint64_t *bigram, int32_t *o)
{
    uint64_t total = 0, row[256] = {}, col[256] = {};
    for (int a = 0; a < 256; ++a)
        total += hist[a];
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) {
            row[a] += bigram[a * 256 + b];
            col[b] += bigram[a * 256 + b];
        }
    std::vector<uint8_t> done(m, 0);
    std::vector<uint32_t> version(m, 0);
    auto estimate = [&](uint64_t j) -> Frac {
        const bool left = j > 0 && done[j - 1], right = j + 1 < m && done[j + 1];
        if (!left && !right)
            return make_frac(hist[p[j]], total);
        Frac el{0, 1}, er{0, 1};
        if (left)
            el = make_frac(bigram[(uint64_t)p[j - 1] * 256 + p[j]], row[p[j - 1]]);
        if (right)
            er = make_frac(bigram[(uint64_t)p[j] * 256 + p[j + 1]], col[p[j + 1]]);
        return !right ? el : !left ? er : (frac_lt(er, el) ? er : el);
    };
    struct Item {
        Frac e;
        uint64_t j;
        uint32_t ver;
    };
    auto after = [](const Item &x, const Item &y) {  // heap order: smallest (e, j) on top
        if (frac_lt(x.e, y.e))
            return false;
        if (frac_lt(y.e, x.e))
            return true;
        return x.j > y.j;
    };
    std::priority_queue<Item, std::vector<Item>, decltype(after)> heap(after);
    for (uint64_t j = 0; j < m; ++j)
        heap.push({estimate(j), j, 0});
    for (uint64_t k = 0; k < m; ++k) {
        Item it = heap.top();
        heap.pop();
        while (done[it.j] || it.ver != version[it.j]) {
            it = heap.top();
            heap.pop();
        }
        o[k] = (int32_t)it.j;
        done[it.j] = 1;
        for (int dj = -1; dj <= 1; dj += 2) {
            const int64_t nj = (int64_t)it.j + dj;
            if (nj < 0 || (uint64_t)nj >= m || done[nj])
                continue;
            heap.push({estimate((uint64_t)nj), (uint64_t)nj, ++version[nj]});
        }
    }
}

// Section 2.4, 1-based listing 1, m, 4, 7, ..., 3, 6, ..., 2, 5, ...: position 1,
// position m, then the residue chains 1, 0, 2 (mod 3) upward from 4, 3, 2,
// each position once.
void order_fixed_h(uint64_t m, int32_t *o)
{
    uint64_t k = 0;
    o[k++] = 0;
    if (m > 1)
        o[k++] = (int32_t)(m - 1);
    const uint64_t from[3] = {4, 3, 2};
    for (uint64_t c = 0; c < 3; ++c)
        for (uint64_t j = from[c]; j <= m; j += 3)
            if (j != m)
                o[k++] = (int32_t)(j - 1);
}

void order_fixed_hs(const uint8_t *p, uint64_t m, int32_t *o)
{
    std::vector<int32_t> h(m);
    order_fixed_h(m, h.data());
    std::stable_partition(h.begin(), h.end(), [&](int32_t j) { return p[j] != 0x20; });
    std::copy(h.begin(), h.end(), o);
}

// Step table for compare order `order` (NULL: left to right).
void build_steps(const uint8_t *p, uint64_t m, const int32_t *order, uint64_t *out)
{
    for (uint64_t l = 0; l < m; ++l) {
        const uint64_t j = order ? (uint64_t)order[l] : l;
        const uint64_t rep = (uint64_t)p[j] * 0x01010101ull;
        out[l] = j | (rep << 32);
    }
    for (uint32_t l = 0; l < kStepPad; ++l)
        out[m + l] = 0;
}

// -------------------------------------------------------------- geometry

// Tiles are dealt to workgroups in chunks of 4 contiguous tiles.
constexpr uint32_t kChunkLog2 = 2;
// Texts (and byte-tile batches whose texts together are) from this size on
// are read with non-temporal tile loads: repeated searches of a 1 GiB text run
// about 8% faster with them, while texts of 128 to 384 MiB, which the 256 MB
// last-level cache partly holds between searches, run faster without.
constexpr uint64_t kStreamLoadBytes = 512ull << 20;

struct Tune {
    int r;
    int cpl;
    int wpc;
    int chunk_log2;
    bool bitmap = false;  // count through symbol bitmaps where the pattern allows (SM_BITMAP)
    int bm_cpw = 2;       // bitmap tile: kWG * bm_cpw words of 32 starts (8 KiB of text per unit)
};

// The distinct symbols of a pattern, up to kBcMaxSyms of them (ns = kBcMaxSyms + 1: more).
struct PatSyms {
    uint32_t packed = 0;  // byte c: symbol of slot c, in order of first appearance
    uint32_t ns = 0;
};

PatSyms pattern_syms(const uint8_t *p, uint64_t m)
{
    // eight pattern bytes at a time: a byte differs from all kept symbols when its high bit stays
    // set in the AND over the symbols of ((v & 0x7F) + 0x7F) | v, v = byte ^ symbol (exact, no
    // carries between bytes); the lowest such byte is the next new symbol
    constexpr uint64_t kOnes = 0x0101010101010101ull, kLow7 = 0x7F7F7F7F7F7F7F7Full, kHigh = 0x8080808080808080ull;
    PatSyms ps;
    if (m == 0)
        return ps;
    uint64_t rep[kBcMaxSyms];
    for (auto &r : rep)
        r = kOnes * p[0];
    ps.packed = p[0];
    ps.ns = 1;
    // the last word ends at byte m - 1 (bytes read twice are already kept); under 8 bytes, the
    // word is padded with the first symbol
    const uint64_t nw = m >= 8 ? (m + 7) / 8 : 1;
    for (uint64_t w = 0; w < nw; ++w) {
        uint64_t x = rep[0];
        if (m < 8)
            for (uint64_t j = 0; j < m; ++j)
                x = (x & ~(0xFFull << (8 * j))) | ((uint64_t)p[j] << (8 * j));
        else
            std::memcpy(&x, p + std::min<uint64_t>(8 * w, m - 8), 8);
        while (true) {
            uint64_t miss = kHigh;
            for (uint32_t c = 0; c < kBcMaxSyms; ++c) {
                const uint64_t v = x ^ rep[c];
                miss &= ((v & kLow7) + kLow7) | v;
            }
            if (!miss)
                break;
            if (ps.ns == kBcMaxSyms) {
                ps.ns = kBcMaxSyms + 1;
                return ps;
            }
            const uint8_t b = (uint8_t)(x >> (__builtin_ctzll(miss) & ~7u));
            ps.packed |= (uint32_t)b << (8 * ps.ns);
            rep[ps.ns++] = kOnes * b;
        }
    }
    return ps;
}

Tune resolve(const sm_params *p, uint64_t m, uint64_t n)
{
    Tune t;
    // p has passed check_flags: every field is 0 (default) or in range
    t.r = (p && p->peel > 0) ? p->peel : 2;
    t.r = (int)std::min<uint64_t>((uint64_t)t.r, m);
    t.bitmap = p && (p->flags & SM_BITMAP);
    if (t.bitmap && p->tile_kib > 0)
        t.bm_cpw = p->tile_kib / 8;
    if (p && p->tile_kib > 0 && !t.bitmap)
        t.cpl = p->tile_kib / 4;
    else
        t.cpl = n >= (8ull << 20) ? 2 : 1;  // 8 KiB tiles measured best on 1 GiB texts
    // 6 workgroups per CU: a full 8 (the occupancy limit) starts every CU's
    // workgroups in lock step and measured ~15% slower on 1 GiB texts.
    t.wpc = (p && p->wgs_per_cu > 0) ? p->wgs_per_cu : 6;
    t.chunk_log2 = kChunkLog2;
    return t;
}

TextView make_view(const uint8_t *t, uint64_t n)
{
    TextView v;
    const uintptr_t a = reinterpret_cast<uintptr_t>(t);
    v.base = reinterpret_cast<const uint8_t *>(a & ~(uintptr_t)15);
    v.first = a & 15u;
    v.n = n;
    v.end16 = round_up(v.first + n, 16);
    return v;
}

uint32_t halo_for(uint64_t m) { return (uint32_t)round_up(m + 4, 16); }

// Bitmap tile words per thread for a pattern of length m: the requested size, doubled
// (up to 4) while the halo words would exceed half the tile; 0 if even that is too small.
int bitmap_cpw(int want, uint64_t m)
{
    const uint64_t h = ((m - 1) >> 5) + 1;
    int cpw = want;
    while (cpw < 4 && h > kWG * (uint64_t)cpw / 2)
        cpw *= 2;
    return h <= kWG * (uint64_t)cpw / 2 ? cpw : 0;
}

// Single search through symbol bitmaps (count only).
int launch_count_bm(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                    const PatSyms &sy, int cpw, unsigned long long *count_dev, hipStream_t s)
{
    BmCountArgs a{};
    a.tv = tv;
    a.last = tv.first + tv.n - m;
    a.steps = steps_dev;
    a.count = count_dev;
    a.m = (uint32_t)m;
    a.r = (uint32_t)tu.r;
    a.syms = sy.packed;
    a.halo_words = (uint32_t)(((m - 1) >> 5) + 1);
    const uint64_t S = 32ull * (kWG * (uint64_t)cpw - a.halo_words);
    a.ntiles = ceil_div(a.last + 1, S);
    const uint64_t target = (uint64_t)std::max(d.cus, 1) * (uint64_t)tu.wpc;
    uint32_t ck = (uint32_t)tu.chunk_log2;
    while (ck > 0 && ceil_div(a.ntiles, 1ull << ck) < target)
        --ck;
    a.chunk_log2 = ck;
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(a.ntiles, 1ull << ck), target));
    HIP_TRY(launch_count_bitmap(a, (int)sy.ns, cpw, tv.n >= kStreamLoadBytes, (unsigned)grid, s));
    return SM_OK;
}

// Fills the geometry of a single search and launches the count kernel.  sy: the
// pattern's distinct symbols, for the bitmap kernel (counts only, SM_BITMAP).
int launch_count(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                 unsigned long long *count_dev, uint32_t *block_counts, unsigned long long *group_sums,
                 hipStream_t s, const PatSyms *sy = nullptr)
{
    if (tu.bitmap && sy && sy->ns >= 1 && sy->ns <= kBcMaxSyms && !block_counts && count_dev)
        if (const int cpw = bitmap_cpw(tu.bm_cpw, m))
            return launch_count_bm(d, tv, m, steps_dev, tu, *sy, cpw, count_dev, s);
    CountArgs a{};
    a.tv = tv;
    a.last = tv.first + tv.n - m;
    a.nblocks = ceil_div(a.last + 1, kBlock);
    a.steps = steps_dev;
    a.m = (uint32_t)m;
    a.count = count_dev;
    a.block_counts = block_counts;
    a.group_sums = group_sums;
    const uint64_t target = (uint64_t)std::max(d.cus, 1) * (uint64_t)tu.wpc;
    int cpl = tu.cpl;
    const uint64_t halo = halo_for(m);
    while (cpl > 1 && 2 * (4096ull * cpl + halo) > kMaxLds)
        cpl >>= 1;
    if (2 * (4096ull * cpl + halo) <= kMaxLds) {
        const uint64_t T = 4096ull * cpl;
        a.halo = (uint32_t)halo;
        a.ntiles = ceil_div(a.last + 1, T);
        // small texts: deal single tiles so that every workgroup gets work
        uint32_t ck = (uint32_t)tu.chunk_log2;
        while (ck > 0 && ceil_div(a.ntiles, 1ull << ck) < target)
            --ck;
        a.chunk_log2 = ck;
        const uint64_t nchunks = ceil_div(a.ntiles, 1ull << a.chunk_log2);
        const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(nchunks, target));
        HIP_TRY(launch_count_staged(a, cpl, tu.r, tv.n >= kStreamLoadBytes, (unsigned)grid, s));
    } else {
        const uint64_t grid = std::min<uint64_t>(ceil_div(a.nblocks, kWaves), target);
        HIP_TRY(launch_count_global(a, tu.r, (unsigned)grid, s));
    }
    return SM_OK;
}

// Uploads the step table of one pattern through the ring.
int upload_steps(Dev &d, const uint8_t *p, uint64_t m, const int32_t *order, hipStream_t s, Upload *u)
{
    const size_t bytes = (m + kStepPad) * sizeof(uint64_t);
    SM_TRY(ring_reserve(d, bytes, u));
    build_steps(p, m, order, reinterpret_cast<uint64_t *>(u->host));
    return ring_copy(*u, bytes, s);
}

// The state of an already initialised device, or null.
Dev *find_dev(int id)
{
    if (id < 0 || id >= kMaxDev)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_devs_mu);
    return g_devs[id];
}

int ensure_report_scratch(Dev &d, uint64_t nblocks, uint64_t ngroups)
{
    if ((d.bc_cap < nblocks || d.g_cap < ngroups) && d.rep_pending)
        HIP_TRY(hipEventSynchronize(d.rep_ev));  // the old buffers may still be in use
    if (d.bc_cap < nblocks) {
        if (d.bc)
            HIP_TRY(hipFree(d.bc));
        d.bc = nullptr;
        d.bc_cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&d.bc), nblocks * sizeof(uint32_t));
        if (e != hipSuccess)
            return fail(SM_ENOMEM, std::string("report scratch: ") + hipGetErrorString(e));
        d.bc_cap = nblocks;
        d.rep_dirty = true;
    }
    if (d.g_cap < ngroups) {
        if (d.gs)
            HIP_TRY(hipFree(d.gs));
        if (d.go)
            HIP_TRY(hipFree(d.go));
        d.gs = d.go = nullptr;
        d.g_cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&d.gs), ngroups * sizeof(unsigned long long));
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&d.go), ngroups * sizeof(unsigned long long));
        if (e != hipSuccess)
            return fail(SM_ENOMEM, std::string("report scratch: ") + hipGetErrorString(e));
        d.g_cap = ngroups;
        d.rep_dirty = true;
    }
    return SM_OK;
}

int check_flags(const sm_params *params, bool nonoverlap_ok);
bool nonoverlap(const sm_params *params);
int64_t nonoverlap_core(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                        uint64_t *pos, uint64_t cap, hipStream_t s);

int64_t count_sync(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                   const sm_params *params, hipStream_t s)
{
    g_err.clear();
    SM_TRY(check_pattern(p, m, order));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, true));
    if (m > n)
        return 0;
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    Upload u;
    SM_TRY(upload_steps(*d, p, m, order, s, &u));
    if (nonoverlap(params)) {
        const int64_t r = nonoverlap_core(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu,
                                          nullptr, 0, s);
        const std::string msg = g_err;
        SM_TRY(ring_commit(*d, u, s));
        return r < 0 ? fail((int)r, msg) : r;
    }
    auto enqueue = [&]() -> int {
        HIP_TRY(hipMemsetAsync(d->u64, 0, sizeof(unsigned long long), s));
        const PatSyms sy = pattern_syms(p, m);
        SM_TRY(launch_count(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu, d->u64, nullptr,
                            nullptr, s, &sy));
        HIP_TRY(hipMemcpyAsync(d->hpin, d->u64, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        return SM_OK;
    };
    const int rc = enqueue();
    const std::string msg = g_err;
    SM_TRY(ring_commit(*d, u, s));  // also after an error: the upload may still be in flight
    if (rc < 0)
        return fail(rc, msg);
    HIP_TRY(hipStreamSynchronize(s));
    return (int64_t)d->hpin[0];
}

// Report with a device step table already in place, in two halves.  The
// count pass writes nonzero per-vector counts and their group sums, then the
// exclusive scan gives group offsets and the total (on the device); the write
// pass searches the vectors with matches again and writes their starts in
// increasing order.  The caller holds d.mu, commits any upload afterwards and
// synchronises `s`.
int report_count_pass(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                      unsigned long long *total_dev, hipStream_t s)
{
    const uint64_t last = tv.first + tv.n - m;
    const uint64_t nblocks = ceil_div(last + 1, kBlock);
    const uint64_t ngroups = ceil_div(nblocks, kGroupBlocks);
    SM_TRY(ensure_report_scratch(d, nblocks, ngroups));
    if (!d.rep_ev)
        HIP_TRY(hipEventCreateWithFlags(&d.rep_ev, hipEventDisableTiming));
    if (d.rep_pending && d.rep_stream != s)  // scratch is shared by all reports (in order on one stream)
        HIP_TRY(hipStreamWaitEvent(s, d.rep_ev, 0));
    if (d.rep_dirty)
        HIP_TRY(launch_fill_report(d.bc, d.bc_cap, d.gs, d.g_cap, s));
    d.rep_dirty = true;  // until a write pass has cleaned up after this count pass
    SM_TRY(launch_count(d, tv, m, steps_dev, tu, nullptr, d.bc, d.gs, s));
    HIP_TRY(launch_scan_groups(d.gs, ngroups, d.go, total_dev, s));
    return SM_OK;
}

// The ordered write of a report whose count pass filled bc and gs and whose scan filled go.
int launch_write(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu, uint32_t *bc,
                 unsigned long long *gs, const unsigned long long *go, uint64_t *pos, uint64_t cap, hipStream_t s)
{
    const uint64_t last = tv.first + tv.n - m;
    const uint64_t nblocks = ceil_div(last + 1, kBlock);
    const uint64_t ngroups = ceil_div(nblocks, kGroupBlocks);
    const uint64_t target = (uint64_t)std::max(d.cus, 1) * (uint64_t)tu.wpc;
    const unsigned ggrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ngroups, target));
    CountArgs a{};
    a.tv = tv;
    a.last = last;
    a.nblocks = nblocks;
    a.steps = steps_dev;
    a.m = (uint32_t)m;
    uint64_t win = kBlock + halo_for(m);
    if (kWaves * win + kGroupBlocks * sizeof(uint32_t) + 64 > kMaxLds)
        win = 0;  // long pattern: read the text from global memory
    HIP_TRY(launch_report_write(a, bc, gs, go, ngroups, reinterpret_cast<unsigned long long *>(pos), cap,
                                (uint32_t)win, ggrid, s));
    return SM_OK;
}

int report_write_pass(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                      uint64_t *pos, uint64_t cap, hipStream_t s)
{
    SM_TRY(launch_write(d, tv, m, steps_dev, tu, d.bc, d.gs, d.go, pos, cap, s));
    HIP_TRY(hipEventRecord(d.rep_ev, s));
    d.rep_stream = s;
    d.rep_pending = true;
    d.rep_dirty = false;
    return SM_OK;
}

int report_core(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu, uint64_t *pos,
                uint64_t cap, unsigned long long *total_dev, hipStream_t s)
{
    SM_TRY(report_count_pass(d, tv, m, steps_dev, tu, total_dev, s));
    return report_write_pass(d, tv, m, steps_dev, tu, pos, cap, s);
}

// report_core on the device's static scratch: the same kernels, no allocation,
// no event, no host-device copy.  The used part of the per-vector counts and
// group sums is cleared first by a fill kernel, since the array keeps whatever
// the previous call on this device left in it.
int report_core_noalloc(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                        uint64_t *pos, uint64_t cap, unsigned long long *total_dev, hipStream_t s)
{
    // at most kNaMaxStarts starts, whatever the text's alignment (tv.first <= 15)
    if (tv.n - m + 1 > kNaMaxStarts)
        return fail(SM_EINVAL, "text too long for the allocation-free report: n - m + 1 = " +
                                   std::to_string(tv.n - m + 1) + " starts, at most " +
                                   std::to_string(kNaMaxStarts) + " are supported");
    const uint64_t nblocks = ceil_div(tv.first + tv.n - m + 1, kBlock);
    const uint64_t ngroups = ceil_div(nblocks, kGroupBlocks);
    if (!d.na_scratch)
        return fail(SM_EDEVICE, "the allocation-free report's scratch has no device address on this device");
    uint32_t *bc = reinterpret_cast<uint32_t *>(d.na_scratch);
    unsigned long long *gs = reinterpret_cast<unsigned long long *>(d.na_scratch + kNaBcBytes);
    unsigned long long *go = gs + kNaMaxGroups;
    HIP_TRY(launch_fill_report(bc, nblocks, gs, ngroups, s));
    SM_TRY(launch_count(d, tv, m, steps_dev, tu, nullptr, bc, gs, s));
    HIP_TRY(launch_scan_groups(gs, ngroups, go, total_dev, s));
    return launch_write(d, tv, m, steps_dev, tu, bc, gs, go, pos, cap, s);
}

// Non-overlapping mode (greedy leftmost disjoint occurrences, see the
// selection kernels): all occurrences are listed in library scratch, the
// taken ones are selected on the device, and the first cap of them are
// written to pos.  Returns the number taken.  Synchronous; the caller holds
// d.mu and commits any upload afterwards.
int64_t nonoverlap_core(Dev &d, const TextView &tv, uint64_t m, const uint64_t *steps_dev, const Tune &tu,
                        uint64_t *pos, uint64_t cap, hipStream_t s)
{
    unsigned long long *tot = d.u64 + 1;
    SM_TRY(report_count_pass(d, tv, m, steps_dev, tu, tot, s));
    HIP_TRY(hipMemcpyAsync(d.hpin + 1, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t c = d.hpin[1];
    if (c == 0) {
        d.rep_dirty = false;  // no vector had a match: the count pass wrote nothing
        return 0;
    }
    if (c >= 0xFFFFFFFFull)
        return fail(SM_EINVAL, "non-overlapping mode supports fewer than 2^32 - 1 occurrences");
    const uint64_t ng = ceil_div(c, kNoChunkEntries);
    const size_t o_pos = 0, o_na = round_up(c * 8, 256), o_nb = o_na + round_up(c * 4, 256),
                 o_mark = o_nb + round_up(c * 4, 256), o_gs = o_mark + round_up(c * 4, 256),
                 o_go = o_gs + round_up(ng * 8, 256), bytes = o_go + round_up(ng * 8, 256);
    if (d.no_cap < bytes) {
        if (d.no_buf)
            HIP_TRY(hipFree(d.no_buf));
        d.no_buf = nullptr;
        d.no_cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&d.no_buf), bytes);
        if (e != hipSuccess)
            return fail(SM_ENOMEM, std::string("non-overlapping scratch: ") + hipGetErrorString(e));
        d.no_cap = bytes;
    }
    unsigned long long *all = reinterpret_cast<unsigned long long *>(d.no_buf + o_pos);
    uint32_t *na = reinterpret_cast<uint32_t *>(d.no_buf + o_na), *nb = reinterpret_cast<uint32_t *>(d.no_buf + o_nb);
    uint32_t *mark = reinterpret_cast<uint32_t *>(d.no_buf + o_mark);
    unsigned long long *gs = reinterpret_cast<unsigned long long *>(d.no_buf + o_gs);
    unsigned long long *go = reinterpret_cast<unsigned long long *>(d.no_buf + o_go);
    SM_TRY(report_write_pass(d, tv, m, steps_dev, tu, reinterpret_cast<uint64_t *>(all), c, s));
    // successors and cluster starts; the longest cluster bounds the doubling rounds
    HIP_TRY(launch_fill_u64(d.u64, 1, 0ull, s));
    HIP_TRY(launch_no_next(all, c, (uint32_t)m, na, mark, d.u64, s));
    HIP_TRY(hipMemcpyAsync(d.hpin, d.u64, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t longest = d.hpin[0] + 1;  // a cluster holds at most every non-start entry plus its start
    for (uint64_t span = 1; span < longest; span <<= 1) {
        HIP_TRY(launch_no_round(na, nb, mark, c, s));
        std::swap(na, nb);
    }
    HIP_TRY(launch_no_chunk_counts(mark, c, gs, ng, s));
    HIP_TRY(launch_scan_groups(gs, ng, go, tot, s));
    if (cap > 0)
        HIP_TRY(launch_no_compact(all, mark, c, go, ng, reinterpret_cast<unsigned long long *>(pos), cap, s));
    HIP_TRY(hipMemcpyAsync(d.hpin + 1, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return (int64_t)d.hpin[1];
}

// sm_params: every field in its documented range (0 = default), SM_NONOVERLAP only where
// `nonoverlap_ok`.
int check_flags(const sm_params *params, bool nonoverlap_ok)
{
    if (!params)
        return SM_OK;
    auto tile_ok = [](int32_t v) { return v == 0 || v == 4 || v == 8 || v == 16; };
    if (params->peel < 0 || params->peel > (int32_t)kMaxPeel)
        return fail(SM_EINVAL, "sm_params.peel must be 0 (default) or 1..8");
    if (params->flags & SM_BITMAP) {
        if (params->tile_kib != 0 && params->tile_kib != 8 && params->tile_kib != 16 && params->tile_kib != 32)
            return fail(SM_EINVAL, "sm_params.tile_kib must be 0 (default), 8, 16 or 32 with SM_BITMAP");
    } else if (!tile_ok(params->tile_kib)) {
        return fail(SM_EINVAL, "sm_params.tile_kib must be 0 (default), 4, 8 or 16");
    }
    if (params->wgs_per_cu < 0 || params->wgs_per_cu > 32)
        return fail(SM_EINVAL, "sm_params.wgs_per_cu must be 0 (default) or 1..32");
    if (const sm_batch_tune *b = params->batch) {
        for (int c = 0; c < 4; ++c) {
            if (b->bm_min[c] < 0)
                return fail(SM_EINVAL, "sm_batch_tune.bm_min must be >= 0");
            if (b->bm_chunk[c] != 0 && (b->bm_chunk[c] < 64 || b->bm_chunk[c] > (int32_t)kBmQChunk))
                return fail(SM_EINVAL, "sm_batch_tune.bm_chunk must be 0 (default) or 64..1024");
            if (b->peel[c] < 0 || b->peel[c] > (int32_t)kMaxPeel)
                return fail(SM_EINVAL, "sm_batch_tune.peel must be 0 (default) or 1..8");
        }
        if (!tile_ok(b->tile_kib))
            return fail(SM_EINVAL, "sm_batch_tune.tile_kib must be 0 (default), 4, 8 or 16");
        if (b->wgs_per_cu < 0 || b->wgs_per_cu > 32 || b->deal_wgs_per_cu < 0 || b->deal_wgs_per_cu > 64)
            return fail(SM_EINVAL, "sm_batch_tune workgroups per CU out of range");
    }
    if (params->flags & ~(int32_t)(SM_NONOVERLAP | SM_BITMAP))
        return fail(SM_EINVAL, "unknown sm_params flags");
    if (!(params->flags & SM_NONOVERLAP))
        return SM_OK;
    if (!nonoverlap_ok)
        return fail(SM_EINVAL, "SM_NONOVERLAP is supported by the synchronous calls only "
                               "(sm_count_ex, sm_report_ex, sm_patterns_report)");
    return SM_OK;
}

bool nonoverlap(const sm_params *params)
{
    return params && (params->flags & SM_NONOVERLAP);
}

int64_t report_sync(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                    const sm_params *params, uint64_t *pos, uint64_t cap, hipStream_t s)
{
    g_err.clear();
    SM_TRY(check_pattern(p, m, order));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, true));
    if (cap > 0 && !pos)
        return fail(SM_EINVAL, "pos is NULL with cap > 0");
    if (m > n)
        return 0;
    if (cap == 0)
        return count_sync(p, m, t, n, order, params, s);
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    Upload u;
    SM_TRY(upload_steps(*d, p, m, order, s, &u));
    if (nonoverlap(params)) {
        const int64_t r = nonoverlap_core(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu,
                                          pos, cap, s);
        const std::string msg = g_err;
        SM_TRY(ring_commit(*d, u, s));
        return r < 0 ? fail((int)r, msg) : r;
    }
    const int rc = report_core(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu, pos, cap,
                               d->u64 + 1, s);
    SM_TRY(ring_commit(*d, u, s));
    SM_TRY(rc);
    HIP_TRY(hipMemcpyAsync(d->hpin + 1, d->u64 + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return (int64_t)d->hpin[1];
}

int report_async(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                 const sm_params *params, uint64_t *pos, uint64_t cap, uint64_t *total_dev, hipStream_t s)
{
    g_err.clear();
    SM_TRY(check_pattern(p, m, order));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, false));
    if (cap > 0 && !pos)
        return fail(SM_EINVAL, "pos is NULL with cap > 0");
    if (!total_dev)
        return fail(SM_EINVAL, "total_dev is NULL");
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(total_dev);
    if (m > n) {
        HIP_TRY(launch_fill_u64(tot, 1, 0ull, s));
        return SM_OK;
    }
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    Upload u;
    SM_TRY(upload_steps(*d, p, m, order, s, &u));
    const int rc = report_core(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu, pos, cap, tot, s);
    SM_TRY(ring_commit(*d, u, s));
    return rc;
}

// ------------------------------------------------------------- batch plan

struct PlanQuery {
    uint64_t idx;     // caller's query index
    uint32_t text;
    uint64_t m;
    uint32_t bucket;  // halo (byte tiles) or pattern-length (bitmaps) bucket
    uint64_t first = 0;  // bitmap queries: symbol << 32 | word of the first compare (sort key)
};

// A text of at least kSoloMinBytes with at most kSoloMaxQueries byte-tile queries runs them
// through the single-search kernel.
constexpr uint64_t kSoloMinBytes = 64ull << 20;
constexpr uint64_t kSoloMaxQueries = 2;

// Workgroups per CU of the single-query deal kernel (about twice the resident number).
constexpr uint64_t kDealsPerCu = 16;

// Reporting batches are split so that one part's per-query scratch stays within this many bytes.
constexpr uint64_t kRepScratchMax = 8ull << 30;

// A text runs in bitmap mode when it has a histogram and at least this many queries.
constexpr uint64_t kBmMinQueries = 32;
// ... and when a work item's LDS holds its bitmaps and the records of at least this many queries.
constexpr uint64_t kBmMinCap = 128;

}  // namespace

namespace {
int validate_batch(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt)
{
    g_err.clear();
    if (!q)
        return fail(SM_EINVAL, "q is NULL");
    if (nq >= (1ull << 32))
        return fail(SM_EINVAL, "too many queries");
    if (nt > 0 && !texts)
        return fail(SM_EINVAL, "texts is NULL");
    AllocCache cache;
    for (uint64_t i = 0; i < nt; ++i) {
        int rc = check_text(texts[i].t, texts[i].n, &cache);
        if (rc < 0)
            return fail(rc, "text " + std::to_string(i) + ": " + g_err);
    }
    for (uint64_t i = 0; i < nq; ++i) {
        if (q[i].text_id >= nt)
            return fail(SM_EINVAL, "query " + std::to_string(i) + ": text_id out of range");
        if (q[i].flags != 0)
            return fail(SM_EINVAL, "query " + std::to_string(i) + ": unknown flags");
        int rc = check_pattern(q[i].p, q[i].m, q[i].order);
        if (rc < 0)
            return fail(rc, "query " + std::to_string(i) + ": " + g_err);
    }
    return SM_OK;
}

// Launch description of a planned batch.  Tables live in one device buffer
// (`dev`) laid out at the offsets below; they hold absolute device addresses
// into that buffer, so a plan is bound to the buffer it was filled for.
struct LaunchPlan {
    size_t bytes = 0;
    bool fill_counts = true;  // launch_plan zeroes counts[0, nq) first (false: the caller did)
    size_t o_items = 0, o_tchunk = 0, o_queries = 0, o_steps = 0, o_bitems = 0, o_bq = 0, o_bout = 0,
           o_smap = 0, o_bsteps = 0, o_reports = 0;  // o_reports: reporting batches only (0: none)
    uint64_t nq = 0;
    // bitmap launch
    uint64_t n_bitems = 0;
    uint32_t bm_lds = 0;  // dynamic LDS bytes: the largest item's bitmaps, symbol map, records and counters
    uint64_t bm_grid = 0;
    bool bm_two = false;  // two workgroups per CU fit the bitmaps' LDS
    // single-query byte-tile chunks: deals
    size_t o_deals = 0, o_solos = 0;
    uint64_t ndeals = 0;
    uint32_t deal_halo = 16;
    uint64_t deal_grid = 0;
    bool deal_stream = false;
    // single-query chunks on texts of at most 4 symbols: bitmap deals
    size_t o_bmdeals = 0, o_bmsolos = 0;
    uint64_t n_bmdeals = 0;
    uint32_t bm_deal_halo = 1;
    uint64_t bm_deal_grid = 0;
    bool bm_deal_stream = false;
    // byte-tile launch
    uint64_t ntiles = 0;
    uint32_t halo_max = 0;
    int cpl = 2;
    uint64_t st_grid = 0;
    // long patterns: one global-kernel search each
    struct Long {
        TextView tv;
        uint64_t m, steps_off, out;
        Tune tu;
        PatSyms sy;  // the pattern's distinct symbols (bitmap compares on small-alphabet texts)
        uint32_t *bc = nullptr;  // reporting: per-vector counts and group sums
        unsigned long long *gs = nullptr;
    };
    std::vector<Long> longs;
    // reporting batches: where each query's step table went
    std::vector<uint64_t> steps_of;  // per caller query index (step-pool index), or ~0 if none
};

// Per-query scratch of a reporting batch (device), indexed by query.
struct ReportScratch {
    std::vector<uint32_t *> bc;
    std::vector<unsigned long long *> gs;
};

// Planning threads: started once and kept, since starting threads on every
// batch call cost more than the per-query work of a few thousand queries.
// run() splits [0, n) into `parts` contiguous ranges; the calling thread and
// the workers take ranges from a shared counter.  One run at a time.
class PlanPool {
public:
    static PlanPool &get()
    {
        static PlanPool pool;
        return pool;
    }
    size_t width() const { return workers_.size() + 1; }
    // body(begin, end); false if a range threw (host memory exhaustion)
    bool run(size_t n, size_t parts, const std::function<void(size_t, size_t)> &body)
    {
        std::lock_guard<std::mutex> one(run_mu_);
        {
            std::lock_guard<std::mutex> lk(mu_);
            body_ = &body;
            n_ = n;
            parts_ = std::max<size_t>(parts, 1);
            next_ = 0;
            done_ = 0;
            adone_.store(0, std::memory_order_relaxed);
            ok_ = true;
            ++gen_;
            agen_.store(gen_, std::memory_order_release);
        }
        cv_.notify_all();
        work();
        // the other parts usually end within microseconds: spin a little before sleeping
        const auto t0 = std::chrono::steady_clock::now();
        while (adone_.load(std::memory_order_acquire) != parts_ && std::chrono::steady_clock::now() - t0 < kSpin)
            std::this_thread::yield();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return done_ == parts_; });
        body_ = nullptr;
        return ok_;
    }

private:
    PlanPool()
    {
        const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
        const size_t nw = std::min<size_t>(kThreads, hw) - 1;
        try {
            for (size_t i = 0; i < nw; ++i)
                workers_.emplace_back([this] { loop(); });
        } catch (...) {  // fewer workers: the calling thread does the rest
        }
    }
    ~PlanPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            astop_.store(true, std::memory_order_release);
        }
        cv_.notify_all();
        for (auto &t : workers_)
            t.join();
    }
    void loop()
    {
        uint64_t seen = 0;
        while (true) {
            // a batch's planning issues several ranges in quick succession: wait for the next one
            // spinning (yielding the core) for a while, then sleeping
            const auto t0 = std::chrono::steady_clock::now();
            while (agen_.load(std::memory_order_acquire) == seen && !astop_.load(std::memory_order_acquire) &&
                   std::chrono::steady_clock::now() - t0 < kSpin)
                std::this_thread::yield();
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_)
                return;
            seen = gen_;
            lk.unlock();
            work();
        }
    }
    void work()
    {
        while (true) {
            size_t p;
            const std::function<void(size_t, size_t)> *body;
            size_t n, parts;
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (!body_ || next_ >= parts_)
                    return;
                p = next_++;
                body = body_;
                n = n_;
                parts = parts_;
            }
            const size_t per = (n + parts - 1) / parts;
            bool good = true;
            try {
                (*body)(std::min(n, p * per), std::min(n, (p + 1) * per));
            } catch (...) {
                good = false;
            }
            std::lock_guard<std::mutex> lk(mu_);
            ok_ = ok_ && good;
            adone_.store(done_ + 1, std::memory_order_release);
            if (++done_ == parts_)
                done_cv_.notify_all();
        }
    }
    static constexpr size_t kThreads = 16;
    static constexpr std::chrono::microseconds kSpin{300};
    std::atomic<uint64_t> agen_{0};   // gen_, readable without the mutex
    std::atomic<size_t> adone_{0};    // done_, likewise
    std::atomic<bool> astop_{false};
    std::vector<std::thread> workers_;
    std::mutex run_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(size_t, size_t)> *body_ = nullptr;
    size_t n_ = 0, parts_ = 0, next_ = 0, done_ = 0;
    uint64_t gen_ = 0;
    bool ok_ = true, stop_ = false;
};

// Runs body(begin, end) over [0, n) in contiguous ranges, on the planning
// threads when n is large enough to pay for them.  Returns false if any range
// threw (host memory exhaustion); the ranges are then incomplete.
constexpr size_t kPlanPerPart = 128;
template <typename F>
bool parallel_for(size_t n, const F &body)
{
    if (n < 2 * kPlanPerPart) {
        try {
            body(0, n);
        } catch (...) {
            return false;
        }
        return true;
    }
    PlanPool &pool = PlanPool::get();
    const std::function<void(size_t, size_t)> fn = [&](size_t b, size_t e) { body(b, e); };
    return pool.run(n, std::min(pool.width() * 4, n / kPlanPerPart), fn);
}

// Peel factor from the text's symbol frequencies.  Section 3 finds r = 2
// best for English, 3 for protein and 5 for DNA; this picks the smallest r
// after which the expected number of the W starts of a vector still alive
// (W times the product of the first r compared symbols' frequencies, in the
// query's compare order) is at most one, capped at 5 and at m.  That gives
// 2, 3 and 5 for large, protein-sized and DNA alphabets.  Speed only.
constexpr uint32_t kModelPeelMax = 5;
uint32_t model_peel(const uint8_t *p, uint64_t m, const int32_t *order, const uint64_t *hist, double hsum, double W)
{
    const uint32_t cap = (uint32_t)std::min<uint64_t>(m, kModelPeelMax);
    double e = W;
    for (uint32_t k = 1; k <= cap; ++k) {
        const uint64_t j = order ? (uint64_t)order[k - 1] : k - 1;
        e *= hsum > 0 ? (double)hist[p[j]] / hsum : 0.0;
        if (e <= 1.0)
            return k;
    }
    return cap;
}

using AllocFn = std::function<int(size_t, uint8_t **, uint8_t **)>;

// Plans a validated batch: classifies the queries (bitmap / byte tiles /
// long), builds every table into host memory obtained from `alloc` (which
// also names the device address the tables will live at) and fills `lp`.
int plan_batch(Dev &d, const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt, const sm_params *params,
               const AllocFn &alloc, LaunchPlan *lp, const ReportScratch *rep = nullptr,
               const uint32_t *out_map = nullptr)
{
    lp->nq = nq;
    // output slot of query i: i, or out_map[i] when the queries are part of a larger batch
    auto out_of = [&](uint64_t i) -> uint32_t { return out_map ? out_map[i] : (uint32_t)i; };
    if (rep)
        lp->steps_of.assign(nq, ~0ull);
    // params has passed check_flags.  Explicit peel / tile / workgroups take precedence over the
    // per-class batch tuning, which takes precedence over the defaults.
    const sm_batch_tune *bt = params ? params->batch : nullptr;
    // (a tile size given with SM_BITMAP is a bitmap tile size, which batches do not use)
    const bool tile_given = params && params->tile_kib > 0 && !(params->flags & SM_BITMAP);
    const int cpl = tile_given ? params->tile_kib / 4 : (bt && bt->tile_kib > 0) ? bt->tile_kib / 4 : 2;
    const uint64_t T = 4096ull * cpl;
    const bool peel_given = params && params->peel > 0;
    const int rdef = peel_given ? params->peel : 2;
    // workgroups per CU: the byte-tile batch kernel measured best at 8 (short per-query work per
    // tile needs more waves in flight); long queries run the single-search kernel, best at 6
    const bool wpc_given = params && params->wgs_per_cu > 0;
    const int wpc = wpc_given ? params->wgs_per_cu : (bt && bt->wgs_per_cu > 0) ? bt->wgs_per_cu : 8;
    const int wpc_long = wpc_given ? wpc : 6;
    const uint64_t deal_wpc = wpc_given ? (uint64_t)wpc : (bt && bt->deal_wgs_per_cu > 0) ? (uint64_t)bt->deal_wgs_per_cu
                                                                                             : kDealsPerCu;
    // alphabet class of a text with a histogram (symbols with a nonzero entry: <= 2, <= 4, <= 32,
    // more) and the histogram's total for the peel model, in one pass over each histogram of a
    // text some query reads
    std::vector<uint8_t> used(nt, 0);
    for (uint64_t i = 0; i < nq; ++i)
        used[q[i].text_id] = 1;
    std::vector<uint8_t> text_cls(nt, 3);
    std::vector<double> hsum(nt, 0.0);
    if (!parallel_for(nt, [&](size_t t0, size_t t1) {
            for (size_t t = t0; t < t1; ++t) {
                const uint64_t *h = texts[t].hist;
                if (!h || !used[t])
                    continue;
                uint32_t nsym = 0;
                uint64_t sum = 0;
                for (int b = 0; b < 256; ++b) {
                    nsym += h[b] != 0;
                    sum += h[b];
                }
                text_cls[t] = nsym <= 2 ? 0 : nsym <= 4 ? 1 : nsym <= 32 ? 2 : 3;
                hsum[t] = (double)sum;
            }
        }))
        return fail(SM_ENOMEM, "batch planning ran out of host memory");
    auto bm_min_of = [&](uint64_t t) -> uint64_t {
        return (bt && bt->bm_min[text_cls[t]] > 0) ? (uint64_t)bt->bm_min[text_cls[t]] : kBmMinQueries;
    };
    auto bm_chunk_of = [&](uint64_t t) -> uint32_t {
        return (bt && bt->bm_chunk[text_cls[t]] > 0) ? (uint32_t)bt->bm_chunk[text_cls[t]] : kBmQChunk;
    };
    const uint64_t target = (uint64_t)std::max(d.cus, 1) * (uint64_t)wpc;
    // two LDS tile buffers of T + halo and the query counters must fit
    const uint64_t max_halo = (kMaxLds - kQChunk * sizeof(uint32_t)) / 2 - T;

    // ---- per-text alphabets (bitmap mode needs the histogram and kBmMinQueries queries)
    auto bm_wps = [](uint64_t m_max) { return (uint32_t)round_up(kBmT / 32 + 2 + ceil_div(m_max, 32), 4); };
    // queries per bitmap work item that fit the LDS beside the bitmaps of `slots` symbols
    auto bm_cap = [](uint32_t slots, uint32_t wps) -> uint64_t {
        const uint64_t fixed = bm_item_lds(slots, wps, 0);
        return fixed >= kBmMaxLds ? 0 : std::min<uint64_t>(kBmQChunk, (kBmMaxLds - fixed) / kBmPerQueryLds);
    };
    auto bm_bucket = [](uint64_t m) -> uint32_t { return m <= 256 ? 256 : (m <= 1024 ? 1024 : 4096); };
    std::vector<uint64_t> nbm(nt, 0);
    for (uint64_t i = 0; i < nq; ++i) {
        const uint32_t t = q[i].text_id;
        if (texts[t].hist && q[i].m <= texts[t].n && q[i].m <= 4096)
            nbm[t]++;
    }
    // symbol -> bitmap slot, texts with enough queries only.  Slots go to the symbols the text's
    // candidate queries use, whatever the histogram says: a text byte of any other symbol can never
    // match, so it sets no bit, and a query symbol the text lacks keeps an all-zero bitmap.  The
    // histogram therefore only steers the compare order and the mode, never a count.
    std::vector<std::vector<uint8_t>> smaps(nt);
    std::vector<uint32_t> nslots(nt, 0);
    for (uint64_t t = 0; t < nt; ++t)
        if (nbm[t] >= bm_min_of(t))
            smaps[t].assign(256, 0);
    for (uint64_t i = 0; i < nq; ++i) {
        const uint32_t t = q[i].text_id;
        if (smaps[t].empty() || q[i].m > texts[t].n || q[i].m > 4096)
            continue;
        uint8_t *seen = smaps[t].data();
        for (uint64_t j = 0; j < q[i].m; ++j)
            seen[q[i].p[j]] = 1;
    }
    for (uint64_t t = 0; t < nt; ++t) {
        if (smaps[t].empty())
            continue;
        for (int b = 0; b < 256; ++b)
            smaps[t][b] = smaps[t][b] ? (uint8_t)nslots[t]++ : (uint8_t)0xFF;
        nbm[t] = 0;
    }
    // a text qualifies if enough of its queries fit the LDS next to their bucket's bitmaps
    for (uint64_t i = 0; i < nq; ++i) {
        const uint32_t t = q[i].text_id;
        if (!smaps[t].empty() && q[i].m <= texts[t].n && q[i].m <= 4096 && nslots[t] > 0 && nslots[t] < 0xFF &&
            bm_cap(nslots[t], bm_wps(bm_bucket(q[i].m))) >= kBmMinCap)
            nbm[t]++;
    }
    std::vector<uint8_t> text_bm(nt, 0);
    std::vector<uint32_t> smap_slot(nt, 0);
    uint32_t n_smaps = 0;
    for (uint64_t t = 0; t < nt; ++t) {
        text_bm[t] = !rep && !smaps[t].empty() && nbm[t] >= bm_min_of(t);  // reports need byte tiles
        if (text_bm[t])
            smap_slot[t] = n_smaps++;
    }

    // byte-tile candidates per text (queries not taken by the bitmap mode)
    std::vector<uint64_t> nstaged(nt, 0);
    for (uint64_t i = 0; i < nq; ++i) {
        const uint32_t t = q[i].text_id;
        if (q[i].m <= texts[t].n &&
            !(text_bm[t] && q[i].m <= 4096 && bm_cap(nslots[t], bm_wps(bm_bucket(q[i].m))) >= kBmMinCap))
            nstaged[t]++;
    }

    // ---- classify queries
    std::vector<PlanQuery> staged, longq, bmq;
    uint64_t total_steps = 0, total_bm_steps = 0;
    for (uint64_t i = 0; i < nq; ++i) {
        const uint32_t t = q[i].text_id;
        const uint64_t n = texts[t].n;
        if (q[i].m > n)
            continue;  // count stays 0
        if (text_bm[t] && q[i].m <= 4096 && bm_cap(nslots[t], bm_wps(bm_bucket(q[i].m))) >= kBmMinCap) {
            bmq.push_back({i, t, q[i].m, bm_bucket(q[i].m)});
            total_bm_steps += q[i].m;
            continue;
        }
        PlanQuery pq{i, t, q[i].m, 0};
        const uint64_t halo = halo_for(q[i].m);
        // queries whose halo is at most T/8 share one chunk per text (one pass over the text, at
        // most 12.5% extra tile reads); longer ones are bucketed by power-of-two halo
        uint64_t b = T / 8;
        while (b < halo)
            b <<= 1;
        pq.bucket = (uint32_t)b;
        // a large text with very few byte-tile queries runs them through the single-search
        // kernel (compile-time peel, one launch each), which is faster than a shared pass there
        const bool solo = texts[t].n >= kSoloMinBytes && nstaged[t] <= kSoloMaxQueries;
        if (halo <= max_halo && !solo)
            staged.push_back(pq);
        else
            longq.push_back(pq);
        total_steps += q[i].m + kStepPad;
    }
    auto by_text_bucket = [](const PlanQuery &a, const PlanQuery &b) {
        return a.text != b.text ? a.text < b.text : a.bucket < b.bucket;
    };
    std::stable_sort(staged.begin(), staged.end(), by_text_bucket);
    // bitmap queries: within a text and bucket, sorted by the symbol and the 32-position word of
    // their first compare, so that the 8 queries run in lock step mostly read the same bitmap words
    // for it (the kernel then loads them once).  The first compare of the frequency order is the
    // first position of the pattern's least frequent symbol; of a given order, its first entry.
    if (!parallel_for(bmq.size(), [&](size_t k0, size_t k1) {
            for (size_t k = k0; k < k1; ++k) {
                const sm_query &Q = q[bmq[k].idx];
                uint64_t j0 = 0;
                if (Q.order) {
                    j0 = (uint64_t)Q.order[0];
                } else {
                    const uint64_t *h = texts[Q.text_id].hist;
                    for (uint64_t j = 1; j < Q.m; ++j)
                        if (h[Q.p[j]] < h[Q.p[j0]])
                            j0 = j;
                }
                bmq[k].first = ((uint64_t)Q.p[j0] << 32) | (j0 >> 5);
            }
        }))
        return fail(SM_ENOMEM, "batch planning ran out of host memory");
    std::stable_sort(bmq.begin(), bmq.end(), [](const PlanQuery &a, const PlanQuery &b) {
        if (a.text != b.text)
            return a.text < b.text;
        return a.bucket != b.bucket ? a.bucket < b.bucket : a.first < b.first;
    });

    struct Chunk {
        uint32_t text;
        uint32_t q0, q1;
        uint64_t m_min, m_max;
    };
    auto make_chunks = [](const std::vector<PlanQuery> &v, const std::function<uint32_t(const PlanQuery &)> &cap_of) {
        std::vector<Chunk> out;
        for (uint32_t i = 0; i < v.size();) {
            uint32_t j = i;
            uint64_t mn = v[i].m, mx = v[i].m;
            const uint32_t cap = cap_of(v[i]);
            while (j < v.size() && j - i < cap && v[j].text == v[i].text && v[j].bucket == v[i].bucket) {
                mn = std::min(mn, v[j].m);
                mx = std::max(mx, v[j].m);
                ++j;
            }
            out.push_back({v[i].text, i, j, mn, mx});
            i = j;
        }
        return out;
    };
    const std::vector<Chunk> chunks = make_chunks(staged, [](const PlanQuery &) { return kQChunk; });
    const std::vector<Chunk> bchunks = make_chunks(bmq, [&](const PlanQuery &pq) {
        return (uint32_t)std::min<uint64_t>(bm_cap(nslots[pq.text], bm_wps(pq.bucket)), bm_chunk_of(pq.text));
    });

    // ---- single-query chunks of counting batches go to deals of up to 2^kChunkLog2 tiles (one
    // record per deal); the rest form one global tile space
    std::vector<uint32_t> solo_q;     // per single-query chunk: its index in `staged`
    std::vector<uint64_t> solo_tiles; // per single-query chunk: its tiles
    std::vector<uint64_t> solo_deal0; // per single-query chunk: its first deal (deals are written later)
    uint64_t ndeals = 0;
    if (!rep) {
        solo_q.reserve(chunks.size());
        solo_tiles.reserve(chunks.size());
        solo_deal0.reserve(chunks.size());
    }
    uint32_t deal_halo = 16;
    uint64_t deal_bytes = 0;
    // single-query chunks on texts whose histogram shows at most 4 symbols, with a pattern of at
    // most 4 distinct symbols and a halo of at most half a tile: bitmap deals (16 KiB bitmap tiles)
    std::vector<uint32_t> bms_q;       // index in `staged`
    std::vector<uint32_t> bms_syms;    // distinct symbols, padded to 4 with the first
    std::vector<uint64_t> bms_tiles, bms_deal0;
    uint64_t n_bmdeals = 0, bm_deal_bytes = 0;
    uint32_t bm_deal_halo = 1;
    // ---- byte-tile chunks in one global tile space
    std::vector<BatchChunk> bchunks_t;
    std::vector<uint32_t> tile_chunk;
    uint32_t halo_max = 16;
    for (auto &c : chunks) {
        if (!rep && c.q1 - c.q0 == 1 && text_cls[c.text] <= 1) {
            const sm_query &Q = q[staged[c.q0].idx];
            const PatSyms sy = pattern_syms(Q.p, Q.m);
            const uint32_t hw = (uint32_t)(((Q.m - 1) >> 5) + 1);
            if (sy.ns <= kBcMaxSyms && hw <= kWG * kBmDealCpw / 2) {
                uint32_t packed = sy.packed;
                for (uint32_t k = sy.ns; k < kBcMaxSyms; ++k)
                    packed |= (sy.packed & 0xFFu) << (8 * k);
                const sm_text &tx = texts[c.text];
                const uint64_t last = (reinterpret_cast<uintptr_t>(tx.t) & 15u) + tx.n - Q.m;
                const uint64_t ntiles = ceil_div(last + 1, 32ull * (kWG * kBmDealCpw - hw));
                if (ntiles >= (1ull << 29))
                    return fail(SM_EINVAL, "batch text too long for a tile index");
                bms_q.push_back(c.q0);
                bms_syms.push_back(packed);
                bms_tiles.push_back(ntiles);
                bms_deal0.push_back(n_bmdeals);
                n_bmdeals += ceil_div(ntiles, 1ull << kChunkLog2);
                bm_deal_halo = std::max(bm_deal_halo, hw);
                bm_deal_bytes += tx.n;
                continue;
            }
        }
        if (!rep && c.q1 - c.q0 == 1) {
            const sm_text &tx = texts[c.text];
            const uint64_t ntiles = ceil_div((reinterpret_cast<uintptr_t>(tx.t) & 15u) + tx.n - c.m_min + 1, T);
            if (ntiles >= (1ull << 29))
                return fail(SM_EINVAL, "batch text too long for a tile index");
            solo_deal0.push_back(ndeals);
            solo_tiles.push_back(ntiles);
            ndeals += ceil_div(ntiles, 1ull << kChunkLog2);
            solo_q.push_back(c.q0);
            deal_halo = std::max(deal_halo, halo_for(c.m_max));
            deal_bytes += ntiles * T;
            continue;
        }
        const sm_text &tx = texts[c.text];
        const TextView tv = make_view(tx.t, tx.n);
        const uint64_t ntiles = ceil_div(tv.first + tx.n - c.m_min + 1, T);
        BatchChunk bc{};
        bc.tv = tv;
        bc.tile0 = tile_chunk.size();
        bc.q_begin = c.q0;
        bc.q_end = c.q1;
        bc.halo = halo_for(c.m_max);
        bc.ntiles = (uint32_t)ntiles;
        halo_max = std::max(halo_max, bc.halo);
        tile_chunk.insert(tile_chunk.end(), ntiles, (uint32_t)bchunks_t.size());
        bchunks_t.push_back(bc);
    }

    // ---- bitmap items
    const uint64_t bm_per_cu_guess = 1;
    const uint64_t bm_grid_target = (uint64_t)std::max(d.cus, 1) * bm_per_cu_guess;
    uint64_t bm_work = 0;
    for (auto &c : bchunks) {
        const uint64_t first = reinterpret_cast<uintptr_t>(texts[c.text].t) & 15u;
        bm_work += ceil_div(first + texts[c.text].n - c.m_min + 1, kBmT);
    }
    const uint64_t bspan = std::max<uint64_t>(1, bm_work / (bm_grid_target * 4));
    std::vector<BmItem> bitems;
    uint64_t bm_lds_max = 0;
    for (auto &c : bchunks) {
        const sm_text &tx = texts[c.text];
        const TextView tv = make_view(tx.t, tx.n);
        const uint64_t ntiles = ceil_div(tv.first + tx.n - c.m_min + 1, kBmT);
        // at most the bucket's bitmap width, which the chunk's capacity was computed for
        const uint32_t wps = bm_wps(c.m_max);
        bm_lds_max = std::max(bm_lds_max, bm_item_lds(nslots[c.text], wps, c.q1 - c.q0));
        for (uint64_t t0 = 0; t0 < ntiles; t0 += bspan) {
            BmItem it{};
            it.tv = tv;
            it.tile_begin = t0;
            it.tile_end = std::min(ntiles, t0 + bspan);
            it.last_min = tv.first + tx.n - c.m_max;
            it.q_begin = c.q0;
            it.q_end = c.q1;
            it.wps = wps;
            it.nslots = nslots[c.text];
            it.smap = nullptr;  // set after upload layout is known
            bitems.push_back(it);
        }
    }

    // ---- one upload: [chunks | tile->chunk | queries | steps | bitmap items | bitmap queries | outs |
    //                   smaps | bitmap steps]
    const size_t o_items = 0;
    const size_t o_tchunk = o_items + round_up(bchunks_t.size() * sizeof(BatchChunk), 256);
    const size_t o_queries = o_tchunk + round_up(tile_chunk.size() * sizeof(uint32_t), 256);
    const size_t o_steps = o_queries + round_up(std::max<size_t>(staged.size(), 1) * sizeof(BatchQuery), 256);
    const size_t o_bitems = o_steps + round_up(total_steps * sizeof(uint64_t), 256);
    const size_t o_bq = o_bitems + round_up(bitems.size() * sizeof(BmItem), 256);
    const size_t o_bout = o_bq + round_up(bmq.size() * kBmRecWords * sizeof(uint32_t), 256);
    const size_t o_smap = o_bout + round_up(bmq.size() * sizeof(uint32_t), 256);
    const size_t o_bsteps = o_smap + round_up((uint64_t)n_smaps * 256, 256);
    if (total_bm_steps >= (1ull << 32))
        return fail(SM_EINVAL, "batch too large: pattern bytes in bitmap mode exceed 2^32");
    const size_t o_reports = o_bsteps + round_up(total_bm_steps * sizeof(uint32_t), 256);
    const size_t o_deals = o_reports + (rep ? round_up(std::max<size_t>(staged.size(), 1) * sizeof(BatchReport), 256) : 0);
    const size_t o_solos = o_deals + round_up(ndeals * sizeof(BatchDeal), 256);
    const size_t o_bmdeals = o_solos + round_up(solo_q.size() * sizeof(BatchSolo), 256);
    const size_t o_bmsolos = o_bmdeals + round_up(n_bmdeals * sizeof(BatchDeal), 256);
    const size_t bytes = o_bmsolos + round_up(bms_q.size() * sizeof(BmSolo), 256);
    uint8_t *uhost = nullptr, *udev = nullptr;
    SM_TRY(alloc(bytes, &uhost, &udev));
    lp->bytes = bytes;
    std::copy(bchunks_t.begin(), bchunks_t.end(), reinterpret_cast<BatchChunk *>(uhost + o_items));
    std::copy(tile_chunk.begin(), tile_chunk.end(), reinterpret_cast<uint32_t *>(uhost + o_tchunk));
    BatchQuery *hq = reinterpret_cast<BatchQuery *>(uhost + o_queries);
    BatchReport *hrep = rep ? reinterpret_cast<BatchReport *>(uhost + o_reports) : nullptr;
    uint64_t *hs = reinterpret_cast<uint64_t *>(uhost + o_steps);
    BmItem *hbi = reinterpret_cast<BmItem *>(uhost + o_bitems);
    uint32_t *hbq = reinterpret_cast<uint32_t *>(uhost + o_bq);
    uint32_t *hbout = reinterpret_cast<uint32_t *>(uhost + o_bout);
    uint8_t *hsm = uhost + o_smap;
    uint32_t *hbs = reinterpret_cast<uint32_t *>(uhost + o_bsteps);
    for (uint64_t t = 0; t < nt; ++t)
        if (text_bm[t])
            std::copy(smaps[t].begin(), smaps[t].end(), hsm + 256 * smap_slot[t]);

    // ---- shared per-text state, prepared before the per-query work is split over threads
    std::vector<std::unique_ptr<FreqRanks>> ranks(nt);
    std::vector<uint64_t> text_bytes(nt, 0);  // pattern bytes per text needing a frequency order
    for (uint64_t i = 0; i < nq; ++i)
        if (!q[i].order && texts[q[i].text_id].hist)
            text_bytes[q[i].text_id] += q[i].m;
    const bool prepared = parallel_for(nt, [&](size_t t0, size_t t1) {
        for (size_t t = t0; t < t1; ++t)
            if (texts[t].hist && text_bytes[t] >= kRanksMinBytes)
                ranks[t].reset(new FreqRanks(texts[t].hist));
    });
    if (!prepared)
        return fail(SM_ENOMEM, "batch planning ran out of host memory");
    // step-table offsets: staged queries, then long ones; bitmap steps separately
    const size_t n_st = staged.size(), n_lg = longq.size(), n_bm = bmq.size();
    std::vector<uint64_t> st_off(n_st + n_lg), bm_off(n_bm);
    std::vector<uint32_t> bm_wps_of(n_bm);
    {
        uint64_t acc = 0;
        for (size_t i = 0; i < n_st + n_lg; ++i) {
            st_off[i] = acc;
            acc += (i < n_st ? staged[i].m : longq[i - n_st].m) + kStepPad;
        }
        acc = 0;
        for (size_t i = 0; i < n_bm; ++i) {
            bm_off[i] = acc;
            acc += bmq[i].m;
        }
        for (auto &c : bchunks)
            for (uint32_t i = c.q0; i < c.q1; ++i)
                bm_wps_of[i] = bm_wps(c.m_max);  // as the chunk's items
    }
    std::vector<uint32_t> long_peel(n_lg);

    // ---- per-query tables: compare order, step entries, peel (independent per query)
    struct Scratch {
        std::vector<int32_t> ord;
        std::vector<uint32_t> cnt;
    };
    auto order_of = [&](uint64_t qi, Scratch &w) -> const int32_t * {
        const sm_query &Q = q[qi];
        if (Q.order)
            return Q.order;
        w.ord.resize(Q.m);
        const uint64_t *h = texts[Q.text_id].hist;
        if (!h)
            order_ltr(Q.m, w.ord.data());
        else if (ranks[Q.text_id])
            ranks[Q.text_id]->order(Q.p, Q.m, w.ord.data(), w.cnt);
        else
            order_freq_sparse(h, Q.p, Q.m, w.ord.data());
        return w.ord.data();
    };
    // peel of a query: the caller's, else the frequency model when the text has a histogram, else 2
    auto peel_of = [&](uint64_t qi, const int32_t *o, double W) -> uint32_t {
        const sm_query &Q = q[qi];
        const uint64_t *h = texts[Q.text_id].hist;
        if (peel_given || !h)
            return (uint32_t)std::min<uint64_t>((uint64_t)rdef, Q.m);
        if (bt && bt->peel[text_cls[Q.text_id]] > 0)
            return (uint32_t)std::min<uint64_t>((uint64_t)bt->peel[text_cls[Q.text_id]], Q.m);
        return model_peel(Q.p, Q.m, o, h, hsum[Q.text_id], W);
    };
    auto fill = [&](size_t k, Scratch &w) {
        if (k < n_st + n_lg) {
            const PlanQuery &pq = k < n_st ? staged[k] : longq[k - n_st];
            const sm_query &Q = q[pq.idx];
            const int32_t *o = order_of(pq.idx, w);
            build_steps(Q.p, Q.m, o, hs + st_off[k]);
            const uint32_t r = peel_of(pq.idx, o, (double)kBlock);
            if (rep)
                lp->steps_of[pq.idx] = st_off[k];
            if (k >= n_st) {
                long_peel[k - n_st] = r;
                return;
            }
            const sm_text &tx = texts[pq.text];
            BatchQuery bq{};
            bq.steps_off = st_off[k];
            bq.last = (reinterpret_cast<uintptr_t>(tx.t) & 15u) + tx.n - pq.m;
            bq.m = (uint32_t)pq.m;
            bq.r = r;
            bq.out = out_of(pq.idx);
            hq[k] = bq;
            if (rep)
                hrep[k] = BatchReport{rep->bc[pq.idx], rep->gs[pq.idx]};
            return;
        }
        const size_t i = k - n_st - n_lg;
        const PlanQuery &pq = bmq[i];
        const sm_query &Q = q[pq.idx];
        const int32_t *o = order_of(pq.idx, w);
        const uint32_t wps = bm_wps_of[i];
        uint32_t *e = hbs + bm_off[i];
        for (uint64_t l = 0; l < Q.m; ++l) {
            const uint32_t j = (uint32_t)o[l];
            const uint32_t slot = smaps[pq.text][Q.p[j]];
            e[l] = ((slot * wps + (j >> 5)) << 7) | (j & 31u);
        }
        // record: m | r << 24, the step table's index, its first entries (past m: entry m - 1)
        uint32_t *rq = hbq + (size_t)i * kBmRecWords;
        rq[0] = (uint32_t)pq.m | (peel_of(pq.idx, o, (double)kBmT) << 24);
        rq[1] = (uint32_t)bm_off[i];
        for (uint32_t l = 0; l < kBmRecSteps; ++l)
            rq[2 + l] = e[std::min<uint64_t>(l, Q.m - 1)];
        hbout[i] = out_of(pq.idx);
    };
    const bool planned = parallel_for(n_st + n_lg + n_bm, [&](size_t k0, size_t k1) {
        Scratch w;
        for (size_t k = k0; k < k1; ++k)
            fill(k, w);
    });
    if (!planned)
        return fail(SM_ENOMEM, "batch planning ran out of host memory");
    std::vector<uint64_t> long_steps_off(st_off.begin() + n_st, st_off.end());
    {
        // each single-query chunk's deals (runs of up to 2^kChunkLog2 of its tiles) and its record
        BatchDeal *hdeal = reinterpret_cast<BatchDeal *>(uhost + o_deals);
        BatchSolo *hso = reinterpret_cast<BatchSolo *>(uhost + o_solos);
        const bool filled = parallel_for(solo_q.size(), [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const BatchQuery &bq = hq[solo_q[i]];
                const PlanQuery &pq = staged[solo_q[i]];
                BatchSolo S{};
                S.tv = make_view(texts[pq.text].t, texts[pq.text].n);
                S.last = bq.last;
                S.steps = reinterpret_cast<const uint64_t *>(udev + o_steps) + bq.steps_off;
                S.halo = halo_for(pq.m);
                S.m = bq.m;
                S.r = bq.r;
                S.out = bq.out;
                hso[i] = S;
                BatchDeal *dp = hdeal + solo_deal0[i];
                for (uint64_t k0 = 0; k0 < solo_tiles[i]; k0 += 1ull << kChunkLog2)
                    *dp++ = {(uint32_t)i,
                             (uint32_t)(k0 << 3) | (uint32_t)std::min<uint64_t>(solo_tiles[i] - k0, 1ull << kChunkLog2)};
            }
        });
        if (!filled)
            return fail(SM_ENOMEM, "batch planning ran out of host memory");
        BatchDeal *hbd = reinterpret_cast<BatchDeal *>(uhost + o_bmdeals);
        BmSolo *hbms = reinterpret_cast<BmSolo *>(uhost + o_bmsolos);
        const bool bfilled = parallel_for(bms_q.size(), [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const BatchQuery &bq = hq[bms_q[i]];
                const PlanQuery &pq = staged[bms_q[i]];
                BmSolo S{};
                S.tv = make_view(texts[pq.text].t, texts[pq.text].n);
                S.last = bq.last;
                S.steps = reinterpret_cast<const uint64_t *>(udev + o_steps) + bq.steps_off;
                S.m = bq.m;
                S.r = bq.r;
                S.syms = bms_syms[i];
                S.halo_words = (uint32_t)(((pq.m - 1) >> 5) + 1);
                S.out = bq.out;
                hbms[i] = S;
                BatchDeal *dp = hbd + bms_deal0[i];
                for (uint64_t k0 = 0; k0 < bms_tiles[i]; k0 += 1ull << kChunkLog2)
                    *dp++ = {(uint32_t)i,
                             (uint32_t)(k0 << 3) | (uint32_t)std::min<uint64_t>(bms_tiles[i] - k0, 1ull << kChunkLog2)};
            }
        });
        if (!bfilled)
            return fail(SM_ENOMEM, "batch planning ran out of host memory");
    }
    {
        size_t k = 0;
        for (auto &c : bchunks) {
            const uint64_t first = reinterpret_cast<uintptr_t>(texts[c.text].t) & 15u;
            const uint64_t ntiles = ceil_div(first + texts[c.text].n - c.m_min + 1, kBmT);
            for (uint64_t t0 = 0; t0 < ntiles; t0 += bspan) {
                bitems[k].smap = udev + o_smap + 256 * smap_slot[c.text];
                ++k;
            }
        }
        std::copy(bitems.begin(), bitems.end(), hbi);
    }
    lp->o_items = o_items;
    lp->o_tchunk = o_tchunk;
    lp->o_queries = o_queries;
    lp->o_steps = o_steps;
    lp->o_bitems = o_bitems;
    lp->o_bq = o_bq;
    lp->o_bout = o_bout;
    lp->o_smap = o_smap;
    lp->o_bsteps = o_bsteps;
    lp->o_reports = rep ? o_reports : 0;
    lp->n_bitems = bitems.size();
    lp->bm_lds = (uint32_t)bm_lds_max;
    {
        const uint64_t per_cu = std::max<uint64_t>(1, kBmMaxLds / std::max<uint64_t>(bm_lds_max, 1));
        lp->bm_two = per_cu >= 2;
        lp->bm_grid = std::min<uint64_t>(bitems.size(), (uint64_t)std::max(d.cus, 1) * std::min<uint64_t>(per_cu, 2));
    }
    lp->ntiles = tile_chunk.size();
    lp->halo_max = halo_max;
    lp->cpl = cpl;
    lp->st_grid = std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(tile_chunk.size(), 1ull << kChunkLog2), target));
    lp->o_deals = o_deals;
    lp->o_solos = o_solos;
    lp->ndeals = ndeals;
    lp->deal_halo = deal_halo;
    // deals differ in length (texts' last deals are partial): twice the resident workgroups, dealt
    // round robin, let the ones that finish early take over the rest (measured 0.58 -> 0.51 ms on
    // 4,096 texts of 4 KiB - 4 MiB)
    lp->deal_grid = std::max<uint64_t>(
        1, std::min<uint64_t>(ndeals, (uint64_t)std::max(d.cus, 1) * deal_wpc));
    lp->deal_stream = deal_bytes >= kStreamLoadBytes;
    lp->o_bmdeals = o_bmdeals;
    lp->o_bmsolos = o_bmsolos;
    lp->n_bmdeals = n_bmdeals;
    lp->bm_deal_halo = bm_deal_halo;
    lp->bm_deal_grid = std::max<uint64_t>(1, std::min<uint64_t>(n_bmdeals, (uint64_t)std::max(d.cus, 1) * deal_wpc));
    lp->bm_deal_stream = bm_deal_bytes >= kStreamLoadBytes;
    for (size_t i = 0; i < longq.size(); ++i) {
        const PlanQuery &pq = longq[i];
        LaunchPlan::Long L;
        L.tv = make_view(texts[pq.text].t, texts[pq.text].n);
        L.m = pq.m;
        L.steps_off = long_steps_off[i];
        L.out = out_of(pq.idx);
        // long patterns: 4 KiB tiles (room for the halo); solo queries: the single-search tile
        const bool fits8 = 2 * (8192 + halo_for(pq.m)) <= kMaxLds;
        L.tu = Tune{(int)long_peel[i], (texts[pq.text].n >= (8ull << 20) && fits8) ? 2 : 1, wpc_long,
                    (int)kChunkLog2};
        // a counted query on a text whose histogram shows at most 4 symbols takes the bitmap
        // compares (32 KiB tiles, 6 workgroups per CU: the single-search tuning's choice on 1 GiB
        // texts of 2 and 4 symbols); the pattern's own symbols decide whether it can
        if (!rep && text_cls[pq.text] <= 1 && !wpc_given) {
            L.tu.bitmap = true;
            L.tu.bm_cpw = 4;
            L.tu.wpc = 6;
            L.sy = pattern_syms(q[pq.idx].p, pq.m);
        }
        if (rep) {
            L.bc = rep->bc[pq.idx];
            L.gs = rep->gs[pq.idx];
        }
        lp->longs.push_back(L);
    }
    return SM_OK;
}

// Zeroes the counts and launches the planned kernels; no host-device copy
// and no allocation, so it can be captured in a graph.
int launch_plan(Dev &d, const LaunchPlan &lp, const uint8_t *dev, unsigned long long *counts, hipStream_t s)
{
    if (lp.fill_counts)
        HIP_TRY(launch_fill_u64(counts, lp.nq, 0ull, s));
    if (lp.n_bitems) {
        BmArgs a{};
        a.items = reinterpret_cast<const BmItem *>(dev + lp.o_bitems);
        a.nitems = lp.n_bitems;
        a.recs = reinterpret_cast<const uint32_t *>(dev + lp.o_bq);
        a.outs = reinterpret_cast<const uint32_t *>(dev + lp.o_bout);
        a.steps = reinterpret_cast<const uint32_t *>(dev + lp.o_bsteps);
        a.counts = counts;
        HIP_TRY(launch_batch_bitmap(a, (unsigned)lp.bm_grid, lp.bm_lds, lp.bm_two, s));
    }
    if (lp.ndeals) {
        DealArgs a{};
        a.deals = reinterpret_cast<const BatchDeal *>(dev + lp.o_deals);
        a.solos = reinterpret_cast<const BatchSolo *>(dev + lp.o_solos);
        a.ndeals = lp.ndeals;
        a.counts = counts;
        a.halo_max = lp.deal_halo;
        HIP_TRY(launch_batch_deals(a, lp.cpl, lp.deal_stream, (unsigned)lp.deal_grid, s));
    }
    if (lp.n_bmdeals) {
        BmDealArgs a{};
        a.deals = reinterpret_cast<const BatchDeal *>(dev + lp.o_bmdeals);
        a.solos = reinterpret_cast<const BmSolo *>(dev + lp.o_bmsolos);
        a.ndeals = lp.n_bmdeals;
        a.counts = counts;
        HIP_TRY(launch_bm_deals(a, lp.bm_deal_halo, lp.bm_deal_stream, (unsigned)lp.bm_deal_grid, s));
    }
    if (lp.ntiles) {
        BatchArgs a{};
        a.chunks = reinterpret_cast<const BatchChunk *>(dev + lp.o_items);
        a.tile_chunk = reinterpret_cast<const uint32_t *>(dev + lp.o_tchunk);
        a.ntiles = lp.ntiles;
        a.queries = reinterpret_cast<const BatchQuery *>(dev + lp.o_queries);
        a.reports = lp.o_reports ? reinterpret_cast<const BatchReport *>(dev + lp.o_reports) : nullptr;
        a.steps = reinterpret_cast<const uint64_t *>(dev + lp.o_steps);
        a.counts = counts;
        a.halo_max = lp.halo_max;
        a.chunk_log2 = kChunkLog2;
        // the plan's tiles hold all its texts once: stream them when they far exceed the cache
        const bool stream_loads = lp.ntiles * (4096ull * (uint64_t)lp.cpl) >= kStreamLoadBytes;
        HIP_TRY(launch_batch_staged(a, lp.cpl, stream_loads, (unsigned)lp.st_grid, s));
    }
    for (const auto &L : lp.longs)
        SM_TRY(launch_count(d, L.tv, L.m, reinterpret_cast<const uint64_t *>(dev + lp.o_steps) + L.steps_off, L.tu,
                            counts + L.out, L.bc, L.gs, s, &L.sy));
    return SM_OK;
}

}  // namespace

// A planned batch: tables in one plan-owned device buffer.
struct sm_batch {
    int dev = -1;
    uint8_t *buf = nullptr;
    LaunchPlan lp;
};

// A prepared pattern set: step tables of all patterns in one device buffer.
struct sm_patterns {
    int dev = -1;
    uint64_t *steps = nullptr;
    std::vector<uint64_t> off, m;
    std::vector<PatSyms> syms;  // distinct symbols, for bitmap counts
};

namespace {
int check_set(const sm_patterns *ps, uint64_t i)
{
    if (!ps)
        return fail(SM_EINVAL, "pattern set is NULL");
    if (i >= ps->m.size())
        return fail(SM_EINVAL, "pattern index out of range");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != ps->dev)
        return fail(SM_EINVAL, "pattern set belongs to another device");
    return SM_OK;
}
}  // namespace

// ======================================================================= C ABI

extern "C" {

int32_t sm_version(void) { return 10200; }

const char *sm_last_error(void) { return g_err.c_str(); }

int32_t sm_device_cus(void)
{
    g_err.clear();
    Dev *d;
    SM_TRY(get_dev(&d));
    return d->cus;
}

int32_t sm_shutdown(void)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_devs_mu);
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    for (int i = 0; i < kMaxDev; ++i) {
        Dev *d = g_devs[i];
        if (!d)
            continue;
        HIP_TRY(hipSetDevice(i));
        HIP_TRY(hipDeviceSynchronize());
        for (auto &s : d->inflight)
            (void)hipEventDestroy(s.ev);
        for (auto ev : d->evpool)
            (void)hipEventDestroy(ev);
        (void)hipHostFree(d->rh);
        (void)hipFree(d->rd);
        (void)hipFree(d->u64);
        (void)hipHostFree(d->hpin);
        if (d->bc) (void)hipFree(d->bc);
        if (d->gs) (void)hipFree(d->gs);
        if (d->go) (void)hipFree(d->go);
        if (d->rep_ev) (void)hipEventDestroy(d->rep_ev);
        if (d->no_buf) (void)hipFree(d->no_buf);
        if (d->rb_buf) (void)hipFree(d->rb_buf);
        if (d->rb_ev) (void)hipEventDestroy(d->rb_ev);
        delete d;
        g_devs[i] = nullptr;
    }
    HIP_TRY(hipSetDevice(cur));
    return SM_OK;
}

int32_t sm_histogram(const uint8_t *t, uint64_t n, uint64_t *hist_dev, void *stream)
{
    g_err.clear();
    if (!hist_dev)
        return fail(SM_EINVAL, "hist_dev is NULL");
    SM_TRY(check_text(t, n));
    Dev *d;
    SM_TRY(get_dev(&d));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *h = reinterpret_cast<unsigned long long *>(hist_dev);
    HIP_TRY(launch_fill_u64(h, 256, 0ull, s));
    if (n == 0)
        return SM_OK;
    const TextView tv = make_view(t, n);
    const uint64_t nchunks = tv.end16 / 16;
    // two 64 KiB workgroups fit a compute unit's LDS
    const uint64_t grid =
        std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(nchunks, kHistWG), (uint64_t)std::max(d->cus, 1) * 2));
    HIP_TRY(launch_hist(tv, h, n >= kStreamLoadBytes, (unsigned)grid, s));
    return SM_OK;
}

int32_t sm_bigram(const uint8_t *t, uint64_t n, const uint64_t *hist_host, uint64_t *bigram_dev, void *stream)
{
    g_err.clear();
    SM_TRY(check_text(t, n));
    if (!bigram_dev)
        return fail(SM_EINVAL, "bigram_dev is NULL");
    Dev *d;
    SM_TRY(get_dev(&d));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *out = reinterpret_cast<unsigned long long *>(bigram_dev);
    HIP_TRY(launch_fill_u64(out, 65536, 0ull, s));
    if (n < 2)
        return SM_OK;
    const TextView tv = make_view(t, n);
    const uint64_t nchunks = tv.end16 / 16;
    const unsigned grid =
        (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(nchunks, kBgWG), (uint64_t)std::max(d->cus, 1)));
    // Both halves always run: a pass whose first symbols do not occur adds nothing, and skipping it
    // on the strength of a caller's histogram would make the table depend on that histogram.
    (void)hist_host;
    for (uint32_t half = 0; half < 2; ++half)
        HIP_TRY(launch_bigram(tv, half, out, grid, s));
    return SM_OK;
}

int32_t sm_order_bigram(const uint8_t *p, uint64_t m, const uint64_t *hist_host, const uint64_t *bigram_host,
                        int32_t *order_out)
{
    g_err.clear();
    if (m == 0 || m >= (1ull << 31))
        return fail(SM_EINVAL, "pattern length m must be in 1..2^31-1");
    if (!p || !order_out || !hist_host || !bigram_host)
        return fail(SM_EINVAL, "p, hist_host, bigram_host and order_out must not be NULL");
    try {
        order_bigram(p, m, hist_host, bigram_host, order_out);
    } catch (const std::bad_alloc &) {
        return fail(SM_ENOMEM, "bigram order: out of host memory");
    }
    return SM_OK;
}

int32_t sm_order(int32_t kind, const uint8_t *p, uint64_t m, const uint64_t *hist_host, int32_t *order_out)
{
    g_err.clear();
    if (m == 0 || m >= (1ull << 31))
        return fail(SM_EINVAL, "pattern length m must be in 1..2^31-1");
    if (!order_out)
        return fail(SM_EINVAL, "order_out is NULL");
    if (kind != SM_ORDER_LTR && kind != SM_ORDER_H && !p)
        return fail(SM_EINVAL, "p is NULL");
    switch (kind) {
    case SM_ORDER_LTR: order_ltr(m, order_out); return SM_OK;
    case SM_ORDER_FREQ: {
        if (!hist_host)
            return fail(SM_EINVAL, "SM_ORDER_FREQ needs hist_host");
        if (m >= kRanksMinBytes) {
            std::vector<uint32_t> cnt;
            FreqRanks(hist_host).order(p, m, order_out, cnt);
        } else {
            order_freq_sparse(hist_host, p, m, order_out);
        }
        return SM_OK;
    }
    case SM_ORDER_H: order_fixed_h(m, order_out); return SM_OK;
    case SM_ORDER_HS: order_fixed_hs(p, m, order_out); return SM_OK;
    default: return fail(SM_EINVAL, "unknown order kind");
    }
}

int64_t sm_count(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order)
{
    return count_sync(p, m, t, n, order, nullptr, nullptr);
}

int64_t sm_count_ex(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                    const sm_params *params, void *stream)
{
    return count_sync(p, m, t, n, order, params, reinterpret_cast<hipStream_t>(stream));
}

int32_t sm_count_async(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                       const sm_params *params, uint64_t *count_dev, void *stream)
{
    g_err.clear();
    SM_TRY(check_pattern(p, m, order));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, false));
    if (!count_dev)
        return fail(SM_EINVAL, "count_dev is NULL");
    if (m > n)
        return SM_OK;
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Tune tu = resolve(params, m, n);
    Upload u;
    SM_TRY(upload_steps(*d, p, m, order, s, &u));
    const PatSyms sy = pattern_syms(p, m);
    const int rc = launch_count(*d, make_view(t, n), m, reinterpret_cast<const uint64_t *>(u.dev), tu,
                                reinterpret_cast<unsigned long long *>(count_dev), nullptr, nullptr, s, &sy);
    const std::string msg = g_err;
    const int rc2 = ring_commit(*d, u, s);  // also after an error: the upload may still be in flight
    return rc < 0 ? fail(rc, msg) : rc2;
}

int64_t sm_report(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                  uint64_t *pos_dev, uint64_t cap)
{
    return report_sync(p, m, t, n, order, nullptr, pos_dev, cap, nullptr);
}

int64_t sm_report_ex(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                     const sm_params *params, uint64_t *pos_dev, uint64_t cap, void *stream)
{
    return report_sync(p, m, t, n, order, params, pos_dev, cap, reinterpret_cast<hipStream_t>(stream));
}

int32_t sm_report_async(const uint8_t *p, uint64_t m, const uint8_t *t, uint64_t n, const int32_t *order,
                        const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev, void *stream)
{
    return report_async(p, m, t, n, order, params, pos_dev, cap, total_dev, reinterpret_cast<hipStream_t>(stream));
}

int32_t sm_patterns_create(uint64_t np, const uint8_t *const *p, const uint64_t *m, const int32_t *const *order,
                           sm_patterns **out)
{
    g_err.clear();
    if (!out)
        return fail(SM_EINVAL, "out is NULL");
    *out = nullptr;
    if (np > 0 && (!p || !m))
        return fail(SM_EINVAL, "p or m is NULL");
    uint64_t total = 0;
    for (uint64_t i = 0; i < np; ++i) {
        int rc = check_pattern(p[i], m[i], order ? order[i] : nullptr);
        if (rc < 0)
            return fail(rc, "pattern " + std::to_string(i) + ": " + g_err);
        total += m[i] + kStepPad;
    }
    Dev *d;
    SM_TRY(get_dev(&d));
    std::unique_ptr<sm_patterns> ps(new sm_patterns());
    ps->dev = d->id;
    const size_t bytes = std::max<uint64_t>(total, 1) * sizeof(uint64_t);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&ps->steps), bytes);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                    std::string("pattern set: ") + hipGetErrorString(e));
    // the tables are built in pinned staging and go up in one copy (a copy
    // from pageable memory is staged by the runtime in many small pieces)
    std::lock_guard<std::mutex> lk(d->mu);
    Upload u;
    int rc = ring_reserve(*d, bytes, &u);
    if (rc == SM_OK) {
        uint64_t *host = reinterpret_cast<uint64_t *>(u.host);
        uint64_t at = 0;
        for (uint64_t i = 0; i < np; ++i) {
            build_steps(p[i], m[i], order ? order[i] : nullptr, host + at);
            ps->off.push_back(at);
            ps->m.push_back(m[i]);
            ps->syms.push_back(pattern_syms(p[i], m[i]));
            at += m[i] + kStepPad;
        }
        if ((e = hipMemcpyAsync(ps->steps, u.host, bytes, hipMemcpyHostToDevice, nullptr)) != hipSuccess)
            rc = fail(SM_EDEVICE, std::string("pattern set upload: ") + hipGetErrorString(e));
        const int rc2 = ring_commit(*d, u, nullptr);
        if (rc == SM_OK)
            rc = rc2;
    }
    if (rc == SM_OK && (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        rc = fail(SM_EDEVICE, std::string("pattern set upload: ") + hipGetErrorString(e));
    if (rc != SM_OK) {
        (void)hipFree(ps->steps);
        return rc;
    }
    *out = ps.release();
    return SM_OK;
}

int32_t sm_patterns_create_ordered(uint64_t np, const uint8_t *const *p, const uint64_t *m, int32_t kind,
                                   const uint64_t *hist_host, sm_patterns **out)
{
    g_err.clear();
    if (kind != SM_ORDER_LTR && kind != SM_ORDER_FREQ && kind != SM_ORDER_H && kind != SM_ORDER_HS)
        return fail(SM_EINVAL, "unknown order kind");
    if (kind == SM_ORDER_FREQ && !hist_host)
        return fail(SM_EINVAL, "SM_ORDER_FREQ needs hist_host");
    if (np > 0 && (!p || !m))
        return fail(SM_EINVAL, "p or m is NULL");
    std::vector<std::vector<int32_t>> ords(np);
    std::vector<const int32_t *> optr(np, nullptr);
    const uint64_t zero_hist[256] = {};
    const FreqRanks ranks(hist_host ? hist_host : zero_hist);
    std::vector<uint32_t> cnt;
    for (uint64_t i = 0; i < np; ++i) {
        if (m[i] == 0 || m[i] >= (1ull << 31) || !p[i])
            return fail(SM_EINVAL, "pattern " + std::to_string(i) + ": bad pattern or length");
        if (kind == SM_ORDER_LTR)
            continue;
        ords[i].resize(m[i]);
        if (kind == SM_ORDER_FREQ)
            ranks.order(p[i], m[i], ords[i].data(), cnt);
        else if (kind == SM_ORDER_H)
            order_fixed_h(m[i], ords[i].data());
        else
            order_fixed_hs(p[i], m[i], ords[i].data());
        optr[i] = ords[i].data();
    }
    return sm_patterns_create(np, p, m, optr.data(), out);
}

int32_t sm_patterns_destroy(sm_patterns *ps)
{
    g_err.clear();
    if (!ps)
        return SM_OK;
    if (ps->steps)
        HIP_TRY(hipFree(ps->steps));
    delete ps;
    return SM_OK;
}

int32_t sm_patterns_count(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n, const sm_params *params,
                          uint64_t *count_dev, void *stream)
{
    g_err.clear();
    SM_TRY(check_set(ps, i));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, false));
    if (!count_dev)
        return fail(SM_EINVAL, "count_dev is NULL");
    const uint64_t m = ps->m[i];
    if (m > n)
        return SM_OK;
    Dev *d;
    SM_TRY(get_dev(&d));
    const Tune tu = resolve(params, m, n);
    return launch_count(*d, make_view(t, n), m, ps->steps + ps->off[i], tu,
                        reinterpret_cast<unsigned long long *>(count_dev), nullptr, nullptr,
                        reinterpret_cast<hipStream_t>(stream), &ps->syms[i]);
}

int64_t sm_patterns_report(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n, const sm_params *params,
                           uint64_t *pos_dev, uint64_t cap, void *stream)
{
    g_err.clear();
    SM_TRY(check_set(ps, i));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, true));
    if (cap > 0 && !pos_dev)
        return fail(SM_EINVAL, "pos is NULL with cap > 0");
    const uint64_t m = ps->m[i];
    if (m > n)
        return 0;
    Dev *d;
    SM_TRY(get_dev(&d));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    if (nonoverlap(params))
        return nonoverlap_core(*d, make_view(t, n), m, ps->steps + ps->off[i], tu, pos_dev, cap, s);
    SM_TRY(report_core(*d, make_view(t, n), m, ps->steps + ps->off[i], tu, cap ? pos_dev : nullptr, cap, d->u64 + 1, s));
    HIP_TRY(hipMemcpyAsync(d->hpin + 1, d->u64 + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return (int64_t)d->hpin[1];
}

int32_t sm_patterns_report_async(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                                 const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev,
                                 void *stream)
{
    g_err.clear();
    SM_TRY(check_set(ps, i));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, false));
    if (cap > 0 && !pos_dev)
        return fail(SM_EINVAL, "pos is NULL with cap > 0");
    if (!total_dev)
        return fail(SM_EINVAL, "total_dev is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(total_dev);
    const uint64_t m = ps->m[i];
    if (m > n) {
        HIP_TRY(launch_fill_u64(tot, 1, 0ull, s));
        return SM_OK;
    }
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    return report_core(*d, make_view(t, n), m, ps->steps + ps->off[i], tu, cap ? pos_dev : nullptr, cap, tot, s);
}

int32_t sm_patterns_report_noalloc(const sm_patterns *ps, uint64_t i, const uint8_t *t, uint64_t n,
                                   const sm_params *params, uint64_t *pos_dev, uint64_t cap, uint64_t *total_dev,
                                   void *stream)
{
    g_err.clear();
    SM_TRY(check_set(ps, i));
    SM_TRY(check_text(t, n));
    SM_TRY(check_flags(params, false));
    if (cap > 0 && !pos_dev)
        return fail(SM_EINVAL, "pos is NULL with cap > 0");
    if (!total_dev)
        return fail(SM_EINVAL, "total_dev is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(total_dev);
    const uint64_t m = ps->m[i];
    if (m > n) {
        HIP_TRY(launch_fill_u64(tot, 1, 0ull, s));
        return SM_OK;
    }
    // the pattern set's creation initialised this device; never initialise (allocate) here
    Dev *d = find_dev(ps->dev);
    if (!d)
        return fail(SM_EINVAL, "the pattern set's device is not initialised (was sm_shutdown called?)");
    std::lock_guard<std::mutex> lk(d->mu);
    const Tune tu = resolve(params, m, n);
    return report_core_noalloc(*d, make_view(t, n), m, ps->steps + ps->off[i], tu, cap ? pos_dev : nullptr, cap,
                               tot, s);
}

// Plans, uploads and launches one validated count batch, or part of one: out_map gives each
// query's output slot, and counts[0, fill_n) are zeroed after the planning succeeded and before
// the kernels run (a batch's first part zeroes the whole batch's counts, the second none).  The
// caller holds d.mu.
static int count_batch_part(Dev &d, const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt,
                            const sm_params *params, unsigned long long *counts, hipStream_t s,
                            const uint32_t *out_map, uint64_t fill_n)
{
    Upload u;
    LaunchPlan lp;
    bool reserved = false;
    AllocFn alloc = [&](size_t bytes, uint8_t **h, uint8_t **dv) {
        SM_TRY(ring_reserve(d, bytes, &u));
        reserved = true;
        *h = u.host;
        *dv = u.dev;
        return (int)SM_OK;
    };
    {
        const int prc = plan_batch(d, q, nq, texts, nt, params, alloc, &lp, nullptr, out_map);
        if (prc < 0) {
            const std::string msg = g_err;
            if (reserved)
                (void)ring_commit(d, u, s);  // give the reservation back
            return fail(prc, msg);
        }
    }
    lp.fill_counts = false;
    int rc = ring_copy(u, lp.bytes, s);
    if (rc == SM_OK && fill_n)
        rc = launch_fill_u64(counts, fill_n, 0ull, s) == hipSuccess ? SM_OK
                                                                      : fail(SM_EDEVICE, "launching the counts fill");
    if (rc == SM_OK)
        rc = launch_plan(d, lp, u.dev, counts, s);
    const std::string msg = g_err;
    const int rc2 = ring_commit(d, u, s);
    if (rc < 0)
        return fail(rc, msg);
    return rc2;
}

// One-shot batches of at least this many queries over at least this many texts are planned in
// two parts, so that the GPU runs the first while the host plans the second.
constexpr uint64_t kSplitMinQueries = 2048;
constexpr uint64_t kSplitMinTexts = 512;

int32_t sm_count_batch(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt,
                       uint64_t *counts_dev, const sm_params *params, void *stream)
{
    g_err.clear();
    if (nq == 0)
        return SM_OK;
    if (!counts_dev)
        return fail(SM_EINVAL, "counts_dev is NULL");
    SM_TRY(check_flags(params, false));
    SM_TRY(validate_batch(q, nq, texts, nt));
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *counts = reinterpret_cast<unsigned long long *>(counts_dev);
    if (nq >= kSplitMinQueries && nt >= kSplitMinTexts) {
        // The parts are split by text id at about half the queries, so each text's queries stay in
        // one part and every text gets the launch mode it would get in a single plan.
        std::vector<uint64_t> per_text(nt, 0);
        for (uint64_t i = 0; i < nq; ++i)
            per_text[q[i].text_id]++;
        uint64_t below = 0, cut = 0;
        while (cut < nt && 2 * below < nq)
            below += per_text[cut++];
        if (below > 0 && below < nq) {
            std::vector<sm_query> part[2];
            std::vector<uint32_t> map[2];
            part[0].reserve(below);
            map[0].reserve(below);
            part[1].reserve(nq - below);
            map[1].reserve(nq - below);
            for (uint64_t i = 0; i < nq; ++i) {
                const int h = q[i].text_id < cut ? 0 : 1;
                part[h].push_back(q[i]);
                map[h].push_back((uint32_t)i);
            }
            for (int h = 0; h < 2; ++h)
                SM_TRY(count_batch_part(*d, part[h].data(), part[h].size(), texts, nt, params, counts, s,
                                        map[h].data(), h == 0 ? nq : 0));
            return SM_OK;
        }
    }
    return count_batch_part(*d, q, nq, texts, nt, params, counts, s, nullptr, nq);
}

// One reporting batch whose scratch fits (see sm_report_batch); the caller
// holds d->mu.
static int report_batch_part(Dev *d, const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt,
                      const uint64_t *caps, uint64_t *pos_dev, uint64_t *totals_dev, const sm_params *params,
                      hipStream_t s)
{
    // per-query report scratch: vector counts, group sums, group offsets
    std::vector<uint64_t> nb(nq, 0), ng(nq, 0), o_bc(nq, 0), o_gs(nq, 0), o_go(nq, 0);
    size_t bytes = 0;
    for (uint64_t i = 0; i < nq; ++i) {
        const sm_text &tx = texts[q[i].text_id];
        if (q[i].m > tx.n)
            continue;
        const uint64_t last = (reinterpret_cast<uintptr_t>(tx.t) & 15u) + tx.n - q[i].m;
        nb[i] = ceil_div(last + 1, kBlock);
        ng[i] = ceil_div(nb[i], kGroupBlocks);
        o_bc[i] = bytes;
        bytes += round_up(nb[i] * sizeof(uint32_t), 256);
        o_gs[i] = bytes;
        bytes += round_up(ng[i] * sizeof(unsigned long long), 256);
        o_go[i] = bytes;
        bytes += round_up(ng[i] * sizeof(unsigned long long), 256);
    }
    if (!d->rb_ev)
        HIP_TRY(hipEventCreateWithFlags(&d->rb_ev, hipEventDisableTiming));
    if (d->rb_cap < bytes) {
        if (d->rb_pending)
            HIP_TRY(hipEventSynchronize(d->rb_ev));  // the old buffer may still be in use
        if (d->rb_buf)
            HIP_TRY(hipFree(d->rb_buf));
        d->rb_buf = nullptr;
        d->rb_cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&d->rb_buf), bytes);
        if (e != hipSuccess)
            return fail(SM_ENOMEM, std::string("report batch scratch: ") + hipGetErrorString(e));
        d->rb_cap = bytes;
    }
    if (d->rb_pending && d->rb_stream != s)  // scratch is shared by all reporting batches (in order on one stream)
        HIP_TRY(hipStreamWaitEvent(s, d->rb_ev, 0));
    if (bytes)
        HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long *>(d->rb_buf), bytes / 8, 0ull, s));
    ReportScratch rs;
    rs.bc.assign(nq, nullptr);
    rs.gs.assign(nq, nullptr);
    for (uint64_t i = 0; i < nq; ++i)
        if (nb[i]) {
            rs.bc[i] = reinterpret_cast<uint32_t *>(d->rb_buf + o_bc[i]);
            rs.gs[i] = reinterpret_cast<unsigned long long *>(d->rb_buf + o_gs[i]);
        }
    // one upload: the batch plan's tables, then the reporting descriptors and the work-item list
    uint64_t nd = 0, nitems = 0;
    for (uint64_t i = 0; i < nq; ++i)
        if (nb[i]) {
            ++nd;
            nitems += ng[i];
        }
    if (nitems >= (1ull << 32))
        return fail(SM_EINVAL, "report batch too large: more than 2^32 groups");
    const size_t rep_items_off = round_up(nd * sizeof(RepDesc), 256);
    const size_t rep_bytes = rep_items_off + nitems * sizeof(uint32_t);
    Upload u;
    LaunchPlan lp;
    bool reserved = false;
    size_t o_rep = 0;
    AllocFn alloc = [&](size_t b, uint8_t **h, uint8_t **dv) {
        o_rep = round_up(b, 256);
        SM_TRY(ring_reserve(*d, o_rep + rep_bytes, &u));
        reserved = true;
        *h = u.host;
        *dv = u.dev;
        return (int)SM_OK;
    };
    {
        const int prc = plan_batch(*d, q, nq, texts, nt, params, alloc, &lp, &rs);
        if (prc < 0) {
            const std::string msg = g_err;
            if (reserved)
                (void)ring_commit(*d, u, s);  // give the reservation back
            return fail(prc, msg);
        }
    }
    unsigned long long *totals = reinterpret_cast<unsigned long long *>(totals_dev);
    RepDesc *hd = reinterpret_cast<RepDesc *>(u.host + o_rep);
    uint32_t *hitem = reinterpret_cast<uint32_t *>(u.host + o_rep + rep_items_off);
    uint32_t win_max = 0;
    uint64_t off = 0, k = 0, item = 0;
    for (uint64_t i = 0; i < nq; ++i) {
        const uint64_t cap = caps[i];
        uint64_t *pos = cap ? pos_dev + off : nullptr;
        off += cap;
        if (!nb[i])
            continue;
        const sm_text &tx = texts[q[i].text_id];
        RepDesc D{};
        D.tv = make_view(tx.t, tx.n);
        D.last = D.tv.first + tx.n - q[i].m;
        D.nblocks = nb[i];
        D.steps = reinterpret_cast<const uint64_t *>(u.dev + lp.o_steps) + lp.steps_of[i];
        D.m = (uint32_t)q[i].m;
        uint64_t win = kBlock + halo_for(q[i].m);
        if (kWaves * win + kGroupBlocks * sizeof(uint32_t) + 64 > kMaxLds)
            win = 0;  // long pattern: read the text from global memory
        D.win = (uint32_t)win;
        win_max = std::max(win_max, D.win);
        D.bc = rs.bc[i];
        D.gs = rs.gs[i];
        D.go = reinterpret_cast<unsigned long long *>(d->rb_buf + o_go[i]);
        D.total = totals + i;
        D.pos = reinterpret_cast<unsigned long long *>(pos);
        D.cap = cap;
        D.ngroups = ng[i];
        D.item0 = item;
        hd[k] = D;
        std::fill(hitem + item, hitem + item + ng[i], (uint32_t)k);
        item += ng[i];
        ++k;
    }
    int rc = ring_copy(u, o_rep + rep_bytes, s);
    if (rc == SM_OK)
        rc = launch_plan(*d, lp, u.dev, totals, s);  // counts, plus the per-vector counts of every query
    if (rc == SM_OK && nd) {
        // every query's group offsets, then the ordered writes of all matching vectors: two launches
        const int wpc = (params && params->wgs_per_cu > 0) ? std::min(params->wgs_per_cu, 32) : 6;
        const uint64_t target = (uint64_t)std::max(d->cus, 1) * (uint64_t)wpc;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nitems, target));
        hipError_t e = launch_report_multi(reinterpret_cast<const RepDesc *>(u.dev + o_rep), nd,
                                           reinterpret_cast<const uint32_t *>(u.dev + o_rep + rep_items_off), nitems,
                                           win_max, grid, s);
        if (e != hipSuccess)
            rc = fail(SM_EDEVICE, std::string("report batch: ") + hipGetErrorString(e));
    }
    if (rc == SM_OK) {
        hipError_t e = hipEventRecord(d->rb_ev, s);
        if (e == hipSuccess) {
            d->rb_pending = true;
            d->rb_stream = s;
        }
        else
            rc = fail(SM_EDEVICE, std::string("report batch: ") + hipGetErrorString(e));
    }
    const std::string msg = g_err;
    const int rc2 = ring_commit(*d, u, s);
    if (rc < 0)
        return fail(rc, msg);
    return rc2;
}


int32_t sm_report_batch(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt, const uint64_t *caps,
                        uint64_t *pos_dev, uint64_t *totals_dev, const sm_params *params, void *stream)
{
    g_err.clear();
    if (nq == 0)
        return SM_OK;
    if (!caps || !totals_dev)
        return fail(SM_EINVAL, "caps or totals_dev is NULL");
    SM_TRY(check_flags(params, false));
    SM_TRY(validate_batch(q, nq, texts, nt));
    uint64_t total_cap = 0;
    for (uint64_t i = 0; i < nq; ++i) {
        if (caps[i] > (1ull << 60) || total_cap + caps[i] > (1ull << 60))
            return fail(SM_EINVAL, "query " + std::to_string(i) + ": caps too large");
        total_cap += caps[i];
    }
    if (total_cap > 0 && !pos_dev)
        return fail(SM_EINVAL, "pos_dev is NULL with caps > 0");
    Dev *d;
    SM_TRY(get_dev(&d));
    std::lock_guard<std::mutex> lk(d->mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // split into parts whose per-query scratch (vector counts, group sums and offsets) stays bounded
    uint64_t i0 = 0, pos_off = 0;
    while (i0 < nq) {
        uint64_t i1 = i0, need = 0, part_cap = 0;
        while (i1 < nq) {
            const sm_text &tx = texts[q[i1].text_id];
            uint64_t b = 0;
            if (q[i1].m <= tx.n) {
                const uint64_t nbk = ceil_div((reinterpret_cast<uintptr_t>(tx.t) & 15u) + tx.n - q[i1].m + 1, kBlock);
                b = round_up(nbk * 4, 256) + 2 * round_up(ceil_div(nbk, kGroupBlocks) * 8, 256);
            }
            if (i1 > i0 && need + b > kRepScratchMax)
                break;
            need += b;
            part_cap += caps[i1];
            ++i1;
        }
        SM_TRY(report_batch_part(d, q + i0, i1 - i0, texts, nt, caps + i0, pos_dev ? pos_dev + pos_off : nullptr,
                                 totals_dev + i0, params, s));
        pos_off += part_cap;
        i0 = i1;
    }
    return SM_OK;
}

int32_t sm_batch_create(const sm_query *q, uint64_t nq, const sm_text *texts, uint64_t nt, const sm_params *params,
                        sm_batch **out)
{
    g_err.clear();
    if (!out)
        return fail(SM_EINVAL, "out is NULL");
    *out = nullptr;
    SM_TRY(check_flags(params, false));
    if (nq > 0)
        SM_TRY(validate_batch(q, nq, texts, nt));
    Dev *d;
    SM_TRY(get_dev(&d));
    sm_batch *b = new sm_batch();
    b->dev = d->id;
    std::vector<uint8_t> host;
    AllocFn alloc = [&](size_t bytes, uint8_t **h, uint8_t **dv) {
        host.assign(bytes, 0);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->buf), bytes);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                        std::string("batch plan buffer: ") + hipGetErrorString(e));
        *h = host.data();
        *dv = b->buf;
        return (int)SM_OK;
    };
    int rc = nq > 0 ? plan_batch(*d, q, nq, texts, nt, params, alloc, &b->lp) : SM_OK;
    if (rc == SM_OK && b->buf) {
        hipError_t e = hipMemcpy(b->buf, host.data(), b->lp.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess)
            rc = fail(SM_EDEVICE, std::string("batch plan upload: ") + hipGetErrorString(e));
    }
    if (rc < 0) {
        if (b->buf)
            (void)hipFree(b->buf);
        delete b;
        return rc;
    }
    *out = b;
    return SM_OK;
}

int32_t sm_batch_run(const sm_batch *b, uint64_t *counts_dev, void *stream)
{
    g_err.clear();
    if (!b)
        return fail(SM_EINVAL, "batch plan is NULL");
    if (b->lp.nq == 0)
        return SM_OK;
    if (!counts_dev)
        return fail(SM_EINVAL, "counts_dev is NULL");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->dev)
        return fail(SM_EINVAL, "batch plan belongs to another device");
    Dev *d;
    SM_TRY(get_dev(&d));
    return launch_plan(*d, b->lp, b->buf, reinterpret_cast<unsigned long long *>(counts_dev),
                       reinterpret_cast<hipStream_t>(stream));
}

int32_t sm_batch_destroy(sm_batch *b)
{
    g_err.clear();
    if (!b)
        return SM_OK;
    if (b->buf)
        HIP_TRY(hipFree(b->buf));
    delete b;
    return SM_OK;
}

}  // extern "C"
