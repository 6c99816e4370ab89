// HIP kernels for exact string matching on gfx950 (MI355X).
//
// Method (arXiv 1612.01506): for each block of start positions, AND the
// result of comparing one pattern symbol against the text at every start of
// the block (SIMDcompare, Section 2.1) into a found mask, taking the pattern
// positions in compare order pi (Section 2.2), doing the first r compares
// unconditionally and testing found for zero after each later one (loop
// peeling, Section 2.3, Algorithm 4), and adding popcount(found) to the count.
//
// gfx950 mapping:
//   * A wave vector covers 1024 starts: lane L holds four dwords d[0..3], and
//     byte b of d[k] stands for start wb + 256k + 4L + b.  The lane-strided
//     layout makes every LDS dword read of a compare step conflict free.
//   * found is kept inverted, as a byte-wise difference: byte == 0 means the
//     start is still alive.  One compare step for pattern position j is, per
//     dword, an aligned LDS dword pair, v_alignbyte_b32 by j mod 4, XOR with
//     p[j] replicated into four bytes, OR into d.  Three VALU ops per four
//     starts; no per-byte compares.
//   * The zero test of found (Algorithm 4's exit) is a wave-wide "any byte of
//     any d is zero" test: ((d - 0x01..01) & ~d & 0x80..80) != 0 is exact for
//     the existence of a zero byte, and one ballot makes it wave uniform.
//   * popcount(found) counts exactly-zero bytes:
//     ~(((d & 0x7F..7F) + 0x7F..7F) | d | 0x7F..7F) has 0x80 in each zero byte.
//   * Text tiles (4, 8 or 16 KiB) plus an (m + 4)-byte halo are staged in LDS
//     by DMA (global_load_lds_dwordx4) into two buffers: the next tile's loads
//     are in flight while the current one is searched.  Tiles are dealt to
//     workgroups in chunks of contiguous tiles, so a halo is mostly the start
//     of the tile the same workgroup loads next (an L2 hit, not a second HBM
//     read).  Texts far larger than the last-level cache are read with the
//     non-temporal policy.
//   * Counts: 32-bit lane accumulators, DPP wave reductions, one LDS
//     reduction and one 64-bit atomicAdd per workgroup.
//   * Small alphabets: a single search may instead build, per tile, one bitmap
//     per distinct pattern symbol from the text bytes held in registers (byte
//     transposes, then byte-equality tests or bit planes), after which every
//     compare is a funnel shift and AND over 32 starts.
//   * Batches: byte-tile kernels run many queries over one staged tile (or one
//     query over runs of tiles, with a record per run), and the bitmap kernel
//     turns every compare of every query into a funnel shift and AND over
//     per-tile symbol bitmaps (one SIMDcompare per symbol and tile, shared).
//     A lone query on a text of at most 4 symbols takes runs of bitmap tiles
//     the same way (the single search's bitmap tile code, one record per run).
#include "sm_internal.h"

namespace smk {

// ------------------------------------------------------------------ helpers

// Index of this wave in the workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ uint32_t wave_id()
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Load from a table the kernels never write (step tables, query records,
// work lists) through the constant address space, so a wave-uniform address
// becomes a scalar load.
template <typename T>
__device__ __forceinline__ T ldc(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "whole dwords only");
    constexpr int N = sizeof(T) / 4;
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)(p);
    uint32_t w[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
        w[i] = q[i];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

__device__ __forceinline__ uint32_t step_pos(uint64_t st) { return (uint32_t)st; }
__device__ __forceinline__ uint32_t step_rep(uint64_t st) { return (uint32_t)(st >> 32); }

// Initial found for the wave vector at coordinate wb: starts outside
// [first, last] are dead (byte 0xFF); all others alive (0).
__device__ __forceinline__ uint32_t bytes_below(uint32_t c)  // low c bytes set, c in 0..4
{
    return c >= 4u ? 0xFFFFFFFFu : (1u << (8u * c)) - 1u;
}

__device__ __forceinline__ void init_alive(uint64_t wb, uint64_t first, uint64_t last, uint32_t lane,
                                           uint32_t (&d)[4])
{
    if (wb >= first && wb + (kBlock - 1) <= last) {
        d[0] = d[1] = d[2] = d[3] = 0u;
        return;
    }
    // valid offsets within the vector: [lo, hi] (wave uniform, 32-bit)
    const uint32_t lo = first > wb ? (uint32_t)(first - wb) : 0u;
    const int64_t hi64 = (int64_t)last - (int64_t)wb;
    const int32_t hi = hi64 > (int64_t)kBlock ? (int32_t)kBlock : (int32_t)hi64;  // may be negative
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t q = (int32_t)(256u * k + 4u * lane);
        const int32_t cl = min(max((int32_t)lo - q, 0), 4), ch = min(max(hi - q + 1, 0), 4);
        const uint32_t valid = bytes_below((uint32_t)ch) & ~bytes_below((uint32_t)cl);
        d[k] = ~valid;
    }
}

// The same dead-start bytes for the vector at tile offset boff, given the
// valid starts of its tile as tile offsets lo..hi (32-bit, wave uniform),
// ORed into d.
__device__ __forceinline__ void mask_dead_tile(uint32_t boff, uint32_t lo, uint32_t hi, uint32_t lane,
                                               uint32_t (&d)[4])
{
    const int32_t vlo = (int32_t)lo - (int32_t)boff, vhi = (int32_t)hi - (int32_t)boff;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t q = (int32_t)(256u * k + 4u * lane);
        const int32_t cl = min(max(vlo - q, 0), 4), ch = min(max(vhi - q + 1, 0), 4);
        d[k] |= ~(bytes_below((uint32_t)ch) & ~bytes_below((uint32_t)cl));
    }
}

// One compare step from an LDS tile.  lb points at the lane's first dword of
// the wave vector; the window for pattern position j starts j bytes later.
__device__ __forceinline__ void step_lds(const uint8_t *lb, uint64_t st, uint32_t (&d)[4])
{
    const uint32_t j = step_pos(st), rep = step_rep(st), sh = j & 3u;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(lb + (j & ~3u));
#pragma unroll
    for (int k = 0; k < 4; ++k)
        d[k] |= __builtin_amdgcn_alignbyte(w[64 * k + 1], w[64 * k], sh) ^ rep;
}

// The first compare of a vector, which sets d instead of ORing into it.
__device__ __forceinline__ void step_lds_first(const uint8_t *lb, uint64_t st, uint32_t (&d)[4])
{
    const uint32_t j = step_pos(st), rep = step_rep(st), sh = j & 3u;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(lb + (j & ~3u));
#pragma unroll
    for (int k = 0; k < 4; ++k)
        d[k] = __builtin_amdgcn_alignbyte(w[64 * k + 1], w[64 * k], sh) ^ rep;
}

__device__ __forceinline__ uint32_t load_dword(const TextView &tv, uint64_t u)
{
    // u is a multiple of 4 and end16 a multiple of 16: the dword lies inside a
    // loaded chunk iff u < end16.
    return u < tv.end16 ? *reinterpret_cast<const uint32_t *>(tv.base + u) : 0u;
}

// One compare step reading the text from global memory (long patterns and the
// report write pass).  lu = wb + 4 * lane.
__device__ __forceinline__ void step_global(const TextView &tv, uint64_t lu, uint64_t st, uint32_t (&d)[4])
{
    const uint32_t j = step_pos(st), rep = step_rep(st), sh = j & 3u;
    const uint64_t u = lu + (j & ~3u);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t lo = load_dword(tv, u + 256u * k), hi = load_dword(tv, u + 256u * k + 4u);
        d[k] |= __builtin_amdgcn_alignbyte(hi, lo, sh) ^ rep;
    }
}

// Wave-uniform: does any start of the wave vector survive?
__device__ __forceinline__ bool any_alive(const uint32_t (&d)[4])
{
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        h |= (d[k] - 0x01010101u) & ~d[k];
    return __any((h & 0x80808080u) != 0u);
}

// 0x80 in every byte of d that is exactly zero.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t d)
{
    return ~((((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) | 0x7F7F7F7Fu);
}

__device__ __forceinline__ uint32_t count_alive(const uint32_t (&d)[4])
{
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c += __popc(zero_bytes(d[k]));
    return c;
}

// Wave-wide reductions with DPP moves (no LDS traffic): quad permutes, row
// shifts by 4 and 8, then row broadcasts of lanes 15 and 31; lane 63 ends
// with the whole wave's value.  Lanes a DPP move does not write receive
// `ident`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v, uint32_t ident)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROWMASK, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
    v += dpp_mov<0xb1>(v, 0u);        // quad_perm [1,0,3,2]
    v += dpp_mov<0x4e>(v, 0u);        // quad_perm [2,3,0,1]
    v += dpp_mov<0x114>(v, 0u);       // row_shr:4
    v += dpp_mov<0x118>(v, 0u);       // row_shr:8
    v += dpp_mov<0x142, 0xa>(v, 0u);  // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xc>(v, 0u);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Text sources for the compare steps of one wave vector.
// LdsText: the vector's window is staged in LDS; vb = byte 0 of the vector.
struct LdsText {
    const uint8_t *vb;
    const uint8_t *lb;  // vb + 4 * lane
    __device__ __forceinline__ void step(uint64_t st, uint32_t (&d)[4]) const { step_lds(lb, st, d); }
    __device__ __forceinline__ uint32_t byte(uint32_t rel) const { return vb[rel]; }
};

// GlobalText: the window is read from global memory; wb = coordinate of the vector.
struct GlobalText {
    const TextView *tv;
    uint64_t wb;
    uint64_t lu;  // wb + 4 * lane
    __device__ __forceinline__ void step(uint64_t st, uint32_t (&d)[4]) const { step_global(*tv, lu, st, d); }
    __device__ __forceinline__ uint32_t byte(uint32_t rel) const
    {
        const uint64_t u = wb + rel;
        return u < tv->end16 ? (uint32_t)tv->base[u] : 0u;
    }
};

constexpr uint32_t kTestEach = 4;   // tail compares each followed by a zero test
constexpr uint32_t kGroup = 8;      // later tail compares per zero test
constexpr uint32_t kVerifyMin = 64; // remaining compares from which lone candidates are verified across lanes
constexpr uint32_t kVerifyMax = 4;  // most alive starts verified one at a time

__device__ __forceinline__ uint32_t wave_min32(uint32_t v)
{
    const uint32_t I = 0xFFFFFFFFu;
    v = min(v, dpp_mov<0xb1>(v, I));
    v = min(v, dpp_mov<0x4e>(v, I));
    v = min(v, dpp_mov<0x114>(v, I));
    v = min(v, dpp_mov<0x118>(v, I));
    v = min(v, dpp_mov<0x142, 0xa>(v, I));
    v = min(v, dpp_mov<0x143, 0xc>(v, I));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Verify each alive start of the vector on compares l..m-1, 64 compares at
// a time across the lanes (a mismatch in any lane ends that start).  The
// AND over the remaining compares is the same; it is only grouped by start
// instead of by compare.  Starts are visited in increasing offset `rel`
// (256k + 4 * lane + byte) through a wave-uniform cursor; a start that fails
// gets its byte of d set nonzero.  Leaves d final.
template <typename Text>
__device__ __forceinline__ void verify_candidates(const uint64_t *steps, uint32_t l, uint32_t m, uint32_t lane,
                                                  uint32_t (&d)[4], const Text &tx)
{
    // the first 64 remaining compares, one per lane, serve every candidate
    const uint32_t idx0 = l + lane;
    const uint64_t st0 = idx0 < m ? steps[idx0] : 0ull;
    uint32_t cursor = 0;
    while (true) {
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 3; k >= 0; --k) {
            const uint32_t base = 256u * k + 4u * lane;
            uint32_t z = zero_bytes(d[k]);
            if (cursor > base)
                z = cursor - base >= 4u ? 0u : z & (0xFFFFFFFFu << (8 * (cursor - base)));
            if (z)
                best = base + ((uint32_t)__builtin_ctz(z) >> 3);
        }
        best = wave_min32(best);
        if (best == 0xFFFFFFFFu)
            break;
        bool ok = !__any(idx0 < m && tx.byte(best + step_pos(st0)) != (step_rep(st0) & 0xFFu));
        for (uint32_t b0 = l + 64u; ok && b0 < m; b0 += 64u) {
            const uint32_t idx = b0 + lane;
            bool bad = false;
            if (idx < m) {
                const uint64_t st = steps[idx];
                bad = tx.byte(best + step_pos(st)) != (step_rep(st) & 0xFFu);
            }
            ok = !__any(bad);
        }
        if (!ok && lane == ((best & 255u) >> 2)) {
            const uint32_t k = best >> 8, dead = 0xFFu << (8 * (best & 3u));
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                if ((uint32_t)kk == k)
                    d[kk] |= dead;
        }
        cursor = best + 1u;
    }
}

// Compares l..m-1 for a vector still alive after the peel.  The first
// kTestEach are each followed by the zero test of Algorithm 4; later ones go
// in groups of kGroup per test, so a lone long survivor does not serialise on
// one load-compare-test round trip per compare; after a group, a handful of
// survivors facing many more compares are verified one at a time.  Returns false if the vector
// died; otherwise d is final (byte == 0 exactly at the matching starts).
template <typename Text>
__device__ __forceinline__ bool search_tail(const uint64_t *steps, uint32_t l, uint32_t m, uint32_t lane,
                                            uint32_t (&d)[4], const Text &tx)
{
    const uint32_t l1 = min(m, l + kTestEach);
    for (; l < l1; ++l) {
        tx.step(ldc(&steps[l]), d);
        if (!any_alive(d))
            return false;
    }
    // candidates are verified one by one only once a group of compares has
    // left a few alive: earlier, few survivors are common and mostly die
    // within the next group, which costs less than the verification loop
    bool grouped = false;
    while (l < m) {
        if (grouped && m - l >= kVerifyMin) {
            const uint32_t alive = wave_sum32(count_alive(d));
            if (alive <= kVerifyMax) {
                verify_candidates(steps, l, m, lane, d, tx);
                return true;
            }
        }
        const uint32_t g = min(kGroup, m - l);
#pragma unroll 1
        for (uint32_t u = 0; u < g; ++u)
            tx.step(ldc(&steps[l + u]), d);
        l += g;
        grouped = true;
        if (!any_alive(d))
            return false;
    }
    return true;
}

// Algorithm 4 over one wave vector with a compile-time peel factor R (R <= m):
// R unconditional compares, a zero test, then the tail.  Returns whether any
// start survived; d is then final.
template <int R, typename Text>
__device__ __forceinline__ bool search_vector(const uint64_t *steps, const uint64_t (&pk)[R], uint32_t m,
                                              uint32_t lane, uint32_t (&d)[4], const Text &tx)
{
#pragma unroll
    for (int l = 0; l < R; ++l)
        tx.step(pk[l], d);
    if (m == (uint32_t)R)  // every compare done: d is final, and count_alive gives 0 for a dead vector
        return true;
    if (!any_alive(d))
        return false;
    return search_tail(steps, R, m, lane, d, tx);
}

// The same for a vector at tile offset boff of an LDS tile whose valid starts
// are the tile offsets lo..hi.  The first compare sets d, and the dead starts
// of an edge vector (one not wholly inside lo..hi) are marked after the peel
// rather than before: the AND of the compares with the validity mask, taken
// in another order.  An inner vector thus spends no work on its bounds.
template <int R>
__device__ __forceinline__ bool search_vector_tile(const uint64_t *steps, const uint64_t (&pk)[R], uint32_t m,
                                                   uint32_t lane, uint32_t (&d)[4], const LdsText &tx, bool edge,
                                                   uint32_t boff, uint32_t lo, uint32_t hi)
{
    step_lds_first(tx.lb, pk[0], d);
#pragma unroll
    for (int l = 1; l < R; ++l)
        tx.step(pk[l], d);
    if (edge)
        mask_dead_tile(boff, lo, hi, lane, d);
    if (m == (uint32_t)R)
        return true;
    if (!any_alive(d))
        return false;
    return search_tail(steps, R, m, lane, d, tx);
}

// Same with a run-time peel factor r (batch queries carry their own r).
template <typename Text>
__device__ __forceinline__ bool search_vector_rt(const uint64_t *steps, uint32_t r, uint32_t m, uint32_t lane,
                                                 uint32_t (&d)[4], const Text &tx)
{
    for (uint32_t l = 0; l < r; ++l)
        tx.step(ldc(&steps[l]), d);
    if (!any_alive(d))
        return false;
    return search_tail(steps, r, m, lane, d, tx);
}

// Search of a vector whose number of matches `want` (>= 1) is already known
// from the count pass: the matches are among the starts still alive after any
// prefix of the compares, so once exactly `want` are alive, d is final.  The
// compares go in groups of kTestEach per test (from none), so a vector whose
// survivors are its matches costs a few compares whatever m is; a handful of
// other survivors facing many more compares are verified one at a time.
template <typename Text>
__device__ __forceinline__ void search_known(const uint64_t *steps, uint32_t m, uint32_t lane, uint32_t want,
                                             uint32_t (&d)[4], const Text &tx)
{
    uint32_t l = 0;
    while (l < m) {
        const uint32_t alive = wave_sum32(count_alive(d));
        if (alive <= want)
            return;
        if (m - l >= kVerifyMin && alive <= kVerifyMax) {
            verify_candidates(steps, l, m, lane, d, tx);
            return;
        }
        const uint32_t g = min(kTestEach, m - l);
#pragma unroll 1
        for (uint32_t u = 0; u < g; ++u)
            tx.step(ldc(&steps[l + u]), d);
        l += g;
    }
}

// ------------------------------------------------------------- tile staging

__device__ __forceinline__ void wg_add_count(unsigned long long acc, unsigned long long *dst, uint32_t tid)
{
    __shared__ unsigned long long red[kWaves];
    const unsigned long long w = wave_sum64(acc);
    if ((tid & 63u) == 0)
        red[tid >> 6] = w;
    __syncthreads();
    if (tid == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (uint32_t i = 0; i < kWaves; ++i)
            s += red[i];
        if (s && dst)
            atomicAdd(dst, s);
    }
}

// ----------------------------------------------------------- count kernels

// Cache-policy operand of the tile loads.  A text much larger than the last
// level cache streams through once per search, and the non-temporal policy
// (the `nt` bit) reads it about 10% faster; a text the cache can partly hold
// across searches is read faster without it.
constexpr int kLoadDefault = 0;
constexpr int kLoadStream = 2;  // nt

// Asynchronous tile load straight into LDS (global_load_lds_dwordx4): lane
// i of a wave writes its 16 bytes at the wave-uniform LDS base + 16 * i.
// Chunks at or past end16 are skipped; their LDS bytes keep stale values,
// which only ever meet dead (out-of-text) starts.
template <int POLICY>
__device__ __forceinline__ void dma16(const TextView &tv, uint64_t u, uint8_t *lds_wave_base)
{
    if (u < tv.end16)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(tv.base + u),
                                         (__attribute__((address_space(3))) void *)(lds_wave_base),
                                         16, 0, POLICY);
}

// Issues the loads of tile [ts, ts + T) and its halo [ts + T, ts + T + 16 * hch)
// into the LDS buffer buf.
template <int CPL, int POLICY = kLoadDefault>
__device__ __forceinline__ void dma_tile(const TextView &tv, uint64_t ts, uint32_t tid, uint32_t hch, uint8_t *buf)
{
    constexpr uint32_t T = kWG * 16u * CPL;
    const uint32_t wbase = tid & ~63u, lane = tid & 63u;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        dma16<POLICY>(tv, ts + 16ull * (tid + kWG * c), buf + 16u * (wbase + kWG * c));
    for (uint32_t ch = tid; ch < hch; ch += kWG)
        dma16<POLICY>(tv, ts + T + 16ull * ch, buf + T + 16u * (ch - lane));
}

__device__ __forceinline__ void wait_dma()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's LDS loads have landed
}

// Single search, text staged in LDS.  Tiles are dealt out in chunks of
// 2^chunk_log2 contiguous tiles, chunk c to workgroup c mod G, so the tiles in
// flight at any moment form a nearly contiguous window of the text (even HBM
// channel load) while a halo is still mostly the start of the tile the same
// workgroup loads next.  Wave w takes vectors w*CPL .. w*CPL + CPL - 1 of each
// tile.  Two LDS buffers of T + halo bytes: the loads of the next tile are in
// flight while the current one is searched.
template <int CPL, int R, bool STREAM>
__global__ __launch_bounds__(kWG) void k_count_staged(CountArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t T = kWG * 16u * CPL;
    constexpr int kPolicy = STREAM ? kLoadStream : kLoadDefault;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    const uint32_t hch = a.halo >> 4;
    const uint32_t TB = T + a.halo;
    const uint64_t kmask = (1ull << a.chunk_log2) - 1u;
    auto tile_of = [&](uint64_t i) {
        return (((uint64_t)blockIdx.x + (i >> a.chunk_log2) * gridDim.x) << a.chunk_log2) + (i & kmask);
    };

    uint64_t pk[R];
#pragma unroll
    for (int l = 0; l < R; ++l)
        pk[l] = ldc(&a.steps[l]);

    unsigned long long acc = 0;
    uint64_t tile = tile_of(0);
    if (tile < a.ntiles)
        dma_tile<CPL, kPolicy>(a.tv, tile * T, tid, hch, lds);
    for (uint64_t i = 0; tile < a.ntiles; ++i) {
        const uint64_t ts = tile * T;
        uint8_t *cur = lds + (i & 1u) * TB;
        const uint64_t next = tile_of(i + 1);
        wait_dma();
        __syncthreads();  // tile visible to all waves; the other buffer is free
        if (next < a.ntiles)
            dma_tile<CPL, kPolicy>(a.tv, next * T, tid, hch, lds + ((i + 1) & 1u) * TB);
        // the tile's valid starts as 32-bit tile offsets lo..hi (tile < ntiles, so last >= ts)
        const uint64_t rem = a.last - ts;
        const uint32_t hi = rem >= T ? T - 1u : (uint32_t)rem;
        const uint32_t lo = ts < a.tv.first ? (uint32_t)(a.tv.first - ts) : 0u;
#pragma unroll
        for (int b = 0; b < CPL; ++b) {
            const uint32_t boff = (wave * CPL + b) * kBlock;
            const uint64_t wb = ts + boff;
            if (boff > hi)
                break;
            uint32_t d[4];
            const bool edge = boff < lo || boff + (kBlock - 1u) > hi;
            const LdsText tx{cur + boff, cur + boff + 4u * lane};
            const uint32_t c =
                search_vector_tile<R>(a.steps, pk, a.m, lane, d, tx, edge, boff, lo, hi) ? count_alive(d) : 0u;
            if (a.block_counts && __any(c != 0u)) {
                const uint32_t s = wave_sum32(c);
                if (lane == 0) {
                    a.block_counts[wb / kBlock] = s;
                    atomicAdd(&a.group_sums[wb / kBlock / kGroupBlocks], (unsigned long long)s);
                }
            }
            acc += c;
        }
        tile = next;
    }
    wg_add_count(acc, a.count, tid);
}

// Single search reading the text straight from global memory (patterns too
// long for an LDS halo).  Waves take vectors in a grid-stride loop.
template <int R>
__global__ __launch_bounds__(kWG) void k_count_global(CountArgs a)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    uint64_t pk[R];
#pragma unroll
    for (int l = 0; l < R; ++l)
        pk[l] = ldc(&a.steps[l]);
    unsigned long long acc = 0;
    for (uint64_t blk = (uint64_t)blockIdx.x * kWaves + wave_id(); blk < a.nblocks; blk += nw) {
        const uint64_t wb = blk * kBlock;
        uint32_t d[4];
        init_alive(wb, a.tv.first, a.last, lane, d);
        const GlobalText tx{&a.tv, wb, wb + 4u * lane};
        const uint32_t c = search_vector<R>(a.steps, pk, a.m, lane, d, tx) ? count_alive(d) : 0u;
        if (a.block_counts && __any(c != 0u)) {
            const uint32_t s = wave_sum32(c);
            if (lane == 0) {
                a.block_counts[blk] = s;
                atomicAdd(&a.group_sums[blk / kGroupBlocks], (unsigned long long)s);
            }
        }
        acc += c;
    }
    wg_add_count(acc, a.count, tid);
}

// ---------------------------------------------------------- report kernels
//
// Reporting version (Section 2.1) in two steps after the count pass has
// written the nonzero per-vector counts into a zero-filled array and added
// them to the sums of their groups of kGroupBlocks vectors:
//   k_scan_groups  exclusive scan of the group sums and the total;
//   k_report_write for each group with matches: exclusive offsets of its
//                  vectors in LDS, then every vector with matches is searched
//                  again (its window staged in a per-wave LDS region) and its
//                  starts are written in increasing order.  Within a vector the
//                  order is k-major, then lane, then byte -- increasing start --
//                  and lane offsets come from a bit-sliced ballot prefix sum.

// Exclusive scan of the group sums (one workgroup of 1024 threads), and the total.
__global__ __launch_bounds__(1024) void k_scan_groups(const unsigned long long *gs, uint64_t ng,
                                                     unsigned long long *go, unsigned long long *total)
{
    __shared__ unsigned long long part[1024];
    const uint32_t tid = threadIdx.x;
    const uint64_t per = (ng + 1023u) / 1024u;
    const uint64_t b0 = min((uint64_t)tid * per, ng), b1 = min(b0 + per, ng);
    unsigned long long s = 0;
    for (uint64_t i = b0; i < b1; ++i)
        s += gs[i];
    part[tid] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
        const unsigned long long v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned long long run = tid ? part[tid - 1] : 0ull;
    for (uint64_t i = b0; i < b1; ++i) {
        go[i] = run;
        run += gs[i];
    }
    if (tid == 1023u)
        *total = part[1023];
}

// Writes the starts of one vector whose final d is known, in increasing order
// from output index o.
__device__ __forceinline__ void write_vector(const uint32_t (&d)[4], uint64_t wb, uint64_t first, uint32_t lane,
                                             unsigned long long o, unsigned long long *pos, uint64_t cap)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t z = zero_bytes(d[k]);
        const uint32_t ck = __popc(z);
        const unsigned long long b1 = __ballot(ck & 1u), b2 = __ballot(ck & 2u), b4 = __ballot(ck & 4u);
        const uint32_t ex = lanes_below(b1) + 2u * lanes_below(b2) + 4u * lanes_below(b4);
        const uint32_t tot = __popcll(b1) + 2u * __popcll(b2) + 4u * __popcll(b4);
        unsigned long long idx = o + ex;
#pragma unroll
        for (int by = 0; by < 4; ++by) {
            if (z & (0x80u << (8 * by))) {
                if (idx < cap)
                    pos[idx] = wb + 256u * k + 4u * lane + by - first;
                ++idx;
            }
        }
        o += tot;
    }
}

// One group of kGroupBlocks vectors of a report: exclusive offsets of its
// vectors in LDS, then every vector with matches is searched again, knowing
// its count (its window staged in the wave's LDS region `mine` of win bytes,
// 1024 + halo, or read from global memory when win is 0 for long patterns),
// and its starts written in increasing order.  Leaves the group's per-vector
// counts and sum zeroed.  Whole workgroup.
__device__ __forceinline__ void report_write_group(const CountArgs &a, uint32_t *bc,
                                                   unsigned long long *gs, const unsigned long long *go, uint64_t g,
                                                   unsigned long long *pos, uint64_t cap, uint32_t win, uint8_t *mine,
                                                   uint32_t *off, uint32_t *wsum)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    if (gs[g] == 0)
        return;
    const uint64_t b0 = g * kGroupBlocks;
    // exclusive offsets of the group's vectors (4 consecutive per thread)
    uint32_t c[kGroupBlocks / kWG], s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kGroupBlocks / kWG; ++i) {
        const uint64_t b = b0 + (kGroupBlocks / kWG) * tid + i;
        c[i] = b < a.nblocks ? bc[b] : 0u;
        s += c[i];
    }
    uint32_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o)
            inc += v;
    }
    if (lane == 63u)
        wsum[wave] = inc;
    __syncthreads();
    uint32_t run = inc - s;
    for (uint32_t w = 0; w < wave; ++w)
        run += wsum[w];
#pragma unroll
    for (uint32_t i = 0; i < kGroupBlocks / kWG; ++i) {
        off[(kGroupBlocks / kWG) * tid + i] = run;
        run += c[i];
    }
    __syncthreads();
    const unsigned long long gbase = go[g];
    for (uint32_t j0 = wave * 64u; j0 < kGroupBlocks; j0 += kWaves * 64u) {
        const uint64_t bb = b0 + j0 + lane;
        const uint32_t cb = bb < a.nblocks ? bc[bb] : 0u;
        unsigned long long nz = __ballot(cb != 0u);
        while (nz) {
            const int bit = __ffsll((long long)nz) - 1;
            nz &= nz - 1;
            const uint32_t want = (uint32_t)__builtin_amdgcn_readlane((int)cb, bit);
            const uint64_t wb = (b0 + j0 + (uint64_t)bit) * kBlock;
            uint32_t d[4];
            init_alive(wb, a.tv.first, a.last, lane, d);
            if (win) {
                for (uint32_t ch = lane; ch < win / 16u; ch += 64u) {
                    const uint64_t u = wb + 16ull * ch;
                    *reinterpret_cast<uint4 *>(mine + 16u * ch) =
                        u < a.tv.end16 ? *reinterpret_cast<const uint4 *>(a.tv.base + u) : make_uint4(0, 0, 0, 0);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const LdsText tx{mine, mine + 4u * lane};
                search_known(a.steps, a.m, lane, want, d, tx);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                const GlobalText tx{&a.tv, wb, wb + 4u * lane};
                search_known(a.steps, a.m, lane, want, d, tx);
            }
            write_vector(d, wb, a.tv.first, lane, gbase + off[j0 + bit], pos, cap);
        }
    }
    __syncthreads();
    // leave the group's scratch zeroed for the next report: every nonzero
    // per-vector count lies in a group with a nonzero sum, so after the pass
    // both arrays are all zero again
#pragma unroll
    for (uint32_t i = 0; i < kGroupBlocks / kWG; ++i)
        if (c[i])
            bc[b0 + (kGroupBlocks / kWG) * tid + i] = 0u;
    if (tid == 0)
        gs[g] = 0ull;
}

__global__ __launch_bounds__(kWG) void k_report_write(CountArgs a, uint32_t *bc,
                                                     unsigned long long *gs, const unsigned long long *go,
                                                     uint64_t ngroups, unsigned long long *pos, uint64_t cap,
                                                     uint32_t win)
{
    extern __shared__ __align__(16) uint8_t wlds[];
    __shared__ uint32_t off[kGroupBlocks];
    __shared__ uint32_t wsum[kWaves];
    uint8_t *mine = wlds + wave_id() * win;
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x)
        report_write_group(a, bc, gs, go, g, pos, cap, win, mine, off, wsum);
}

// Reporting batch: the group offsets of every query (one workgroup of 1024
// threads per query, as k_scan_groups) ...
__global__ __launch_bounds__(1024) void k_scan_groups_multi(const RepDesc *descs)
{
    __shared__ unsigned long long part[1024];
    const RepDesc D = ldc(&descs[blockIdx.x]);
    const uint32_t tid = threadIdx.x;
    const uint64_t ng = D.ngroups, per = (ng + 1023u) / 1024u;
    const uint64_t b0 = min((uint64_t)tid * per, ng), b1 = min(b0 + per, ng);
    unsigned long long s = 0;
    for (uint64_t i = b0; i < b1; ++i)
        s += D.gs[i];
    part[tid] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024u; o <<= 1) {
        const unsigned long long v = tid >= o ? part[tid - o] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned long long run = tid ? part[tid - 1] : 0ull;
    for (uint64_t i = b0; i < b1; ++i) {
        D.go[i] = run;
        run += D.gs[i];
    }
    if (tid == 1023u)
        *D.total = part[1023];
}

// ... and the ordered writes of all their groups: work item i is group
// i - descs[q].item0 of query q = item_query[i].
__global__ __launch_bounds__(kWG) void k_report_write_multi(const RepDesc *descs, const uint32_t *item_query,
                                                           uint64_t nitems)
{
    extern __shared__ __align__(16) uint8_t wlds[];
    __shared__ uint32_t off[kGroupBlocks];
    __shared__ uint32_t wsum[kWaves];
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const RepDesc D = ldc(&descs[ldc(&item_query[it])]);
        CountArgs a{};
        a.tv = D.tv;
        a.last = D.last;
        a.nblocks = D.nblocks;
        a.steps = D.steps;
        a.m = D.m;
        report_write_group(a, D.bc, D.gs, D.go, it - D.item0, D.pos, D.cap, D.win, wlds + wave_id() * D.win,
                           off, wsum);
    }
}

// ------------------------------------------------------------- histogram

// Symbol frequencies (Section 2.2).  Every lane of a wave owns a private copy
// of the 256 bins, laid out bin-major ([bin][lane], 64 KiB per workgroup), so
// the 64 lanes of an LDS atomic never share an address and consecutive lanes
// hit consecutive banks whatever the byte values: a skewed text costs the same
// as a uniform one.  The 16 waves of the workgroup share the 64 copies.  At
// the end each bin's 64 copies are summed and added to the global histogram
// with one 64-bit atomic per nonzero bin and workgroup.
__device__ __forceinline__ void hist_add16(uint8_t *hb, uint32_t lane4, uint4 v)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t bin = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
        atomicAdd(reinterpret_cast<uint32_t *>(hb + (bin << 8) + lane4), 1u);
    }
}

// 16 text bytes, with the streaming (non-temporal) cache policy if STREAM.
template <bool STREAM>
__device__ __forceinline__ uint4 load16(const uint8_t *p)
{
    if constexpr (STREAM) {
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const uint4 *>(p);
    }
}

template <bool STREAM>
__global__ __launch_bounds__(kHistWG) void k_hist(TextView tv, unsigned long long *hist)
{
    extern __shared__ __align__(16) uint32_t h[];  // [256][64]
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    for (uint32_t i = tid; i < 256u * 64u / 4u; i += kHistWG)
        reinterpret_cast<uint4 *>(h)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    uint8_t *hb = reinterpret_cast<uint8_t *>(h);
    const uint32_t lane4 = lane * 4u;
    const uint64_t lo = tv.first, hi = tv.first + tv.n;
    // interior chunks [c_lo, c_hi) hold text bytes only; the (at most two) edge chunks are masked
    const uint64_t c_lo = (lo + 15u) / 16u, c_hi = hi / 16u;
    const uint64_t stride = (uint64_t)gridDim.x * kHistWG;
    uint64_t c = c_lo + (uint64_t)blockIdx.x * kHistWG + tid;
    for (; c + stride < c_hi; c += 2 * stride) {
        const uint4 v0 = load16<STREAM>(tv.base + 16u * c);
        const uint4 v1 = load16<STREAM>(tv.base + 16u * (c + stride));
        hist_add16(hb, lane4, v0);
        hist_add16(hb, lane4, v1);
    }
    if (c < c_hi)
        hist_add16(hb, lane4, load16<STREAM>(tv.base + 16u * c));
    if (blockIdx.x == 0 && tid < 2u) {
        // edge chunks: the one holding the first bytes (if the text starts mid-chunk) and the one
        // holding the last bytes (if it ends mid-chunk and is not that same chunk)
        const uint64_t e_first = lo / 16u, e_last = hi / 16u;
        const bool has_first = lo % 16u != 0u;
        const bool has_last = hi % 16u != 0u && !(has_first && e_last == e_first);
        const uint64_t e = tid == 0u ? e_first : e_last;
        if (tid == 0u ? has_first : has_last) {
            const uint4 v = *reinterpret_cast<const uint4 *>(tv.base + 16u * e);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            for (int i = 0; i < 16; ++i) {
                const uint64_t u = 16u * e + (uint64_t)i;
                if (u >= lo && u < hi) {
                    const uint32_t bin = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                    atomicAdd(reinterpret_cast<uint32_t *>(hb + (bin << 8) + lane4), 1u);
                }
            }
        }
    }
    __syncthreads();
    // four threads per bin, 16 copies each (rotated start spreads the banks), then a quad reduction
    const uint32_t bin = tid >> 2, part = tid & 3u;
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < 16u; ++k)
        sum += h[bin * 64u + part * 16u + ((k + bin) & 15u)];
    sum += dpp_mov<0xb1, 0xf>(sum, 0u);  // quad_perm [1,0,3,2]
    sum += dpp_mov<0x4e, 0xf>(sum, 0u);  // quad_perm [2,3,0,1]
    if (part == 0u && sum)
        atomicAdd(&hist[bin], (unsigned long long)sum);
}

// Adjacent-pair counts for the bigram-aware compare order: out[a * 256 + b]
// += number of s with t[s] == a, t[s+1] == b, for the first symbols a in
// [128 * half, 128 * half + 128).  A 1024-thread workgroup (one per CU) keeps
// that half of the table, 128 x 256 counters, in LDS and adds its nonzero
// counters to the global table at the end.  Each thread takes 16-byte chunks;
// the byte after a chunk comes from a one-byte load (usually cached).
__device__ __forceinline__ void bigram_add(uint32_t *tab, uint32_t half, uint32_t a, uint32_t b)
{
    if ((a >> 7) == half)
        atomicAdd(&tab[((a & 127u) << 8) | b], 1u);
}

__global__ __launch_bounds__(kBgWG) void k_bigram(TextView tv, uint32_t half, unsigned long long *out)
{
    extern __shared__ __align__(16) uint32_t tab[];  // [128][256]
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < 128u * 256u / 4u; i += kBgWG)
        reinterpret_cast<uint4 *>(tab)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const uint64_t lo = tv.first, hi = tv.first + tv.n;  // pairs start at s in [lo, hi - 1)
    if (hi >= lo + 2) {
        const uint64_t c0 = lo / 16u, c1 = (hi - 2) / 16u + 1;  // chunks holding a pair start
        for (uint64_t c = c0 + (uint64_t)blockIdx.x * kBgWG + tid; c < c1; c += (uint64_t)gridDim.x * kBgWG) {
            const uint64_t u = 16u * c;
            const uint4 v = *reinterpret_cast<const uint4 *>(tv.base + u);
            const uint32_t nb = u + 16u < hi ? (uint32_t)tv.base[u + 16u] : 0u;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            if (u >= lo && u + 16u < hi) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint32_t a = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                    const uint32_t b = i < 15 ? (w[(i + 1) >> 2] >> (8 * ((i + 1) & 3))) & 0xFFu : nb;
                    bigram_add(tab, half, a, b);
                }
            } else {
                for (int i = 0; i < 16; ++i) {
                    const uint64_t s = u + (uint64_t)i;
                    if (s < lo || s + 1u >= hi)
                        continue;
                    const uint32_t a = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                    const uint32_t b = i < 15 ? (w[(i + 1) >> 2] >> (8 * ((i + 1) & 3))) & 0xFFu : nb;
                    bigram_add(tab, half, a, b);
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < 128u * 256u; i += kBgWG) {
        const uint32_t v = tab[i];
        if (v)
            atomicAdd(&out[(uint64_t)half * 32768u + i], (unsigned long long)v);
    }
}

// Zeroes the per-vector counts (16-byte stores; bc is 16-byte aligned) and the group sums.
__global__ void k_fill_report(uint32_t *bc, uint64_t n, unsigned long long *gs, uint64_t ng)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n4 = n / 4;
    uint4 *p4 = reinterpret_cast<uint4 *>(bc);
    for (uint64_t i = tid; i < n4; i += nt)
        p4[i] = make_uint4(0, 0, 0, 0);
    for (uint64_t i = 4 * n4 + tid; i < n; i += nt)
        bc[i] = 0u;
    for (uint64_t i = tid; i < ng; i += nt)
        gs[i] = 0ull;
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ batch kernel

// Persistent batched count over byte tiles.  All chunks' tiles form one
// global tile space dealt out like the single search (2^chunk_log2 tiles per
// deal, round robin), with the same double-buffered LDS DMA; the next tile
// may belong to another text.  Every query of the tile's chunk runs over the
// staged tile; per-query counts gather in LDS and are flushed (one 64-bit
// atomicAdd per nonzero query) whenever the workgroup moves to another chunk.
template <int CPL, bool REPORT, bool STREAM>
__global__ __launch_bounds__(kWG) void k_batch_staged(BatchArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t T = kWG * 16u * CPL;
    constexpr int kPolicy = STREAM ? kLoadStream : kLoadDefault;
    const uint32_t TB = T + a.halo_max;
    uint32_t *qc = reinterpret_cast<uint32_t *>(lds + 2u * TB);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    const uint64_t kmask = (1ull << a.chunk_log2) - 1u;
    auto tile_of = [&](uint64_t i) {
        return (((uint64_t)blockIdx.x + (i >> a.chunk_log2) * gridDim.x) << a.chunk_log2) + (i & kmask);
    };
    auto flush = [&](uint32_t c) {
        const BatchChunk C = ldc(&a.chunks[c]);
        for (uint32_t i = tid; i < C.q_end - C.q_begin; i += kWG) {
            const uint32_t v = qc[i];
            if (v)
                atomicAdd(&a.counts[a.queries[C.q_begin + i].out], (unsigned long long)v);
        }
    };

    uint64_t g = tile_of(0);
    if (g < a.ntiles) {
        const BatchChunk C = ldc(&a.chunks[ldc(&a.tile_chunk[g])]);
        dma_tile<CPL, kPolicy>(C.tv, (g - C.tile0) * T, tid, C.halo >> 4, lds);
    }
    uint32_t cur = 0xFFFFFFFFu;
    for (uint64_t i = 0; g < a.ntiles; ++i) {
        const uint32_t c = ldc(&a.tile_chunk[g]);
        const BatchChunk C = ldc(&a.chunks[c]);
        const uint64_t ts = (g - C.tile0) * T;
        uint8_t *buf = lds + (i & 1u) * TB;
        const uint64_t gn = tile_of(i + 1);
        wait_dma();
        __syncthreads();  // tile visible; the other buffer is free
        if (c != cur) {
            if (cur != 0xFFFFFFFFu)
                flush(cur);
            __syncthreads();
            for (uint32_t k = tid; k < C.q_end - C.q_begin; k += kWG)
                qc[k] = 0u;
            __syncthreads();
            cur = c;
        }
        if (gn < a.ntiles) {
            const BatchChunk N = ldc(&a.chunks[ldc(&a.tile_chunk[gn])]);
            dma_tile<CPL, kPolicy>(N.tv, (gn - N.tile0) * T, tid, N.halo >> 4, lds + ((i + 1) & 1u) * TB);
        }
        for (uint32_t q = C.q_begin; q < C.q_end; ++q) {
            const BatchQuery Q = ldc(&a.queries[q]);
            const uint64_t *st = a.steps + Q.steps_off;
            uint32_t cnt = 0;
#pragma unroll 1
            for (int b = 0; b < CPL; ++b) {
                const uint32_t boff = (wave * CPL + b) * kBlock;
                const uint64_t wb = ts + boff;
                if (wb > Q.last)
                    break;
                uint32_t d[4];
                init_alive(wb, C.tv.first, Q.last, lane, d);
                const LdsText tx{buf + boff, buf + boff + 4u * lane};
                if (search_vector_rt(st, Q.r, Q.m, lane, d, tx)) {
                    const uint32_t c = count_alive(d);
                    cnt += c;
                    if constexpr (REPORT) {  // per-vector count for the ordered write
                        const BatchReport P = ldc(&a.reports[q]);
                        const uint32_t sv = wave_sum32(c);
                        if (lane == 0 && sv) {
                            P.block_counts[wb / kBlock] = sv;
                            atomicAdd(&P.group_sums[wb / kBlock / kGroupBlocks], (unsigned long long)sv);
                        }
                    }
                }
            }
            if (__any(cnt != 0u)) {
                const uint32_t s = wave_sum32(cnt);
                if (lane == 0)
                    atomicAdd(&qc[q - C.q_begin], s);
            }
        }
        g = gn;
    }
    __syncthreads();
    if (cur != 0xFFFFFFFFu)
        flush(cur);
}

// The vectors of wave `wave` in a staged tile with valid tile offsets lo..hi, searched with a
// compile-time peel R; returns the lane's count.
template <int CPL, int R>
__device__ __forceinline__ uint32_t search_tile(const uint64_t *steps, uint32_t m, const uint8_t *cur, uint32_t wave,
                                                uint32_t lane, uint32_t lo, uint32_t hi)
{
    uint64_t pk[R];
#pragma unroll
    for (int l = 0; l < R; ++l)
        pk[l] = ldc(&steps[l]);
    uint32_t acc = 0;
#pragma unroll
    for (int b = 0; b < CPL; ++b) {
        const uint32_t boff = (wave * CPL + b) * kBlock;
        if (boff > hi)
            break;
        uint32_t d[4];
        const bool edge = boff < lo || boff + (kBlock - 1u) > hi;
        const LdsText tx{cur + boff, cur + boff + 4u * lane};
        if (search_vector_tile<R>(steps, pk, m, lane, d, tx, edge, boff, lo, hi))
            acc += count_alive(d);
    }
    return acc;
}

// Persistent batched count of single-query chunks.  Deal k (up to 2^chunk_log2
// consecutive tiles of one query's text) goes to workgroup k mod G; the deal
// names its query's record (text, step table, peel, bounds, output slot).  The
// tiles are staged by the same double-buffered LDS DMA as the single search,
// the next tile (possibly the next deal's first) in flight while one is
// searched, with the peel compiled in (a switch on the query's r).  The next
// deal's records are loaded one deal ahead.  The count stays in registers over
// a deal and is added to its output once per wave.
struct DealView {
    BatchSolo S;
    uint64_t ts0;  // coordinate of the deal's first tile
    uint32_t ntiles;
};

template <int CPL>
__device__ __forceinline__ DealView load_deal(const DealArgs &a, uint64_t k)
{
    constexpr uint32_t T = kWG * 16u * CPL;
    const BatchDeal D = ldc(&a.deals[k]);
    DealView v;
    v.S = ldc(&a.solos[D.solo]);
    v.ts0 = (uint64_t)(D.tiles >> 3) * T;
    v.ntiles = D.tiles & 7u;
    return v;
}

template <int CPL, bool STREAM>
__global__ __launch_bounds__(kWG) void k_batch_deals(DealArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t T = kWG * 16u * CPL;
    constexpr int kPolicy = STREAM ? kLoadStream : kLoadDefault;
    const uint32_t TB = T + a.halo_max;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    uint64_t k = blockIdx.x;
    if (k >= a.ndeals)
        return;
    DealView D = load_deal<CPL>(a, k);
    DealView N = k + gridDim.x < a.ndeals ? load_deal<CPL>(a, k + gridDim.x) : D;
    dma_tile<CPL, kPolicy>(D.S.tv, D.ts0, tid, D.S.halo >> 4, lds);
    uint32_t acc = 0;
    uint32_t t = 0;  // tile of the deal
    for (uint64_t i = 0;; ++i) {
        uint8_t *cur = lds + (i & 1u) * TB;
        const bool more = t + 1u < D.ntiles;
        const bool next_deal = k + gridDim.x < a.ndeals;
        wait_dma();
        __syncthreads();  // tile visible to all waves; the other buffer is free
        if (more)
            dma_tile<CPL, kPolicy>(D.S.tv, D.ts0 + (uint64_t)(t + 1u) * T, tid, D.S.halo >> 4,
                                   lds + ((i + 1) & 1u) * TB);
        else if (next_deal)
            dma_tile<CPL, kPolicy>(N.S.tv, N.ts0, tid, N.S.halo >> 4, lds + ((i + 1) & 1u) * TB);
        // the tile's valid starts as 32-bit tile offsets lo..hi (the deal's tiles all hold one)
        const uint64_t ts = D.ts0 + (uint64_t)t * T;
        const uint64_t rem = D.S.last - ts;
        const uint32_t hi = rem >= T ? T - 1u : (uint32_t)rem;
        const uint32_t lo = ts < D.S.tv.first ? (uint32_t)(D.S.tv.first - ts) : 0u;
        const uint64_t *st = D.S.steps;
        const uint32_t m = D.S.m;
        switch (D.S.r) {
        case 1: acc += search_tile<CPL, 1>(st, m, cur, wave, lane, lo, hi); break;
        case 2: acc += search_tile<CPL, 2>(st, m, cur, wave, lane, lo, hi); break;
        case 3: acc += search_tile<CPL, 3>(st, m, cur, wave, lane, lo, hi); break;
        case 4: acc += search_tile<CPL, 4>(st, m, cur, wave, lane, lo, hi); break;
        case 5: acc += search_tile<CPL, 5>(st, m, cur, wave, lane, lo, hi); break;
        case 6: acc += search_tile<CPL, 6>(st, m, cur, wave, lane, lo, hi); break;
        case 7: acc += search_tile<CPL, 7>(st, m, cur, wave, lane, lo, hi); break;
        default: acc += search_tile<CPL, 8>(st, m, cur, wave, lane, lo, hi); break;
        }
        if (more) {
            ++t;
            continue;
        }
        if (__any(acc != 0u)) {  // end of the deal: its count (< 2^32 starts) once per wave
            const uint32_t c = wave_sum32(acc);
            if (lane == 0)
                atomicAdd(&a.counts[D.S.out], (unsigned long long)c);
        }
        acc = 0;
        if (!next_deal)
            break;
        k += gridDim.x;
        D = N;
        if (k + gridDim.x < a.ndeals)
            N = load_deal<CPL>(a, k + gridDim.x);
        t = 0;
    }
}

// ----------------------------------------------------- non-overlapping mode
//
// Disjoint occurrences by greedy leftmost selection over the ascending list of
// all occurrences pos[0..c): take pos[0]; after taking pos[i], take the first
// occurrence at or after pos[i] + m.  nxt[i] is that successor of i (c if
// none), so the taken set is the chain 0, nxt[0], nxt[nxt[0]], ...
// An occurrence at least m after its predecessor in the list starts a cluster
// and is always taken (the last start taken before it is at most its
// predecessor, and every occurrence in between lies within m of that start),
// so the chain is found cluster by cluster.  Pointer doubling marks it: the
// cluster starts are marked first; round k marks nxt^(2^k)(i) of every marked
// i and squares the jump, so ceil(log2 L) rounds cover clusters of up to L
// occurrences.  A mark set early in a round is still on the chain, so the
// order within a round does not matter.

__device__ __forceinline__ bool no_taken(const uint32_t *mark, uint64_t i)
{
    return mark[i] != 0u;
}

// Successors, cluster-start marks, and the number of entries that are not
// cluster starts (added to *overlapped).
__global__ __launch_bounds__(kWG) void k_no_next(const unsigned long long *pos, uint64_t c, uint32_t m, uint32_t *nxt,
                                                 uint32_t *mark, unsigned long long *overlapped)
{
    uint32_t ov = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < c; i += (uint64_t)gridDim.x * kWG) {
        const unsigned long long target = pos[i] + m;
        uint64_t lo = i + 1, hi = c;  // first index in [lo, hi) with pos >= target
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (pos[mid] < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        nxt[i] = (uint32_t)lo;
        const bool start = i == 0 || pos[i] - pos[i - 1] >= m;
        mark[i] = start ? 1u : 0u;
        ov += start ? 0u : 1u;
    }
    const uint32_t s = wave_sum32(ov);
    if ((threadIdx.x & 63u) == 0 && s)
        atomicAdd(overlapped, (unsigned long long)s);
}

__global__ __launch_bounds__(kWG) void k_no_mark(const uint32_t *nxt, uint32_t *mark, uint64_t c)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < c; i += (uint64_t)gridDim.x * kWG) {
        if (no_taken(mark, i)) {
            const uint32_t j = nxt[i];
            if (j < c)
                mark[j] = 1u;
        }
    }
}

__global__ __launch_bounds__(kWG) void k_no_jump(const uint32_t *in, uint32_t *out, uint64_t c)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < c; i += (uint64_t)gridDim.x * kWG) {
        const uint32_t j = in[i];
        out[i] = j < c ? in[j] : (uint32_t)c;
    }
}

// Taken elements per chunk of kNoChunkEntries list entries (four consecutive per thread).

__global__ __launch_bounds__(kWG) void k_no_chunk_counts(const uint32_t *mark, uint64_t c, unsigned long long *gs,
                                                         uint64_t ng)
{
    __shared__ uint32_t ws[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    for (uint64_t g = blockIdx.x; g < ng; g += gridDim.x) {
        const uint64_t i0 = g * kNoChunkEntries + 4u * tid;
        uint32_t k = 0;
#pragma unroll
        for (uint32_t e = 0; e < 4u; ++e)
            k += (i0 + e < c && no_taken(mark, i0 + e)) ? 1u : 0u;
        const uint32_t s = wave_sum32(k);
        if (lane == 0)
            ws[wave] = s;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (uint32_t w = 0; w < kWaves; ++w)
                t += ws[w];
            gs[g] = t;
        }
        __syncthreads();
    }
}

// Writes the taken starts of each chunk at its exclusive offset go[g], in list
// order (thread-major, four entries per thread), keeping the first cap.
__global__ __launch_bounds__(kWG) void k_no_compact(const unsigned long long *pos, const uint32_t *mark, uint64_t c,
                                                    const unsigned long long *go, uint64_t ng,
                                                    unsigned long long *out, uint64_t cap)
{
    __shared__ uint32_t ws[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id();
    for (uint64_t g = blockIdx.x; g < ng; g += gridDim.x) {
        const uint64_t i0 = g * kNoChunkEntries + 4u * tid;
        uint32_t take = 0;  // bit e: entry i0 + e is taken
#pragma unroll
        for (uint32_t e = 0; e < 4u; ++e)
            if (i0 + e < c && no_taken(mark, i0 + e))
                take |= 1u << e;
        const uint32_t k = (uint32_t)__popc(take);
        uint32_t inc = k;  // inclusive prefix over the wave's lanes
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o)
                inc += v;
        }
        if (lane == 63u)
            ws[wave] = inc;
        __syncthreads();
        uint64_t off = go[g] + (inc - k);
        for (uint32_t w = 0; w < wave; ++w)
            off += ws[w];
#pragma unroll
        for (uint32_t e = 0; e < 4u; ++e) {
            if (take & (1u << e)) {
                if (off < cap)
                    out[off] = pos[i0 + e];
                ++off;
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------- batch bitmap kernel

// One compare on the bitmaps for the kBmV 2048-start vectors of the tile:
// bits of the window at offset j are a funnel shift of two bitmap words.  e is
// a bitmap step entry: e >> 5 is the LDS byte offset of the slot word holding
// bit j, and alignbit uses only the low five bits of its shift operand, which
// are j mod 32.  lane4 = 4 * lane.
__device__ __forceinline__ void bm_step(const uint8_t *bmb, uint32_t e, uint32_t lane4, uint32_t (&f)[kBmV])
{
    const uint32_t *w = reinterpret_cast<const uint32_t *>(bmb + (e >> 5) + lane4);
#pragma unroll
    for (int v = 0; v < kBmV; ++v)
        f[v] &= __builtin_amdgcn_alignbit(w[64 * v + 1], w[64 * v], e);
}

// Wave-uniform: any start of the tile still alive?
__device__ __forceinline__ bool bm_any(const uint32_t (&f)[kBmV])
{
    uint32_t o = 0;
#pragma unroll
    for (int v = 0; v < kBmV; ++v)
        o |= f[v];
    return __any(o != 0u);
}

__device__ __forceinline__ uint32_t bm_popc(const uint32_t (&f)[kBmV])
{
    uint32_t c = 0;
#pragma unroll
    for (int v = 0; v < kBmV; ++v)
        c += __popc(f[v]);
    return c;
}

// Bits of the 32 tile offsets o .. o + 31 that lie in [a, b) (tile offsets, all below 2^31).
__device__ __forceinline__ uint32_t range_bits(uint32_t o, uint32_t a, uint32_t b)
{
    const uint32_t lo = a > o ? min(a - o, 32u) : 0u, hi = b > o ? min(b - o, 32u) : 0u;
    if (lo >= hi)
        return 0u;
    return (hi >= 32u ? 0xFFFFFFFFu : (1u << hi) - 1u) & ~((1u << lo) - 1u);
}

// Coordinate c as a tile offset from ts, clamped to [0, 2^20].
__device__ __forceinline__ uint32_t tile_off(uint64_t c, uint64_t ts)
{
    return c > ts ? (uint32_t)min(c - ts, (uint64_t)1 << 20) : 0u;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// Persistent batched count over bitmap tiles.  Work item = (text, tile range,
// chunk of queries).  The item's query records go to LDS once.  Per tile:
// zero the bitmaps, set one bit per text byte of a symbol some query uses (LDS
// atomic OR; the bytes were loaded into registers while the previous tile was
// searched), then each wave runs groups of K queries over the kBmT starts of
// the tile: the first min(r) compares of the K queries in lock step, so that
// the LDS reads of all K are in flight together, then per query its remaining
// peeled compares and one zero test (a wave-wide ballot) after each further
// compare (Algorithm 4).  A group's records are read from LDS by K * 8 lanes
// and their fields taken with readlane, so the loop issues no scalar memory
// loads, whose out-of-order returns would make every LDS wait a full one (only
// compares past the record's first entries read the step pool).  Each query's
// count for the item gathers in an LDS counter owned by one wave.
template <int K>
__device__ __forceinline__ void batch_bitmap(const BmArgs &a)
{
    static_assert(K * kBmRecWords <= 64, "a group's records fit one wave");
    extern __shared__ __align__(16) uint32_t bmlds[];
    uint32_t *lds = bmlds;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = wave_id(), lane4 = 4u * lane;
    const uint8_t *bmb = reinterpret_cast<const uint8_t *>(lds);
    for (uint64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const BmItem I = ldc(&a.items[it]);
        const uint32_t nq = I.q_end - I.q_begin, wps = I.wps, bm_words = I.nslots * wps;
        uint32_t *bm = lds;
        uint32_t *smap = lds + bm_words;          // symbol -> first word of its slot, or ~0
        uint32_t *rec = smap + 256;               // kBmRecWords per query
        uint32_t *qc = rec + nq * kBmRecWords;    // per-query counts of the item
        uint32_t *next = qc + nq;                 // next query group of the tile
        const uint64_t lo = I.tv.first, hi = I.tv.first + I.tv.n;
        __syncthreads();  // the previous item is done with the LDS
        if (tid < 256u) {
            const uint32_t sl = I.smap[tid];
            smap[tid] = sl == 0xFFu ? 0xFFFFFFFFu : sl * wps;
        }
        for (uint32_t i = tid; i < nq * kBmRecWords; i += kBmWG)
            rec[i] = a.recs[(uint64_t)I.q_begin * kBmRecWords + i];
        for (uint32_t i = tid; i < nq; i += kBmWG)
            qc[i] = 0u;
        // the tile window's bytes in 8-byte pieces: piece c (window bytes [8c, 8c + 8)) for c = tid and
        // c = tid + kBmWG, held in registers (zero past the text's chunks); 4 * wps pieces in all
        const uint32_t npieces = 4u * wps;
        uint2 tb0 = make_uint2(0, 0), tb1 = make_uint2(0, 0);
        auto load_tile = [&](uint64_t tile) {
            const uint64_t u0 = tile * kBmT + 8ull * tid, u1 = u0 + 8ull * kBmWG;
            tb0 = (tid < npieces && u0 < I.tv.end16) ? *reinterpret_cast<const uint2 *>(I.tv.base + u0) : make_uint2(0, 0);
            tb1 = (tid + kBmWG < npieces && u1 < I.tv.end16) ? *reinterpret_cast<const uint2 *>(I.tv.base + u1)
                                                              : make_uint2(0, 0);
        };
        load_tile(I.tile_begin);
        for (uint64_t tile = I.tile_begin; tile < I.tile_end; ++tile) {
            const uint64_t ts = tile * kBmT;
            for (uint32_t i = tid; i < bm_words / 4u; i += kBmWG)
                reinterpret_cast<uint4 *>(bm)[i] = make_uint4(0, 0, 0, 0);
            if (tid == 0)
                *next = 0u;
            __syncthreads();
            // text bytes lie at tile offsets [blo, bhi)
            const uint32_t blo = tile_off(lo, ts), bhi = tile_off(hi, ts);
            auto build = [&](uint32_t c, uint2 v) {  // piece c: eight lookups in flight, then their bits
                const uint32_t valid = range_bits(32u * (c >> 2), blo, bhi) >> (8u * (c & 3u));
                const uint32_t w[2] = {v.x, v.y};
                uint32_t base[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    base[i] = smap[(w[i >> 2] >> (8 * (i & 3))) & 0xFFu];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (base[i] != 0xFFFFFFFFu && ((valid >> i) & 1u))
                        atomicOr(&bm[base[i] + (c >> 2)], 1u << (8u * (c & 3u) + i));
            };
            if (tid < npieces)
                build(tid, tb0);
            if (tid + kBmWG < npieces)
                build(tid + kBmWG, tb1);
            __syncthreads();
            if (tile + 1u < I.tile_end)
                load_tile(tile + 1u);  // in flight while this tile is searched
            const bool inner = ts >= lo && ts + (kBmT - 1u) <= I.last_min;  // every start valid for every query
            const uint32_t ngroups = (nq + (uint32_t)K - 1u) / (uint32_t)K;
            // groups are taken from a counter, so that waves whose queries end early take more;
            // a group's records are read one group ahead
            auto take = [&]() -> uint32_t {
                uint32_t g = 0;
                if (lane == 0)
                    g = atomicAdd(next, 1u);
                return readlane(g, 0);
            };
            auto load_rec = [&](uint32_t g) -> uint32_t {
                // lanes 8i .. 8i + 7 hold query gK + i's record; past the chunk, the last query's
                const uint32_t qi = min(g * (uint32_t)K + lane / kBmRecWords, nq - 1u);
                return (g < ngroups && lane < (uint32_t)K * kBmRecWords) ? rec[qi * kBmRecWords + lane % kBmRecWords]
                                                                          : 0u;
            };
            uint32_t g = take();
            uint32_t rv_next = load_rec(g);
            while (g < ngroups) {
                const uint32_t q0 = g * (uint32_t)K;
                const uint32_t rv = rv_next;
                g = take();
                rv_next = load_rec(g);
                uint32_t mr[K], f[K][kBmV];
                uint32_t rmin = kMaxPeel;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    mr[i] = readlane(rv, (uint32_t)i * kBmRecWords);
                    rmin = min(rmin, mr[i] >> 24);
                }
                // the first compare sets f; on edge tiles it is then masked to the query's valid starts.
                // When the group's K first compares read the same two words per lane (same slot and
                // j / 32: the planner sorts a chunk's queries by that key, so most groups do), the
                // words are loaded once and only the shifts differ.
                uint32_t e0[K];
                bool shared = true;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    e0[i] = readlane(rv, (uint32_t)i * kBmRecWords + 2u);
                    shared &= (e0[i] >> 7) == (e0[0] >> 7);
                }
                if (shared) {
                    const uint32_t *w = reinterpret_cast<const uint32_t *>(bmb + (e0[0] >> 5) + lane4);
                    uint32_t lo[kBmV], hi[kBmV];
#pragma unroll
                    for (int v = 0; v < kBmV; ++v)
                        lo[v] = w[64 * v], hi[v] = w[64 * v + 1];
#pragma unroll
                    for (int i = 0; i < K; ++i)
#pragma unroll
                        for (int v = 0; v < kBmV; ++v)
                            f[i][v] = __builtin_amdgcn_alignbit(hi[v], lo[v], e0[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        const uint32_t *w = reinterpret_cast<const uint32_t *>(bmb + (e0[i] >> 5) + lane4);
#pragma unroll
                        for (int v = 0; v < kBmV; ++v)
                            f[i][v] = __builtin_amdgcn_alignbit(w[64 * v + 1], w[64 * v], e0[i]);
                    }
                }
                if (!inner) {
#pragma unroll
                    for (int i = 0; i < K; ++i) {  // valid starts at tile offsets [blo, last + 1)
                        const uint32_t shi = tile_off(hi - (mr[i] & 0xFFFFFFu) + 1u, ts);
#pragma unroll
                        for (int v = 0; v < kBmV; ++v)
                            f[i][v] &= range_bits(2048u * v + 32u * lane, blo, shi);
                    }
                }
                const uint32_t rl = min(rmin, kBmRecSteps);
                for (uint32_t l = 1; l < rl; ++l) {
#pragma unroll
                    for (int i = 0; i < K; ++i)
                        bm_step(bmb, readlane(rv, (uint32_t)i * kBmRecWords + 2u + l), lane4, f[i]);
                }
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    if (q0 + (uint32_t)i >= nq)
                        continue;
                    const uint32_t m = mr[i] & 0xFFFFFFu, r = mr[i] >> 24;
                    const uint32_t rb = (uint32_t)i * kBmRecWords;
                    auto entry = [&](uint32_t l) -> uint32_t {
                        return l < kBmRecSteps ? readlane(rv, rb + 2u + l) : ldc(&a.steps[readlane(rv, rb + 1u) + l]);
                    };
                    uint32_t l = rl;
                    for (; l < r; ++l)
                        bm_step(bmb, entry(l), lane4, f[i]);
                    bool alive = bm_any(f[i]);
                    for (; alive && l < m; ++l) {
                        bm_step(bmb, entry(l), lane4, f[i]);
                        alive = bm_any(f[i]);
                    }
                    if (alive) {
                        const uint32_t c = wave_sum32(bm_popc(f[i]));
                        if (lane == 0)
                            qc[q0 + (uint32_t)i] += c;
                    }
                }
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < nq; i += kBmWG) {
            const uint32_t v = qc[i];
            if (v)
                atomicAdd(&a.counts[a.outs[I.q_begin + i]], (unsigned long long)v);
        }
    }
}

__global__ __launch_bounds__(kBmWG) void k_batch_bitmap(BmArgs a)
{
    batch_bitmap<8>(a);
}

// The same for items whose LDS leaves room for two workgroups per CU (small
// alphabets): registers capped at 64 per lane so that both are resident (8
// waves per SIMD), which hides more of the latency of small alphabets' long
// tails; groups of two queries keep the peel's reads within the cap.
__global__ __launch_bounds__(kBmWG) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_bitmap2(BmArgs a)
{
    batch_bitmap<2>(a);
}

// ------------------------------------------------- bitmap single search

// Section 2.1's SIMDcompare of one symbol against every start of a tile,
// memoised: per tile, one bitmap per distinct pattern symbol (a slot), bit q of
// slot c set when the text byte at tile offset q is that symbol; then a compare
// of pattern position j over 32 starts is one funnel shift of two bitmap words
// and an AND.  Pays off when compares per start are many (small alphabets) and
// the pattern has few distinct symbols: the build costs about 2.9 VALU ops per
// text byte for two slots, the compares about 0.13 per start and compare.

// Slot of pattern symbol `sym` among the NS distinct symbols packed in syms.
template <int NS>
__device__ __forceinline__ uint32_t bc_slot(uint32_t syms, uint32_t sym)
{
    uint32_t c = 0;
#pragma unroll
    for (int s = 1; s < NS; ++s)
        if (((syms >> (8 * s)) & 0xFFu) == sym)
            c = (uint32_t)s;
    return c;
}

// Bitmap step entries of compares 64k .. 64k + 63, entry of compare 64k + i in
// lane i: ((slot * W + (j >> 5)) << 7) | (j & 31), i.e. the slot word holding
// bit j (its word index shifted left by 7) and j mod 32.  Lanes past m hold 0
// (never read: the compares stop at m).
template <int NS, uint32_t W>
__device__ __forceinline__ uint32_t bc_entries(const BmCountArgs &a, uint32_t k, uint32_t lane)
{
    const uint32_t l = 64u * k + lane;
    if (l >= a.m)
        return 0u;
    const uint64_t st = a.steps[l];
    const uint32_t j = step_pos(st), c = bc_slot<NS>(a.syms, step_rep(st) & 0xFFu);
    return ((c * W + (j >> 5)) << 7) | (j & 31u);
}

// One bitmap word per slot from the 32 text bytes D (byte b of D[i] at offset
// 4i + b): bit q set when byte q is the slot's symbol.  First the two 4 x 4
// byte transposes of (D0, D2, D4, D6) and (D1, D3, D5, D7), so that byte k of
// E[d] is the byte at offset 8k + d; then, for one or two slots, per slot an
// exact byte-equality test of each E[d] (0x80 in each byte that differs) and a
// rotate that puts byte k's flag at bit 8k + d (about 41 VALU ops per slot);
// for three or four slots, bit planes of the 32 bytes (about 60 ops once) and
// 8 ops per slot.  out: the word of each slot.  With D[0..3] and D[4..7] two
// separate 16-byte pieces, bits 0..15 of a word are the first piece's offsets
// and bits 16..31 the second's.
// One stage of the 8 x 8 bit transposes: rows d and d + SH (d without the SH bit) exchange the
// bit columns b + SH of row d and b of row d + SH (b without the SH bit), in every byte lane.
template <int SH>
__device__ __forceinline__ void bc_butterfly(uint32_t (&E)[8], uint32_t msk)
{
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        if (d & SH)
            continue;
        const uint32_t t = ((E[d] >> SH) ^ E[d + SH]) & msk;
        E[d + SH] ^= t;
        E[d] ^= t << SH;
    }
}

// Per slot and bit b, all ones when bit b of the slot's symbol is set (the bit-sliced build's masks),
// computed once per kernel as wave-uniform values.
template <int NS>
struct BcPlaneMasks {
    uint32_t c[NS][8];
};

template <int NS>
__device__ __forceinline__ BcPlaneMasks<NS> bc_plane_masks(uint32_t syms)
{
    BcPlaneMasks<NS> pm;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane((int)(0u - ((syms >> (8 * s + b)) & 1u)));
            // opaque to the optimiser (no instruction): otherwise it knows v is 0 or ~0 and turns each
            // XOR with it into a scalar compare and a select, twice the vector ops
            asm("" : "+s"(v));
            pm.c[s][b] = v;
        }
    return pm;
}

template <int NS>
__device__ __forceinline__ void bc_build_word(const uint32_t (&D)[8], uint32_t syms, const BcPlaneMasks<NS> &pm,
                                              uint32_t (&out)[NS])
{
    uint32_t E[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t ablo = __builtin_amdgcn_perm(D[2 + h], D[h], 0x05010400u);
        const uint32_t abhi = __builtin_amdgcn_perm(D[2 + h], D[h], 0x07030602u);
        const uint32_t cdlo = __builtin_amdgcn_perm(D[6 + h], D[4 + h], 0x05010400u);
        const uint32_t cdhi = __builtin_amdgcn_perm(D[6 + h], D[4 + h], 0x07030602u);
        E[4 * h + 0] = __builtin_amdgcn_perm(cdlo, ablo, 0x05040100u);
        E[4 * h + 1] = __builtin_amdgcn_perm(cdlo, ablo, 0x07060302u);
        E[4 * h + 2] = __builtin_amdgcn_perm(cdhi, abhi, 0x05040100u);
        E[4 * h + 3] = __builtin_amdgcn_perm(cdhi, abhi, 0x07060302u);
    }
    if constexpr (NS >= 3) {
        // three or four slots: bit-slice once, then 8 ops per slot.  Three butterfly stages
        // transpose the 8 x 8 bit matrix of each byte lane across E[0..7] (rows: E index, columns:
        // bit within the byte), after which bit 8k + d of E[b] is bit b of the byte at offset 8k + d:
        // E[b] is the word's plane of bit b.  A byte matches symbol c where every plane agrees with
        // c's bit.
        bc_butterfly<4>(E, 0x0F0F0F0Fu);
        bc_butterfly<2>(E, 0x33333333u);
        bc_butterfly<1>(E, 0x55555555u);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            uint32_t miss = 0;
#pragma unroll
            for (int b = 0; b < 8; ++b)
                miss |= E[b] ^ pm.c[s][b];
            out[s] = ~miss;
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint32_t rep = ((syms >> (8 * s)) & 0xFFu) * 0x01010101u;
            uint32_t miss = 0;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const uint32_t x = E[d] ^ rep;
                const uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // bit 8k + 7: byte k differs
                miss |= __builtin_amdgcn_alignbit(y, y, 7u - (uint32_t)d) & (0x01010101u << d);
            }
            out[s] = ~miss;
        }
    }
}

// One compare over the thread's CPW words (words tid + kWG * c of the tile):
// bits j .. j + 31 past each word's first start, a funnel shift of two words.
template <int CPW, bool FIRST>
__device__ __forceinline__ void bc_step(const uint32_t *buf, uint32_t e, uint32_t tid, uint32_t (&f)[CPW])
{
    const uint32_t *w = buf + (e >> 7) + tid;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const uint32_t v = __builtin_amdgcn_alignbit(w[kWG * c + 1], w[kWG * c], e);
        f[c] = FIRST ? v : (f[c] & v);
    }
}

template <int CPW>
__device__ __forceinline__ bool bc_any(const uint32_t (&f)[CPW])
{
    uint32_t o = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        o |= f[c];
    return __any(o != 0u);
}

// Verifies each start still alive in this wave on compares l..m-1, 64
// compares at a time across the lanes (lane i tests compare l + i, then
// l + 64 + i, ...: the bit of the start plus j in its symbol's bitmap), and
// clears the starts that fail.  Only the grouping of the AND changes (by
// start instead of by compare).  Starts are visited in increasing tile offset
// through a wave-uniform cursor.
template <int NS, int CPW, uint32_t W>
__device__ __forceinline__ void bc_verify(const BmCountArgs &a, const uint32_t *buf, uint32_t l, uint32_t tid,
                                          uint32_t (&f)[CPW])
{
    const uint32_t lane = tid & 63u;
    uint32_t cursor = 0;
    while (true) {
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int c = CPW - 1; c >= 0; --c) {
            const uint32_t q0 = 32u * (tid + kWG * c);
            uint32_t z = f[c];
            if (cursor > q0)
                z = cursor - q0 >= 32u ? 0u : z & (0xFFFFFFFFu << (cursor - q0));
            if (z)
                best = q0 + (uint32_t)__builtin_ctz(z);
        }
        best = wave_min32(best);
        if (best == 0xFFFFFFFFu)
            break;
        bool ok = true;
        for (uint32_t b0 = l; ok && b0 < a.m; b0 += 64u) {
            const uint32_t idx = b0 + lane;
            bool bad = false;
            if (idx < a.m) {
                const uint64_t st = a.steps[idx];
                const uint32_t q = best + step_pos(st);
                const uint32_t c = bc_slot<NS>(a.syms, step_rep(st) & 0xFFu);
                bad = ((buf[c * W + (q >> 5)] >> (q & 31u)) & 1u) == 0u;
            }
            ok = !__any(bad);
        }
        const uint32_t w = best >> 5;
        if (!ok && (w & (kWG - 1u)) == tid) {
#pragma unroll
            for (int c = 0; c < CPW; ++c)
                if ((uint32_t)c == w / kWG)
                    f[c] &= ~(1u << (best & 31u));
        }
        cursor = best + 1u;
    }
}

// The 32 text bytes of each word a thread builds, into registers.  Wave w of
// the workgroup builds words 64 (w + 4c) .. + 63 (c < CPW), i.e. 2 KiB of the
// tile per c: lane L loads its 16-byte pieces L and 64 + L of those 2 KiB, so
// that each load instruction of the wave reads 1 KiB contiguously (whole cache
// lines).  A tile wholly inside the text loads without per-chunk bound tests
// (a wave-uniform branch); chunks at or past end16 read as zeros otherwise.
template <int CPW, bool STREAM>
__device__ __forceinline__ void bc_load_tile(const TextView &tv, uint64_t ts, uint32_t tid, uint32_t (&X)[CPW][8])
{
    constexpr uint32_t W = kWG * CPW;
    const uint32_t lane = tid & 63u, wave16 = tid & ~63u;
    if (ts + 32ull * W <= tv.end16) {
        const uint8_t *tb = tv.base + ts;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const uint8_t *q = tb + 32u * (wave16 + kWG * c) + 16u * lane;
            const uint4 lo = load16<STREAM>(q), hi = load16<STREAM>(q + 1024);
            X[c][0] = lo.x, X[c][1] = lo.y, X[c][2] = lo.z, X[c][3] = lo.w;
            X[c][4] = hi.x, X[c][5] = hi.y, X[c][6] = hi.z, X[c][7] = hi.w;
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const uint64_t u = ts + 32ull * (wave16 + kWG * c) + 16u * lane;
        const uint4 lo = u < tv.end16 ? load16<STREAM>(tv.base + u) : make_uint4(0, 0, 0, 0);
        const uint4 hi = u + 1024u < tv.end16 ? load16<STREAM>(tv.base + u + 1024u) : make_uint4(0, 0, 0, 0);
        X[c][0] = lo.x, X[c][1] = lo.y, X[c][2] = lo.z, X[c][3] = lo.w;
        X[c][4] = hi.x, X[c][5] = hi.y, X[c][6] = hi.z, X[c][7] = hi.w;
    }
}

// The tile's slot words from the loaded bytes, stored as half words (16 starts
// each): 2 (wave16 + kWG c) + lane and + 64 of every slot of buf.
template <int NS, int CPW>
__device__ __forceinline__ void bc_build_tile(const uint32_t (&X)[CPW][8], uint32_t syms, const BcPlaneMasks<NS> &pm,
                                              uint32_t *buf, uint32_t tid)
{
    constexpr uint32_t W = kWG * CPW;
    const uint32_t lane = tid & 63u, wave16 = tid & ~63u;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        uint32_t wd[NS];
        bc_build_word<NS>(X[c], syms, pm, wd);
        uint16_t *hb = reinterpret_cast<uint16_t *>(buf) + 2u * (wave16 + kWG * c) + lane;
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            hb[2u * W * sl] = (uint16_t)wd[sl];
            hb[2u * W * sl + 64u] = (uint16_t)(wd[sl] >> 16);
        }
    }
}

// Algorithm 4 over the thread's CPW words of a built tile: its starts at tile
// offsets [lo, hi) (of S; `inner` masks the words with starts when lo = 0 and
// hi = S), the first r compares unconditionally, then the zero test
// (wave-wide) after each of the next kTestEach compares and after each group
// of kGroup later ones, as in the byte-tile kernel; a handful of starts facing
// kVerifyMin or more further compares are verified one at a time across the
// lanes.  Entries of the first 64 compares are in ent0 (readlane); later ones
// are computed per block of 64 when reached.  Returns the thread's matches.
template <int NS, int CPW>
__device__ __forceinline__ uint32_t bc_search_tile(const BmCountArgs &a, const uint32_t *buf, uint32_t ent0,
                                                   uint32_t tid, uint32_t lo, uint32_t hi, uint32_t S,
                                                   const uint32_t (&inner)[CPW])
{
    constexpr uint32_t W = kWG * CPW;
    const uint32_t lane = tid & 63u;
    const uint32_t r = min(a.r, a.m);
    uint32_t f[CPW];
    bc_step<CPW, true>(buf, readlane(ent0, 0), tid, f);
    if (lo == 0u && hi == S) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            f[c] &= inner[c];
    } else {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            f[c] &= range_bits(32u * (tid + kWG * c), lo, hi);
    }
    uint32_t l = 1;
    for (; l < r; ++l)
        bc_step<CPW, false>(buf, readlane(ent0, l), tid, f);
    uint32_t entx = 0, blk = 0;
    auto entry = [&](uint32_t k) {
        if (k < 64u)
            return readlane(ent0, k);
        if ((k >> 6) != blk) {
            blk = k >> 6;
            entx = bc_entries<NS, W>(a, blk, lane);
        }
        return readlane(entx, k & 63u);
    };
    const uint32_t l1 = min(a.m, l + kTestEach);
    for (; l < l1 && bc_any(f); ++l)
        bc_step<CPW, false>(buf, entry(l), tid, f);
    bool grouped = false;
    while (l < a.m && bc_any(f)) {
        if (grouped && a.m - l >= kVerifyMin) {
            uint32_t alive = 0;
#pragma unroll
            for (int c = 0; c < CPW; ++c)
                alive += __popc(f[c]);
            if (wave_sum32(alive) <= kVerifyMax) {
                bc_verify<NS, CPW, W>(a, buf, l, tid, f);
                break;
            }
        }
        const uint32_t g = min(kGroup, a.m - l);
#pragma unroll 1
        for (uint32_t u = 0; u < g; ++u)
            bc_step<CPW, false>(buf, entry(l + u), tid, f);
        l += g;
        grouped = true;
    }
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < CPW; ++k)
        c += __popc(f[k]);
    return c;
}

// Valid starts of the tile at ts as tile offsets [lo, hi) (the tile holds at least one: last >= ts).
__device__ __forceinline__ void bc_tile_range(const BmCountArgs &a, uint64_t ts, uint32_t S, uint32_t &lo,
                                              uint32_t &hi)
{
    const uint64_t rem = a.last - ts;
    hi = rem >= S ? S : (uint32_t)rem + 1u;
    lo = ts < a.tv.first ? (uint32_t)(a.tv.first - ts) : 0u;
}

// Single search over bitmap tiles.  Tiles are dealt out as in the byte-tile
// count kernel.  Thread tid owns words tid + kWG * c (c < CPW) of every tile:
// it loads their bytes into registers (the next tile's while the current one
// is searched), builds their slot words into one of two LDS buffers, and after
// the barrier searches its 32 * CPW starts.
template <int NS, int CPW, bool STREAM>
__global__ __launch_bounds__(kWG) void k_count_bitmap(BmCountArgs a)
{
    extern __shared__ __align__(16) uint32_t bml[];
    constexpr uint32_t W = kWG * CPW;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t S = 32u * (W - a.halo_words);  // starts per tile
    const uint64_t kmask = (1ull << a.chunk_log2) - 1u;
    auto tile_of = [&](uint64_t i) {
        return (((uint64_t)blockIdx.x + (i >> a.chunk_log2) * gridDim.x) << a.chunk_log2) + (i & kmask);
    };
    uint32_t X[CPW][8];
    // inner tiles: every start of the words below W - halo_words is valid
    uint32_t inner[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        inner[c] = tid + kWG * c < W - a.halo_words ? 0xFFFFFFFFu : 0u;
    const uint32_t ent0 = bc_entries<NS, W>(a, 0, lane);
    const BcPlaneMasks<NS> pm = bc_plane_masks<NS>(a.syms);
    uint32_t acc = 0;
    uint64_t tile = tile_of(0);
    if (tile < a.ntiles)
        bc_load_tile<CPW, STREAM>(a.tv, tile * S, tid, X);
    for (uint64_t i = 0; tile < a.ntiles; ++i) {
        const uint64_t ts = tile * S;
        uint32_t *buf = bml + (i & 1u) * (NS * W);
        bc_build_tile<NS, CPW>(X, a.syms, pm, buf, tid);
        const uint64_t next = tile_of(i + 1);
        if (next < a.ntiles)
            bc_load_tile<CPW, STREAM>(a.tv, next * S, tid, X);
        __syncthreads();  // the tile's bitmaps are complete; the other buffer is no longer read
        uint32_t lo, hi;
        bc_tile_range(a, ts, S, lo, hi);
        acc += bc_search_tile<NS, CPW>(a, buf, ent0, tid, lo, hi, S, inner);
        tile = next;
    }
    wg_add_count(acc, a.count, tid);
}

// Batched single-query texts of at most kBcMaxSyms symbols, through bitmap
// tiles of 8 KiB x CPW: a persistent grid takes deals (runs of up to
// 2^chunk_log2 tiles of one query's text) in order, as k_batch_deals does for
// byte tiles.  Each deal's query record gives the search's constants (slots
// padded to four with repeats of the first symbol: a repeated slot holds the
// same bitmap).  The two bitmap buffers alternate by the workgroup's running
// tile count, so the one barrier per tile also separates a deal's first build
// from the previous deal's searches; each wave adds its matches to the query's
// count.
template <int CPW, bool STREAM>
__global__ __launch_bounds__(kWG) void k_bm_deals(BmDealArgs a)
{
    extern __shared__ __align__(16) uint32_t bml[];
    constexpr int NS = (int)kBcMaxSyms;
    constexpr uint32_t W = kWG * CPW;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint32_t X[CPW][8];
    uint64_t gi = 0;  // tiles this workgroup has built
    for (uint64_t k = blockIdx.x; k < a.ndeals; k += gridDim.x) {
        const BatchDeal d = ldc(&a.deals[k]);
        const BmSolo so = ldc(&a.solos[d.solo]);
        BmCountArgs q{};
        q.tv = so.tv;
        q.last = so.last;
        q.steps = so.steps;
        q.m = so.m;
        q.r = so.r;
        q.syms = so.syms;
        q.halo_words = so.halo_words;
        const uint32_t S = 32u * (W - q.halo_words);
        uint32_t inner[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            inner[c] = tid + kWG * c < W - q.halo_words ? 0xFFFFFFFFu : 0u;
        const uint32_t ent0 = bc_entries<NS, W>(q, 0, lane);
        const BcPlaneMasks<NS> pm = bc_plane_masks<NS>(q.syms);
        const uint64_t t0 = d.tiles >> 3;
        const uint32_t nt = d.tiles & 7u;
        bc_load_tile<CPW, STREAM>(q.tv, t0 * S, tid, X);
        uint32_t acc = 0;
        for (uint32_t i = 0; i < nt; ++i, ++gi) {
            const uint64_t ts = (t0 + i) * S;
            uint32_t *buf = bml + (gi & 1u) * (NS * W);
            bc_build_tile<NS, CPW>(X, q.syms, pm, buf, tid);
            if (i + 1u < nt)
                bc_load_tile<CPW, STREAM>(q.tv, ts + S, tid, X);
            __syncthreads();
            uint32_t lo, hi;
            bc_tile_range(q, ts, S, lo, hi);
            acc += bc_search_tile<NS, CPW>(q, buf, ent0, tid, lo, hi, S, inner);
        }
        const uint32_t c = wave_sum32(acc);
        if (lane == 0 && c)
            atomicAdd(&a.counts[so.out], (unsigned long long)c);
    }
}

// ---------------------------------------------------------------- launchers

template <int CPL, int R, bool STREAM>
static hipError_t launch_staged_t(const CountArgs &a, unsigned grid, hipStream_t s)
{
    const uint32_t lds = 2u * (kWG * 16u * CPL + a.halo);
    hipLaunchKernelGGL((k_count_staged<CPL, R, STREAM>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <int CPL, bool STREAM>
static hipError_t launch_staged_r(const CountArgs &a, int r, unsigned grid, hipStream_t s)
{
    switch (r) {
    case 1: return launch_staged_t<CPL, 1, STREAM>(a, grid, s);
    case 2: return launch_staged_t<CPL, 2, STREAM>(a, grid, s);
    case 3: return launch_staged_t<CPL, 3, STREAM>(a, grid, s);
    case 4: return launch_staged_t<CPL, 4, STREAM>(a, grid, s);
    case 5: return launch_staged_t<CPL, 5, STREAM>(a, grid, s);
    case 6: return launch_staged_t<CPL, 6, STREAM>(a, grid, s);
    case 7: return launch_staged_t<CPL, 7, STREAM>(a, grid, s);
    case 8: return launch_staged_t<CPL, 8, STREAM>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool STREAM>
static hipError_t launch_staged_c(const CountArgs &a, int cpl, int r, unsigned grid, hipStream_t s)
{
    switch (cpl) {
    case 1: return launch_staged_r<1, STREAM>(a, r, grid, s);
    case 2: return launch_staged_r<2, STREAM>(a, r, grid, s);
    case 4: return launch_staged_r<4, STREAM>(a, r, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_count_staged(const CountArgs &a, int cpl, int r, bool stream_loads, unsigned grid, hipStream_t s)
{
    return stream_loads ? launch_staged_c<true>(a, cpl, r, grid, s) : launch_staged_c<false>(a, cpl, r, grid, s);
}

template <int R>
static hipError_t launch_global_t(const CountArgs &a, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_count_global<R>), dim3(grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_count_global(const CountArgs &a, int r, unsigned grid, hipStream_t s)
{
    switch (r) {
    case 1: return launch_global_t<1>(a, grid, s);
    case 2: return launch_global_t<2>(a, grid, s);
    case 3: return launch_global_t<3>(a, grid, s);
    case 4: return launch_global_t<4>(a, grid, s);
    case 5: return launch_global_t<5>(a, grid, s);
    case 6: return launch_global_t<6>(a, grid, s);
    case 7: return launch_global_t<7>(a, grid, s);
    case 8: return launch_global_t<8>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int NS, int CPW, bool STREAM>
static hipError_t launch_bitmap_t(const BmCountArgs &a, unsigned grid, hipStream_t s)
{
    // two buffers of NS slots, plus the words a no-start thread's funnel shifts reach past the last slot
    const uint32_t lds = (2u * NS * kWG * CPW + a.halo_words + 1u) * 4u;
    hipLaunchKernelGGL((k_count_bitmap<NS, CPW, STREAM>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <int CPW, bool STREAM>
static hipError_t launch_bitmap_n(const BmCountArgs &a, int ns, unsigned grid, hipStream_t s)
{
    switch (ns) {
    case 1: return launch_bitmap_t<1, CPW, STREAM>(a, grid, s);
    case 2: return launch_bitmap_t<2, CPW, STREAM>(a, grid, s);
    case 3: return launch_bitmap_t<3, CPW, STREAM>(a, grid, s);
    case 4: return launch_bitmap_t<4, CPW, STREAM>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool STREAM>
static hipError_t launch_bitmap_c(const BmCountArgs &a, int ns, int cpw, unsigned grid, hipStream_t s)
{
    switch (cpw) {
    case 1: return launch_bitmap_n<1, STREAM>(a, ns, grid, s);
    case 2: return launch_bitmap_n<2, STREAM>(a, ns, grid, s);
    case 4: return launch_bitmap_n<4, STREAM>(a, ns, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bm_deals(const BmDealArgs &a, uint32_t halo_max, bool stream_loads, unsigned grid, hipStream_t s)
{
    const uint32_t lds = (2u * kBcMaxSyms * kWG * kBmDealCpw + halo_max + 1u) * 4u;
    if (stream_loads)
        hipLaunchKernelGGL((k_bm_deals<kBmDealCpw, true>), dim3(grid), dim3(kWG), lds, s, a);
    else
        hipLaunchKernelGGL((k_bm_deals<kBmDealCpw, false>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_count_bitmap(const BmCountArgs &a, int ns, int cpw, bool stream_loads, unsigned grid, hipStream_t s)
{
    if (a.halo_words == 0 || a.halo_words > kWG * (uint32_t)cpw / 2u)
        return hipErrorInvalidValue;
    return stream_loads ? launch_bitmap_c<true>(a, ns, cpw, grid, s) : launch_bitmap_c<false>(a, ns, cpw, grid, s);
}

hipError_t launch_scan_groups(const unsigned long long *gs, uint64_t ngroups, unsigned long long *go,
                              unsigned long long *total, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_groups, dim3(1), dim3(1024), 0, s, gs, ngroups, go, total);
    return hipGetLastError();
}

hipError_t launch_report_write(const CountArgs &a, uint32_t *bc, unsigned long long *gs, const unsigned long long *go,
                               uint64_t ngroups, unsigned long long *pos, uint64_t cap, uint32_t win, unsigned grid,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_report_write, dim3(grid), dim3(kWG), kWaves * win, s, a, bc, gs, go, ngroups, pos, cap, win);
    return hipGetLastError();
}

hipError_t launch_report_multi(const RepDesc *descs, uint64_t nq, const uint32_t *item_query, uint64_t nitems,
                               uint32_t win_max, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_groups_multi, dim3((unsigned)nq), dim3(1024), 0, s, descs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nitems == 0)
        return e;
    hipLaunchKernelGGL(k_report_write_multi, dim3(grid), dim3(kWG), kWaves * win_max, s, descs, item_query, nitems);
    return hipGetLastError();
}

hipError_t launch_fill_report(uint32_t *bc, uint64_t nblocks, unsigned long long *gs, uint64_t ngroups,
                              hipStream_t s)
{
    const uint64_t g = (nblocks + 1023) / 1024;
    const unsigned grid = (unsigned)(g < 4096 ? (g ? g : 1) : 4096);
    hipLaunchKernelGGL(k_fill_report, dim3(grid), dim3(256), 0, s, bc, nblocks, gs, ngroups);
    return hipGetLastError();
}

hipError_t launch_hist(const TextView &tv, unsigned long long *hist, bool stream_loads, unsigned grid, hipStream_t s)
{
    if (stream_loads)
        hipLaunchKernelGGL(k_hist<true>, dim3(grid), dim3(kHistWG), kHistLds, s, tv, hist);
    else
        hipLaunchKernelGGL(k_hist<false>, dim3(grid), dim3(kHistWG), kHistLds, s, tv, hist);
    return hipGetLastError();
}

hipError_t launch_bigram(const TextView &tv, uint32_t half, unsigned long long *out, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_bigram, dim3(grid), dim3(kBgWG), kBgLds, s, tv, half, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s)
{
    const uint64_t g = (n + 255) / 256;
    const unsigned grid = (unsigned)(g < 1024 ? (g ? g : 1) : 1024);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <int CPL, bool STREAM>
static hipError_t launch_batch_t(const BatchArgs &a, unsigned grid, hipStream_t s)
{
    const uint32_t lds = 2u * (kWG * 16u * CPL + a.halo_max) + kQChunk * (uint32_t)sizeof(uint32_t);
    if (a.reports)
        hipLaunchKernelGGL((k_batch_staged<CPL, true, STREAM>), dim3(grid), dim3(kWG), lds, s, a);
    else
        hipLaunchKernelGGL((k_batch_staged<CPL, false, STREAM>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <bool STREAM>
static hipError_t launch_deals_c(const DealArgs &a, int cpl, unsigned grid, hipStream_t s)
{
    const uint32_t lds = 2u * (kWG * 16u * (uint32_t)cpl + a.halo_max);
    switch (cpl) {
    case 1: hipLaunchKernelGGL((k_batch_deals<1, STREAM>), dim3(grid), dim3(kWG), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_batch_deals<2, STREAM>), dim3(grid), dim3(kWG), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_batch_deals<4, STREAM>), dim3(grid), dim3(kWG), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_deals(const DealArgs &a, int cpl, bool stream_loads, unsigned grid, hipStream_t s)
{
    return stream_loads ? launch_deals_c<true>(a, cpl, grid, s) : launch_deals_c<false>(a, cpl, grid, s);
}

template <bool STREAM>
static hipError_t launch_batch_c(const BatchArgs &a, int cpl, unsigned grid, hipStream_t s)
{
    switch (cpl) {
    case 1: return launch_batch_t<1, STREAM>(a, grid, s);
    case 2: return launch_batch_t<2, STREAM>(a, grid, s);
    case 4: return launch_batch_t<4, STREAM>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_staged(const BatchArgs &a, int cpl, bool stream_loads, unsigned grid, hipStream_t s)
{
    return stream_loads ? launch_batch_c<true>(a, cpl, grid, s) : launch_batch_c<false>(a, cpl, grid, s);
}

}  // namespace smk

namespace smk {
hipError_t launch_batch_bitmap(const BmArgs &a, unsigned grid, uint32_t lds_bytes, bool two_per_cu, hipStream_t s)
{
    if (two_per_cu)
        hipLaunchKernelGGL(k_batch_bitmap2, dim3(grid), dim3(kBmWG), lds_bytes, s, a);
    else
        hipLaunchKernelGGL(k_batch_bitmap, dim3(grid), dim3(kBmWG), lds_bytes, s, a);
    return hipGetLastError();
}
}  // namespace smk

namespace smk {
static unsigned no_grid(uint64_t items)
{
    const uint64_t g = (items + kWG - 1) / kWG;
    return (unsigned)(g < 8192 ? (g ? g : 1) : 8192);
}

hipError_t launch_no_next(const unsigned long long *pos, uint64_t c, uint32_t m, uint32_t *nxt, uint32_t *mark,
                          unsigned long long *overlapped, hipStream_t s)
{
    hipLaunchKernelGGL(k_no_next, dim3(no_grid(c)), dim3(kWG), 0, s, pos, c, m, nxt, mark, overlapped);
    return hipGetLastError();
}

hipError_t launch_no_round(const uint32_t *nxt, uint32_t *nxt_out, uint32_t *mark, uint64_t c, hipStream_t s)
{
    hipLaunchKernelGGL(k_no_mark, dim3(no_grid(c)), dim3(kWG), 0, s, nxt, mark, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_no_jump, dim3(no_grid(c)), dim3(kWG), 0, s, nxt, nxt_out, c);
    return hipGetLastError();
}

hipError_t launch_no_chunk_counts(const uint32_t *mark, uint64_t c, unsigned long long *gs, uint64_t ng,
                                  hipStream_t s)
{
    const unsigned grid = (unsigned)(ng < 4096 ? (ng ? ng : 1) : 4096);
    hipLaunchKernelGGL(k_no_chunk_counts, dim3(grid), dim3(kWG), 0, s, mark, c, gs, ng);
    return hipGetLastError();
}

hipError_t launch_no_compact(const unsigned long long *pos, const uint32_t *mark, uint64_t c,
                             const unsigned long long *go, uint64_t ng, unsigned long long *out, uint64_t cap,
                             hipStream_t s)
{
    const unsigned grid = (unsigned)(ng < 4096 ? (ng ? ng : 1) : 4096);
    hipLaunchKernelGGL(k_no_compact, dim3(grid), dim3(kWG), 0, s, pos, mark, c, go, ng, out, cap);
    return hipGetLastError();
}
}  // namespace smk

namespace smk {
// Raises the dynamic-LDS limit of every kernel that takes more than the
// default.  Called once per device at initialisation, so that later launches
// (possibly under stream capture) make no attribute calls.
template <typename K>
static hipError_t lds_attr(K *k, int bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int CPL>
static hipError_t prime_cpl()
{
    const void *ks[] = {reinterpret_cast<const void *>(&k_count_staged<CPL, 1, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 2, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 3, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 4, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 5, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 6, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 7, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 8, false>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 1, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 2, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 3, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 4, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 5, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 6, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 7, true>),
                        reinterpret_cast<const void *>(&k_count_staged<CPL, 8, true>),
                        reinterpret_cast<const void *>(&k_batch_staged<CPL, false, false>),
                        reinterpret_cast<const void *>(&k_batch_staged<CPL, true, false>),
                        reinterpret_cast<const void *>(&k_batch_staged<CPL, false, true>),
                        reinterpret_cast<const void *>(&k_batch_staged<CPL, true, true>),
                        reinterpret_cast<const void *>(&k_batch_deals<CPL, false>),
                        reinterpret_cast<const void *>(&k_batch_deals<CPL, true>)};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t prime_kernel_attrs()
{
    hipError_t e;
    if ((e = prime_cpl<1>()) != hipSuccess || (e = prime_cpl<2>()) != hipSuccess ||
        (e = prime_cpl<4>()) != hipSuccess)
        return e;
    if ((e = lds_attr(&k_report_write, (int)kMaxLds)) != hipSuccess)
        return e;
    if ((e = lds_attr(&k_report_write_multi, (int)kMaxLds)) != hipSuccess)
        return e;
    if ((e = lds_attr(&k_hist<false>, (int)kHistLds)) != hipSuccess || (e = lds_attr(&k_hist<true>, (int)kHistLds)) != hipSuccess)
        return e;
    if ((e = lds_attr(&k_bigram, (int)kBgLds)) != hipSuccess)
        return e;
    if ((e = lds_attr(&k_batch_bitmap, (int)kBmMaxLds)) != hipSuccess)
        return e;
    return lds_attr(&k_batch_bitmap2, (int)kBmMaxLds);
}
}  // namespace smk
