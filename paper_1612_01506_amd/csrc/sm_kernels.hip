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
//     with coalesced 16-byte loads; the next tile is prefetched into VGPRs
//     while the current one is searched.  Each workgroup owns a contiguous
//     range of tiles, so a halo is the start of the tile it loads next (an L2
//     hit, not a second HBM read).
//   * Counts: per-lane 64-bit accumulators, a wave shuffle reduction, one LDS
//     reduction and one 64-bit atomicAdd per workgroup.
#include "sm_internal.h"

namespace smk {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t step_pos(uint64_t st) { return (uint32_t)st; }
__device__ __forceinline__ uint32_t step_rep(uint64_t st) { return (uint32_t)(st >> 32); }

// Initial found for the wave vector at coordinate wb: starts outside
// [first, last] are dead (byte 0xFF); all others alive (0).
__device__ __forceinline__ void init_alive(uint64_t wb, uint64_t first, uint64_t last, uint32_t lane,
                                           uint32_t (&d)[4])
{
    if (wb >= first && wb + (kBlock - 1) <= last) {
        d[0] = d[1] = d[2] = d[3] = 0u;
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t u0 = wb + 256u * k + 4u * lane;
        uint32_t inv = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint64_t u = u0 + b;
            if (u < first || u > last)
                inv |= 0xFFu << (8 * b);
        }
        d[k] = inv;
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

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
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

// Algorithm 4 over one wave vector with a compile-time peel factor R (R <= m):
// R unconditional compares, a zero test, then compare-and-test for the rest.
// Returns this lane's share of popcount(found) (0 when the vector died).
template <int R, typename Step>
__device__ __forceinline__ uint32_t search_vector(const uint64_t *steps, const uint64_t (&pk)[R], uint32_t m,
                                                  uint32_t (&d)[4], Step step)
{
#pragma unroll
    for (int l = 0; l < R; ++l)
        step(pk[l], d);
    if (!any_alive(d))
        return 0;
    uint64_t nxt = steps[R];
    for (uint32_t l = R; l < m; ++l) {
        const uint64_t cur = nxt;
        nxt = steps[l + 1];  // padded table: in bounds
        step(cur, d);
        if (!any_alive(d))
            return 0;
    }
    return count_alive(d);
}

// Same with a run-time peel factor (batch queries carry their own r).
template <typename Step>
__device__ __forceinline__ uint32_t search_vector_rt(const uint64_t *steps, uint32_t r, uint32_t m,
                                                     uint32_t (&d)[4], Step step)
{
    uint32_t l = 0;
    for (; l < r; ++l)
        step(steps[l], d);
    if (!any_alive(d))
        return 0;
    for (; l < m; ++l) {
        step(steps[l], d);
        if (!any_alive(d))
            return 0;
    }
    return count_alive(d);
}

// ------------------------------------------------------------- tile staging

template <int CPL>
__device__ __forceinline__ void fetch_tile(const TextView &tv, uint64_t ts, uint32_t tid, uint32_t hch,
                                           uint4 (&pre)[CPL], uint4 &hpre)
{
    constexpr uint32_t T = kWG * 16u * CPL;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const uint64_t u = ts + 16ull * (tid + kWG * c);
        pre[c] = u < tv.end16 ? *reinterpret_cast<const uint4 *>(tv.base + u) : make_uint4(0, 0, 0, 0);
    }
    if (tid < hch) {
        const uint64_t u = ts + T + 16ull * tid;
        hpre = u < tv.end16 ? *reinterpret_cast<const uint4 *>(tv.base + u) : make_uint4(0, 0, 0, 0);
    }
}

template <int CPL>
__device__ __forceinline__ void put_tile(uint8_t *lds, uint32_t tid, uint32_t hch, const uint4 (&pre)[CPL],
                                         const uint4 &hpre)
{
    constexpr uint32_t T = kWG * 16u * CPL;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        *reinterpret_cast<uint4 *>(lds + 16u * (tid + kWG * c)) = pre[c];
    if (tid < hch)
        *reinterpret_cast<uint4 *>(lds + T + 16u * tid) = hpre;
}

// Halo chunks past the first kWG are loaded synchronously (long patterns only).
__device__ __forceinline__ void put_halo_rest(uint8_t *halo_lds, const TextView &tv, uint64_t hs, uint32_t tid,
                                              uint32_t hch)
{
    for (uint32_t ch = kWG + tid; ch < hch; ch += kWG) {
        const uint64_t u = hs + 16ull * ch;
        const uint4 v = u < tv.end16 ? *reinterpret_cast<const uint4 *>(tv.base + u) : make_uint4(0, 0, 0, 0);
        *reinterpret_cast<uint4 *>(halo_lds + 16u * ch) = v;
    }
}

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

// Single search, text staged in LDS.  Workgroup g searches tiles
// [g * tiles_per_wg, (g + 1) * tiles_per_wg); wave w takes vectors
// w*CPL .. w*CPL + CPL - 1 of each tile.
template <int CPL, int R>
__global__ __launch_bounds__(kWG) void k_count_staged(CountArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t T = kWG * 16u * CPL;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t t0 = (uint64_t)blockIdx.x * a.tiles_per_wg;
    const uint64_t t1 = min(t0 + a.tiles_per_wg, a.ntiles);
    const uint32_t hch = a.halo >> 4;

    uint64_t pk[R];
#pragma unroll
    for (int l = 0; l < R; ++l)
        pk[l] = a.steps[l];

    uint4 pre[CPL];
    uint4 hpre = make_uint4(0, 0, 0, 0);
    unsigned long long acc = 0;
    if (t0 < t1)
        fetch_tile<CPL>(a.tv, t0 * T, tid, hch, pre, hpre);
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t ts = tile * T;
        __syncthreads();
        put_tile<CPL>(lds, tid, hch, pre, hpre);
        if (hch > kWG)
            put_halo_rest(lds + T, a.tv, ts + T, tid, hch);
        __syncthreads();
        if (tile + 1 < t1)
            fetch_tile<CPL>(a.tv, ts + T, tid, hch, pre, hpre);
#pragma unroll
        for (int b = 0; b < CPL; ++b) {
            const uint32_t boff = (wave * CPL + b) * kBlock;
            const uint64_t wb = ts + boff;
            if (wb > a.last)
                break;
            uint32_t d[4];
            init_alive(wb, a.tv.first, a.last, lane, d);
            const uint8_t *lb = lds + boff + 4u * lane;
            const uint32_t c = search_vector<R>(a.steps, pk, a.m, d,
                                                [&](uint64_t st, uint32_t (&dd)[4]) { step_lds(lb, st, dd); });
            if (a.block_counts) {
                const uint32_t s = wave_sum32(c);
                if (lane == 0)
                    a.block_counts[wb / kBlock] = s;
            }
            acc += c;
        }
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
        pk[l] = a.steps[l];
    unsigned long long acc = 0;
    for (uint64_t blk = (uint64_t)blockIdx.x * kWaves + (tid >> 6); blk < a.nblocks; blk += nw) {
        const uint64_t wb = blk * kBlock;
        uint32_t d[4];
        init_alive(wb, a.tv.first, a.last, lane, d);
        const uint64_t lu = wb + 4u * lane;
        const uint32_t c = search_vector<R>(a.steps, pk, a.m, d,
                                            [&](uint64_t st, uint32_t (&dd)[4]) { step_global(a.tv, lu, st, dd); });
        if (a.block_counts) {
            const uint32_t s = wave_sum32(c);
            if (lane == 0)
                a.block_counts[blk] = s;
        }
        acc += c;
    }
    wg_add_count(acc, a.count, tid);
}

// ---------------------------------------------------------- report kernels

// gs[g] = sum of block counts 64g .. 64g+63 (one wave per group).
__global__ __launch_bounds__(kWG) void k_group_sums(const uint32_t *bc, uint64_t nblocks, uint64_t ngroups,
                                                   unsigned long long *gs)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (g >= ngroups)
        return;
    const uint64_t b = g * 64u + lane;
    const uint32_t c = b < nblocks ? bc[b] : 0u;
    const uint32_t s = wave_sum32(c);
    if (lane == 0)
        gs[g] = s;
}

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

// Write pass of the reporting version: every vector with a nonzero block
// count is searched again (all m compares) and its starts are written in
// increasing order at that block's offset.  Within a vector the order is
// k-major, then lane, then byte -- exactly increasing start -- and lane
// offsets come from a bit-sliced ballot prefix sum (mbcnt).
__global__ __launch_bounds__(kWG) void k_report_write(CountArgs a, const uint32_t *bc,
                                                     const unsigned long long *go, uint64_t ngroups,
                                                     unsigned long long *pos, uint64_t cap)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    for (uint64_t g = (uint64_t)blockIdx.x * kWaves + (tid >> 6); g < ngroups; g += nw) {
        const uint64_t b = g * 64u + lane;
        const uint32_t c = b < a.nblocks ? bc[b] : 0u;
        unsigned long long nz = __ballot(c != 0u);
        if (nz == 0)
            continue;
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o)
                inc += v;
        }
        const uint32_t excl = inc - c;
        const unsigned long long base = go[g];
        while (nz) {
            const int bit = __ffsll((long long)nz) - 1;
            nz &= nz - 1;
            const uint64_t wb = (g * 64u + (uint64_t)bit) * kBlock;
            unsigned long long o = base + (unsigned long long)__shfl(excl, bit, 64);
            uint32_t d[4];
            init_alive(wb, a.tv.first, a.last, lane, d);
            const uint64_t lu = wb + 4u * lane;
            for (uint32_t l = 0; l < a.m; ++l)
                step_global(a.tv, lu, a.steps[l], d);
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
                            pos[idx] = wb + 256u * k + 4u * lane + by - a.tv.first;
                        ++idx;
                    }
                }
                o += tot;
            }
        }
    }
}

// ------------------------------------------------------------- histogram

// Symbol frequencies (Section 2.2): per-wave LDS histograms over 16-byte
// chunks, then one 64-bit atomicAdd per nonzero bin and workgroup.
__global__ __launch_bounds__(kWG) void k_hist(TextView tv, unsigned long long *hist)
{
    __shared__ uint32_t h[kWaves][256];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    for (uint32_t i = tid; i < kWaves * 256u; i += kWG)
        (&h[0][0])[i] = 0u;
    __syncthreads();
    uint32_t *hw = h[wave];
    const uint64_t lo = tv.first, hi = tv.first + tv.n, nchunks = tv.end16 / 16u;
    for (uint64_t c = (uint64_t)blockIdx.x * kWG + tid; c < nchunks; c += (uint64_t)gridDim.x * kWG) {
        const uint64_t u = 16u * c;
        const uint4 v = *reinterpret_cast<const uint4 *>(tv.base + u);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        if (u >= lo && u + 16u <= hi) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                atomicAdd(&hw[(w[i >> 2] >> (8 * (i & 3))) & 0xFFu], 1u);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (u + i >= lo && u + i < hi)
                    atomicAdd(&hw[(w[i >> 2] >> (8 * (i & 3))) & 0xFFu], 1u);
        }
    }
    __syncthreads();
    for (uint32_t bin = tid; bin < 256u; bin += kWG) {
        unsigned long long s = 0;
#pragma unroll
        for (uint32_t i = 0; i < kWaves; ++i)
            s += h[i][bin];
        if (s)
            atomicAdd(&hist[bin], s);
    }
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ batch kernel

// Persistent batched count: work item = (text, contiguous tile range, chunk
// of <= kQChunk queries of one m-bucket).  The workgroup stages each tile of
// the range once and runs every query of the chunk over it; per-query counts
// gather in LDS and are flushed with one 64-bit atomicAdd per nonzero query
// and item.
template <int CPL>
__global__ __launch_bounds__(kWG) void k_batch_staged(BatchArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t T = kWG * 16u * CPL;
    uint32_t *qc = reinterpret_cast<uint32_t *>(lds + a.tile_lds);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    for (uint64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const BatchItem I = a.items[it];
        const uint32_t nq = I.q_end - I.q_begin;
        const uint32_t hch = I.halo >> 4;
        __syncthreads();  // previous item's counters flushed
        for (uint32_t i = tid; i < nq; i += kWG)
            qc[i] = 0u;
        uint4 pre[CPL];
        uint4 hpre = make_uint4(0, 0, 0, 0);
        if (I.tile_begin < I.tile_end)
            fetch_tile<CPL>(I.tv, I.tile_begin * T, tid, hch, pre, hpre);
        for (uint64_t tile = I.tile_begin; tile < I.tile_end; ++tile) {
            const uint64_t ts = tile * T;
            __syncthreads();
            put_tile<CPL>(lds, tid, hch, pre, hpre);
            if (hch > kWG)
                put_halo_rest(lds + T, I.tv, ts + T, tid, hch);
            __syncthreads();
            if (tile + 1 < I.tile_end)
                fetch_tile<CPL>(I.tv, ts + T, tid, hch, pre, hpre);
            for (uint32_t q = I.q_begin; q < I.q_end; ++q) {
                const BatchQuery Q = a.queries[q];
                const uint64_t *st = a.steps + Q.steps_off;
                uint32_t c = 0;
#pragma unroll 1
                for (int b = 0; b < CPL; ++b) {
                    const uint32_t boff = (wave * CPL + b) * kBlock;
                    const uint64_t wb = ts + boff;
                    if (wb > Q.last)
                        break;
                    uint32_t d[4];
                    init_alive(wb, I.tv.first, Q.last, lane, d);
                    const uint8_t *lb = lds + boff + 4u * lane;
                    c += search_vector_rt(st, Q.r, Q.m, d,
                                          [&](uint64_t s, uint32_t (&dd)[4]) { step_lds(lb, s, dd); });
                }
                if (__any(c != 0u)) {
                    const uint32_t s = wave_sum32(c);
                    if (lane == 0)
                        atomicAdd(&qc[q - I.q_begin], s);
                }
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < nq; i += kWG) {
            const uint32_t v = qc[i];
            if (v)
                atomicAdd(&a.counts[a.queries[I.q_begin + i].out], (unsigned long long)v);
        }
    }
}

// ---------------------------------------------------------------- launchers

template <int CPL, int R>
static hipError_t launch_staged_t(const CountArgs &a, unsigned grid, hipStream_t s)
{
    static bool attr_set = false;
    const uint32_t lds = kWG * 16u * CPL + a.halo;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_count_staged<CPL, R>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_count_staged<CPL, R>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <int CPL>
static hipError_t launch_staged_r(const CountArgs &a, int r, unsigned grid, hipStream_t s)
{
    switch (r) {
    case 1: return launch_staged_t<CPL, 1>(a, grid, s);
    case 2: return launch_staged_t<CPL, 2>(a, grid, s);
    case 3: return launch_staged_t<CPL, 3>(a, grid, s);
    case 4: return launch_staged_t<CPL, 4>(a, grid, s);
    case 5: return launch_staged_t<CPL, 5>(a, grid, s);
    case 6: return launch_staged_t<CPL, 6>(a, grid, s);
    case 7: return launch_staged_t<CPL, 7>(a, grid, s);
    case 8: return launch_staged_t<CPL, 8>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_count_staged(const CountArgs &a, int cpl, int r, unsigned grid, hipStream_t s)
{
    switch (cpl) {
    case 1: return launch_staged_r<1>(a, r, grid, s);
    case 2: return launch_staged_r<2>(a, r, grid, s);
    case 4: return launch_staged_r<4>(a, r, grid, s);
    default: return hipErrorInvalidValue;
    }
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

hipError_t launch_group_sums(const uint32_t *bc, uint64_t nblocks, uint64_t ngroups, unsigned long long *gs,
                             hipStream_t s)
{
    const uint64_t grid = (ngroups + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_group_sums, dim3((unsigned)grid), dim3(kWG), 0, s, bc, nblocks, ngroups, gs);
    return hipGetLastError();
}

hipError_t launch_scan_groups(const unsigned long long *gs, uint64_t ngroups, unsigned long long *go,
                              unsigned long long *total, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_groups, dim3(1), dim3(1024), 0, s, gs, ngroups, go, total);
    return hipGetLastError();
}

hipError_t launch_report_write(const CountArgs &a, const uint32_t *bc, const unsigned long long *go,
                               uint64_t ngroups, unsigned long long *pos, uint64_t cap, unsigned grid,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_report_write, dim3(grid), dim3(kWG), 0, s, a, bc, go, ngroups, pos, cap);
    return hipGetLastError();
}

hipError_t launch_hist(const TextView &tv, unsigned long long *hist, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_hist, dim3(grid), dim3(kWG), 0, s, tv, hist);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s)
{
    const uint64_t g = (n + 255) / 256;
    const unsigned grid = (unsigned)(g < 1024 ? (g ? g : 1) : 1024);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <int CPL>
static hipError_t launch_batch_t(const BatchArgs &a, unsigned grid, uint32_t lds, hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_staged<CPL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_batch_staged<CPL>), dim3(grid), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_staged(const BatchArgs &a, int cpl, unsigned grid, uint32_t lds_bytes, hipStream_t s)
{
    switch (cpl) {
    case 1: return launch_batch_t<1>(a, grid, lds_bytes, s);
    case 2: return launch_batch_t<2>(a, grid, lds_bytes, s);
    case 4: return launch_batch_t<4>(a, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace smk
