// Internal definitions shared by the kernels (sm_kernels.hip) and the C-ABI
// host code (sm_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smk {

constexpr uint32_t kWG = 256;            // threads per workgroup: four wave64
constexpr uint32_t kWaves = kWG / 64;
constexpr uint32_t kHistWG = 1024;        // histogram workgroup: 16 waves sharing 64 lane copies
constexpr uint32_t kHistLds = 256 * 64 * 4;
constexpr uint32_t kBgWG = 1024;          // adjacent-pair counts: one 16-wave workgroup per CU
constexpr uint32_t kBgLds = 128 * 256 * 4; // half of the 256 x 256 table per pass
constexpr uint32_t kBlock = 1024;        // starts per wave vector: 64 lanes x 4 dwords x 4 bytes
constexpr uint32_t kMaxPeel = 8;         // largest peel factor r compiled in
constexpr uint32_t kStepPad = 8;         // zero entries after every step table (one-ahead loads)
constexpr uint32_t kMaxLds = 65536;      // dynamic LDS per workgroup used by the staged kernels
constexpr uint32_t kQChunk = 512;        // queries per batch work item (LDS counters)
constexpr uint32_t kGroupBlocks = 1024;  // wave vectors per report scan group

// A text in aligned coordinates: coordinate u is the byte at address base + u.
struct TextView {
    const uint8_t *base;  // 16-byte aligned, <= t
    uint64_t first;       // coordinate of t[0] (0..15)
    uint64_t n;           // text length in bytes
    uint64_t end16;       // first + n rounded up to 16: no chunk at or past it is loaded
};

// Step table entry, one per compare in compare order pi:
//   bits  0..31  pattern position j = pi(l)
//   bits 32..63  p[j] replicated into all four bytes
// Tables are followed by kStepPad zero entries.

struct CountArgs {
    TextView tv;
    uint64_t last;            // coordinate of the last valid start: first + n - m
    uint64_t ntiles;          // staged: tiles covering coordinates [0, last]
    uint32_t chunk_log2;      // staged: tiles are dealt out in chunks of 2^chunk_log2 contiguous tiles,
    uint32_t pad0;            //   chunk c to workgroup c mod gridDim.x
    uint64_t nblocks;         // ceil((last + 1) / kBlock)
    const uint64_t *steps;    // device step table (m + kStepPad entries)
    uint32_t m;
    uint32_t halo;            // staged: LDS bytes past the tile (multiple of 16, >= m + 4)
    unsigned long long *count;     // += total count (may be null)
    uint32_t *block_counts;   // report pass: nonzero per-vector counts (array zeroed before), or null
    unsigned long long *group_sums;  // report pass: += per-vector counts of each kGroupBlocks group
};

// Byte-tile batch: a chunk is one text and up to kQChunk queries of one
// m-bucket; its tiles occupy global tile indices [tile0, tile0 + ntiles).
struct BatchChunk {
    TextView tv;
    uint64_t tile0;
    uint32_t q_begin, q_end;  // into the BatchQuery array
    uint32_t halo;            // LDS halo bytes for the chunk's longest pattern
    uint32_t ntiles;
};

struct BatchQuery {
    uint64_t steps_off;  // index of the query's step table in the steps pool
    uint64_t last;       // coordinate of its last valid start in its text
    uint32_t m;
    uint32_t r;          // peel factor, 1..min(kMaxPeel, m)
    uint32_t out;        // output slot
    uint32_t pad;
};

// Byte-tile batch, single-query chunks.  A deal is up to 2^chunk_log2 consecutive tiles of one
// query's text: (its query's record, first tile << 3 | number of tiles).
struct BatchSolo {
    TextView tv;
    uint64_t last;         // coordinate of the query's last valid start
    const uint64_t *steps; // the query's step table
    uint32_t halo;         // LDS halo bytes (multiple of 16, >= m + 4)
    uint32_t m;
    uint32_t r;            // peel factor, 1..min(kMaxPeel, m)
    uint32_t out;          // output slot
};

struct BatchDeal {
    uint32_t solo;         // index of the query's record
    uint32_t tiles;        // first tile within the text << 3 | number of tiles (1..2^chunk_log2 <= 7)
};

struct DealArgs {
    const BatchDeal *deals;
    const BatchSolo *solos;
    uint64_t ndeals;
    unsigned long long *counts;
    uint32_t halo_max;     // largest halo (LDS buffer size)
    uint32_t pad;
};

// Reporting batches, per query (same index as BatchQuery): nonzero per-vector
// counts (array zeroed before) and their sums per kGroupBlocks group, as the
// single-search report pass writes them.
struct BatchReport {
    uint32_t *block_counts;
    unsigned long long *group_sums;
};

// One query of a reporting batch, for the group scan and the ordered writes.
struct RepDesc {
    TextView tv;
    uint64_t last, nblocks;
    const uint64_t *steps;
    uint32_t m;
    uint32_t win;                  // per-wave LDS window bytes, or 0: read from global memory
    uint32_t *bc;                  // nonzero per-vector counts
    unsigned long long *gs, *go;   // group sums and their exclusive offsets
    unsigned long long *total;     // full count
    unsigned long long *pos;       // output segment
    uint64_t cap;
    uint64_t ngroups;
    uint64_t item0;                // first work item (group 0) of this query
};

struct BatchArgs {
    const BatchChunk *chunks;
    const uint32_t *tile_chunk;  // chunk of every global tile
    uint64_t ntiles;             // global tiles
    const BatchQuery *queries;
    const BatchReport *reports;  // reporting batches only (else null)
    const uint64_t *steps;
    unsigned long long *counts;
    uint32_t halo_max;           // largest chunk halo (LDS buffer size)
    uint32_t chunk_log2;         // tiles are dealt in chunks of 2^chunk_log2
};

// Batched bitmap mode: per tile, one bitmap per symbol the chunk's queries
// use (bit i of word w of slot c: the byte at tile position 32w + i is the
// symbol of slot c), then every query of a chunk runs over the tile with one
// funnel shift + AND per compare.
constexpr uint32_t kBmWG = 1024;             // threads per bitmap workgroup: 16 waves
constexpr uint32_t kBmWaves = kBmWG / 64;
constexpr uint32_t kBmT = 8192;              // starts per bitmap tile: kBmV vectors of 64 lanes x 32 bits
constexpr int kBmV = (int)(kBmT / 2048);
constexpr uint32_t kBmQChunk = 1024;         // largest number of queries per bitmap work item
constexpr uint32_t kBmMaxLds = 163840;       // LDS per workgroup on gfx950
// Per query, a record of kBmRecWords dwords: [0] m | r << 24, [1] index of its full step table
// in the step pool, [2 .. 2 + kBmRecSteps) its first step entries (entries past m repeat entry m-1).
constexpr uint32_t kBmRecWords = 8;
constexpr uint32_t kBmRecSteps = kBmRecWords - 2;
// LDS bytes of a work item besides its bitmaps: the symbol map plus, per query, the record and a counter
constexpr uint32_t kBmSmapBytes = 256 * 4;
constexpr uint32_t kBmPerQueryLds = kBmRecWords * 4 + 4;

struct BmItem {
    TextView tv;
    uint64_t tile_begin, tile_end;  // tiles of kBmT starts
    uint64_t last_min;              // coordinate of the last valid start of the chunk's longest query
    uint32_t q_begin, q_end;        // into the query records
    uint32_t wps;                   // bitmap words per slot (multiple of 4) >= kBmT / 32 + 2 + ceil(m_max / 32)
    uint32_t nslots;                // bitmap slots (symbols the chunk's text's queries use)
    const uint8_t *smap;            // 256 bytes: symbol -> slot, 0xFF if no query uses the symbol
};

// Bitmap step entry (uint32), for compare l of a query with j = pi(l):
//   ((slot * wps + (j >> 5)) << 7) | (j & 31)
// i.e. the LDS byte offset of the slot's word holding bit j, shifted left by 5, and j mod 32.

struct BmArgs {
    const BmItem *items;
    uint64_t nitems;
    const uint32_t *recs;   // kBmRecWords per query
    const uint32_t *outs;   // output slot of each query
    const uint32_t *steps;  // full step tables
    unsigned long long *counts;
};

// LDS bytes a bitmap work item needs: bitmaps, symbol map, records, counters and the group counter.
inline uint64_t bm_item_lds(uint32_t nslots, uint32_t wps, uint32_t nq)
{
    return (uint64_t)nslots * wps * 4 + kBmSmapBytes + (uint64_t)nq * kBmPerQueryLds + 16;
}

// Single search over per-tile symbol bitmaps (patterns of at most kBcMaxSyms distinct symbols).
// A tile is W = kWG * CPW words of 32 coordinates per slot; its last halo_words words carry no
// starts (they hold the bits the funnel shifts of the other words reach), so a tile has
// 32 * (W - halo_words) starts.
constexpr uint32_t kBcMaxSyms = 4;
struct BmCountArgs {
    TextView tv;
    uint64_t last;             // coordinate of the last valid start: first + n - m
    uint64_t ntiles;           // tiles covering coordinates [0, last]
    const uint64_t *steps;     // device step table (m + kStepPad entries)
    unsigned long long *count; // += total count
    uint32_t m;
    uint32_t r;                // peel factor, 1..min(kMaxPeel, m)
    uint32_t syms;             // the pattern's distinct symbols: byte c is the symbol of slot c
    uint32_t halo_words;       // ((m - 1) >> 5) + 1, at most half a tile's words
    uint32_t chunk_log2;       // tiles are dealt in chunks of 2^chunk_log2 contiguous tiles
    uint32_t pad;
};

// Batched single-query texts through bitmap tiles of kBmDealCpw x 8 KiB: a query's record (its
// tiles have 32 * (kWG * kBmDealCpw - halo_words) starts) and deals (BatchDeal: record index,
// first tile << 3 | tiles).  16 KiB tiles measured 3-4% faster than 8 KiB on 4,096 texts of
// 4 KiB-4 MiB, and 32 KiB no faster than 16.
constexpr uint32_t kBmDealCpw = 2;
struct BmSolo {
    TextView tv;
    uint64_t last;             // coordinate of the query's last valid start
    const uint64_t *steps;     // its step table
    uint32_t m;
    uint32_t r;                // peel factor, 1..min(kMaxPeel, m)
    uint32_t syms;             // its distinct symbols, padded to kBcMaxSyms by repeating the first
    uint32_t halo_words;       // ((m - 1) >> 5) + 1, at most kWG / 2
    uint32_t out;              // output slot
    uint32_t pad;
};

struct BmDealArgs {
    const BatchDeal *deals;
    const BmSolo *solos;
    uint64_t ndeals;
    unsigned long long *counts;
};

// Host-side launchers (sm_kernels.hip).  Each returns a hipError_t.
// stream_loads: tile loads with the non-temporal cache policy (texts far larger than the last-level cache)
hipError_t launch_count_staged(const CountArgs &a, int cpl, int r, bool stream_loads, unsigned grid, hipStream_t s);
hipError_t launch_count_global(const CountArgs &a, int r, unsigned grid, hipStream_t s);
// ns: distinct pattern symbols (1..kBcMaxSyms); cpw: bitmap words per thread and tile (1, 2 or 4)
hipError_t launch_count_bitmap(const BmCountArgs &a, int ns, int cpw, bool stream_loads, unsigned grid, hipStream_t s);
// halo_max: the largest halo_words of the deals' records (LDS pad)
hipError_t launch_bm_deals(const BmDealArgs &a, uint32_t halo_max, bool stream_loads, unsigned grid, hipStream_t s);
hipError_t launch_scan_groups(const unsigned long long *gs, uint64_t ngroups, unsigned long long *go,
                              unsigned long long *total, hipStream_t s);
hipError_t launch_report_write(const CountArgs &a, uint32_t *bc, unsigned long long *gs, const unsigned long long *go,
                               uint64_t ngroups, unsigned long long *pos, uint64_t cap, uint32_t win, unsigned grid,
                               hipStream_t s);
hipError_t launch_fill_report(uint32_t *bc, uint64_t nblocks, unsigned long long *gs, uint64_t ngroups,
                              hipStream_t s);
hipError_t launch_hist(const TextView &tv, unsigned long long *hist, bool stream_loads, unsigned grid, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_batch_staged(const BatchArgs &a, int cpl, bool stream_loads, unsigned grid, hipStream_t s);
hipError_t launch_batch_deals(const DealArgs &a, int cpl, bool stream_loads, unsigned grid, hipStream_t s);
// two_per_cu: lds_bytes lets two workgroups share a CU (the register-capped instance runs)
hipError_t launch_batch_bitmap(const BmArgs &a, unsigned grid, uint32_t lds_bytes, bool two_per_cu, hipStream_t s);
// Non-overlapping selection over the ascending occurrence list (c entries).
constexpr uint64_t kNoChunkEntries = 4 * kWG;  // list entries per compaction chunk
hipError_t launch_no_next(const unsigned long long *pos, uint64_t c, uint32_t m, uint32_t *nxt, uint32_t *mark,
                          unsigned long long *overlapped, hipStream_t s);
hipError_t launch_no_round(const uint32_t *nxt, uint32_t *nxt_out, uint32_t *mark, uint64_t c, hipStream_t s);
hipError_t launch_no_chunk_counts(const uint32_t *mark, uint64_t c, unsigned long long *gs, uint64_t ng,
                                  hipStream_t s);
hipError_t launch_no_compact(const unsigned long long *pos, const uint32_t *mark, uint64_t c,
                             const unsigned long long *go, uint64_t ng, unsigned long long *out, uint64_t cap,
                             hipStream_t s);
hipError_t launch_bigram(const TextView &tv, uint32_t half, unsigned long long *out, unsigned grid, hipStream_t s);
hipError_t launch_report_multi(const RepDesc *descs, uint64_t nq, const uint32_t *item_query, uint64_t nitems,
                               uint32_t win_max, unsigned grid, hipStream_t s);
// Sets the dynamic-LDS limits of all kernels on the current device.
hipError_t prime_kernel_attrs();

}  // namespace smk
