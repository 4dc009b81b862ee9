// Shared definitions of the gfx950 skyline kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace skycell {

constexpr int kMaxD = 16;
constexpr uint32_t kMaxCells = 1u << 26;
constexpr int kWave = 64;

// Per-cell record, one 64-bit word per cell of the index space (plus one
// sentinel), read with a single load by the refine's cone walk:
//   bits  0..31  first sorted position of the cell's surviving points
//   bits 32..46  number of those points, saturated at kRecCountSat (then the
//                end is the next record's start)
//   bits 47..62  lower-neighbour mask: bit k set iff the cell one column lower
//                in dimension k exists and some non-empty cell lies in its
//                lower cone; for d <= 8 bits 55..62 hold the cell's slab count
//                when the lane form splits its items (cellops.h), else 0
//   bit  63      surviving non-empty cell: it holds points and no non-empty
//                cell has a smaller column in every dimension (Definition 3)
constexpr uint32_t kRecCountSat = 0x7FFFu;
__host__ __device__ __forceinline__ uint32_t rec_start(uint64_t r) { return (uint32_t)r; }
__host__ __device__ __forceinline__ uint32_t rec_count(uint64_t r) { return (uint32_t)(r >> 32) & kRecCountSat; }
__host__ __device__ __forceinline__ uint32_t rec_nbr(uint64_t r) { return (uint32_t)(r >> 47) & 0xFFFFu; }
__host__ __device__ __forceinline__ bool rec_surv(uint64_t r) { return (r >> 63) != 0u; }
__host__ __device__ __forceinline__ uint32_t rec_slabs(uint64_t r) { return (uint32_t)(r >> 55) & 0xFFu; }

// Coarse screening keys: every coordinate also gets a 7-bit column on a
// 128-column grid (same non-decreasing map as the cell columns), packed one
// byte per dimension, eight dimensions per 64-bit word.  q can dominate p only
// if every screening column of q is <= that of p.
constexpr int kFineCols = 128;
__host__ __device__ constexpr int fine_words(int d) { return (d + 7) / 8; }

// Default number of query points per work item of the lane form of the refine
// (measured: 2 beats 4 on fine grids, where cells hold ~2 points).
__host__ __device__ constexpr int items_per_group(int) { return 2; }

// Query points per work item of the wave form of the refine (one wave per item
// of one cell; the item's count field has 6 bits).  GridDesc::m takes this
// value when a call uses the wave form.
constexpr int kWaveItemPoints = 63;
constexpr int kMaxWaveParts = 64;

// Number of XCDs (each with its own L2) that workgroups are spread over
// round-robin; the refine gives each one a contiguous share of the work.
constexpr int kNumXcd = 8;

// Regular grid of g columns per dimension.  Cells are numbered in Morton (Z)
// order over r = ceil(log2 g) bits per dimension: bit b of column c[k] sits at
// index bit b*d + k.  Cells with a column >= g exist in the index space but
// never hold points.  Morton order is one of the cell orders the paper allows
// (Algorithm 1 sorts points by cell "in any order, e.g. Z-order") and keeps
// cells that are close in every dimension close in memory.
struct GridDesc {
    int32_t d;
    int32_t g;                 // columns per dimension
    int32_t r;                 // index bits per dimension
    uint32_t cells;            // 2^(r*d): size of the index space
    uint32_t mask[kMaxD];      // index bits that hold dimension k
    int32_t m;                 // query points per refine work item (1, 2 or 4)
    int32_t parts;             // wave form: waves that share one item's cone (>= 1)
    int32_t tile;              // 1: tile form of the refine (refine_tile.hip)
    int32_t plain;             // 1: lane form without the walk records' minimum corners
    int32_t split;             // 1: the longest cone walks of the lane form are split into slabs (cellops.h),
                               // 2: as many as the item array has room for
};

// Index of the cell one column lower / higher in the dimension whose bits are
// `m`.  Valid only when that column exists.
__host__ __device__ __forceinline__ uint32_t morton_dec(uint32_t x, uint32_t m)
{
    return (((x & m) - 1u) & m) | (x & ~m);
}
__host__ __device__ __forceinline__ uint32_t morton_inc(uint32_t x, uint32_t m)
{
    return (((x | ~m) + 1u) & m) | (x & ~m);
}
// Spread the low bits of v over the set bits of m (lowest first).
__host__ __device__ __forceinline__ uint32_t deposit_bits(uint32_t v, uint32_t m)
{
    uint32_t out = 0u;
    for (uint32_t bit = 1u; m != 0u; bit <<= 1) {
        const uint32_t low = m & (0u - m);
        if (v & bit) out |= low;
        m ^= low;
    }
    return out;
}

// Device scratch carved out of one workspace allocation.
struct Workspace {
    uint32_t *cell_of;    // [n]     cell of each input point
    uint32_t *rank;       // [n]     position of each point among the points of its cell
    uint32_t *cnt;        // [cells] points per cell
    uint64_t *lc;         // [cells / 64 + 1] lower closure bitmap: some non-empty cell <= this one
    uint64_t *rec;        // [cells + 1] cell records (see above)
    uint32_t *keys;       // [n * d] order-preserving keys of surviving points, AoS, sorted by cell
    uint64_t *fkeys;      // [n * fine_words(d)] packed screening columns, same order
    int32_t *sidx;        // [n]     original index of each sorted surviving point
    uint2 *items;         // [n]     refine work items
    uint8_t *flag;        // [n]     1 = skyline, by original index
    uint64_t *block_sums; // scan partials
    uint32_t *ctr;        // small counters, see CtrIndex
    uint64_t *survbits;   // [cells / 64 + 1] bit x: cell x is a surviving non-empty cell
    uint32_t *bcur;       // [kMaxScatterBuckets * kNumXcd] staging cursors of the two-pass scatter
    uint32_t *stage;      // [n * ((d + 6) & ~3)] staged rows of the two-pass scatter (large n only)
    uint64_t *wrec;       // [2 * cells] walk records of the lane refine (d <= kWrecMaxD only)
};

// Walk records of the lane refine, d <= kWrecMaxD: two words per cell x.
//   word 2x+1: bits 7k..7k+5 hold the minimum over the surviving points of
//     cell x of their screening column in dimension k halved (6 bits); bit
//     7k+6 is zero (a guard bit for fieldwise subtraction); 63 in every field
//     of the d dimensions for a cell without surviving points.
//   word 2x: bits 0..55 the fieldwise minimum of word 2y+1 over the cells y
//     that equal x outside the first P dimensions and are <= x in those
//     (P = wrec_prefix_dims(d, r)); bits 56..63 the lower-neighbour mask of
//     the cell record.
// A point of cell y can only dominate a point whose halved screening columns
// are all >= y's minima, so the refine's cone walk loads a cell's record and
// candidates only when that holds for some query point of its item; and when
// the walk arrives at y by a step along dimension j < P, the part of the cone
// it would walk below y (lower only in dimensions 0..j) is skipped entirely
// unless word 2y passes that test.
constexpr int kWrecMaxD = 8;
__host__ __device__ constexpr uint64_t wrec_guards()
{
    uint64_t gm = 0ull;
    for (int k = 0; k < kWrecMaxD; ++k) gm |= 1ull << (7 * k + 6);
    return gm;
}
constexpr uint64_t kWrecFields = 0x00FFFFFFFFFFFFFFull;
// Index bits of one tile of the prefix pass (its values fill 2^12 * 8 bytes of LDS).
constexpr int kWrecTileBits = 12;
// Dimensions of the prefix in word 2x: the first P dimensions, all their r
// index bits in one LDS tile, at most 4.
__host__ __device__ constexpr int wrec_prefix_dims(int d, int r)
{
    const int p = d < 4 ? d : 4;
    const int fit = r < 1 ? 0 : kWrecTileBits / r;
    return p < fit ? p : fit;
}

// Two-pass scatter, for large inputs.  Pass 1 groups the surviving points by
// ranges of 2^sh consecutive cells ("buckets") into a staging array whose
// bucket regions are the buckets' ranges of sorted positions; a staged row is
// (raw coordinate words, original index, cell, rank), padded to 16 bytes.  Pass 2 sweeps the
// staging array in order, each XCD over a contiguous eighth, and writes every
// row to its sorted position.  The rows in flight on one XCD then target a
// window of a few buckets that stays in its L2 until the window's lines are
// complete, instead of three partial-line writes to random places per point.
constexpr int64_t kScatterTwoPassMin = 1 << 20;
constexpr uint32_t kMaxScatterBuckets = 2048;
__host__ __device__ inline bool scatter_two_pass(int64_t n) { return n >= kScatterTwoPassMin; }
// Buckets: a power of two with 2^14 to 2^15 points each on average, between 64
// and kMaxScatterBuckets, and at most one per cell.
__host__ __device__ inline uint32_t scatter_buckets(int64_t n, uint32_t cells)
{
    uint32_t nb = 64u;
    while (nb < kMaxScatterBuckets && ((int64_t)nb << 15) <= n) nb <<= 1;
    return nb < cells ? nb : cells;
}

// Rank of a point that the pivot pre-filter removed (never a real rank: n < 2^31).
constexpr uint32_t kRankRemoved = 0xFFFFFFFFu;

enum CtrIndex {
    kCtrItems = 0,     // number of refine work items
    kCtrErr = 1,       // bit 0: NaN seen in the input; bit 1: pivot index out of range
    kCtrSurvPts = 2,   // number of surviving points
    kCtrPivSampled = 3,  // pivot pre-filter: sampled points of surviving cells
    kCtrPivHit = 4,      // ... of which a pivot dominates
    kCtrSplitThr = 5,    // float bits: cells whose cone-size product reaches it are split into slabs
    kCtrSplitItems = 6,  // work items of the surviving cells before the split
    kCtrSplitExtra = 7,  // items the split adds (no cell is split if they do not fit in n)
    kCtrHead = 8,      // kNumXcd refine work-queue heads, one per XCD share
    kCtrSplitFail = 16,  // nonzero: the split's added items passed the room (or wrapped)
    kCtrCount = 17     // number of 32-bit counters reserved
};

size_t workspace_layout(int64_t n, int d, uint32_t cells, Workspace *ws, char *base);

// ---- launchers (all enqueue on `st`; return hipSuccess or the launch error) ----
hipError_t launch_init(const Workspace &ws, const GridDesc &gd, uint64_t *stats, hipStream_t st);
hipError_t launch_quantize_hist(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                                int value_bits, const Workspace &ws, hipStream_t st);
// With gd.split, also picks the cells whose items are split into slabs
// (cellops.h); only for callers whose cell records stay as this pass writes
// them, since the split keeps the items within the n slots of the item array.
hipError_t launch_cell_prune(const GridDesc &gd, const Workspace &ws, int64_t n, uint64_t *stats, hipStream_t st);
// recount: the cell counts were taken again after the pivot pre-filter; the
// count field of every record is rewritten from them.
hipError_t launch_cell_scan(const GridDesc &gd, const Workspace &ws, int64_t n, uint64_t *stats, hipStream_t st,
                            bool recount = false);
hipError_t launch_scatter(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                          const Workspace &ws, int value_bits, int num_cus, hipStream_t st);
// The lane form of the refine reads walk records (d <= kWrecMaxD unless the
// plain lane form was asked for).
// The walk-record loop addresses its arrays with 32-bit buffer offsets (items
// and screening words take 8 bytes per point), so larger inputs get the plain
// lane form (pipeline_desc sets gd.plain).
constexpr int64_t kWrecMaxPoints = (int64_t)1 << 28;
static_assert((kMaxD & (kMaxD - 1)) == 0, "the walk's shared tables are indexed modulo kMaxD");
inline bool lane_mc(const GridDesc &gd) { return gd.d <= kWrecMaxD && gd.plain == 0; }
// Work items of the walk-record lane form whose cone walks are expected to be
// the longest are split into one item per slab of the cone (cellops.h); the
// item flag of such a slab item:
constexpr uint32_t kItemSlab = 1u << 31;
inline bool lane_split(const GridDesc &gd)
{
    return lane_mc(gd) && gd.tile == 0 && gd.m != kWaveItemPoints && gd.d >= 2;
}
// Work items per split item (SKYCELL_SPLIT_SHARE overrides it for tuning
// sweeps; 0 splits nothing).
uint32_t split_share();
// Walk records of the lane form (walk_records.hip), built from the sorted
// points; launch_scatter ends with it.
hipError_t launch_walk_records(const GridDesc &gd, const Workspace &ws, int64_t n, hipStream_t st);
hipError_t launch_refine(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                         int num_cus, hipStream_t st);
hipError_t refine_prepare(const GridDesc &gd);
// Wave form (refine_wave.hip), used when gd.m == kWaveItemPoints.
hipError_t launch_refine_wave(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                              hipStream_t st);
hipError_t refine_wave_prepare(const GridDesc &gd);
// Tile form (refine_tile.hip), used when gd.tile is set: 2 <= d <= 8, g = 2^r <= 128.
bool tile_form_supported(int d, int g);
hipError_t launch_refine_tile(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                              hipStream_t st);
hipError_t refine_tile_prepare(const GridDesc &gd);
hipError_t launch_output(int64_t n, const Workspace &ws, int32_t *out_idx, int32_t *out_count,
                         uint64_t *stats, hipStream_t st);
hipError_t launch_write_zero_count(int32_t *out_count, hipStream_t st);

// ---- device helpers ----
#if defined(__HIPCC__)
// Order-preserving key of a binary32 value: key(a) < key(b) iff a < b, with
// -0.0 mapped to the key of +0.0.  Comparing keys as integers is exact for
// subnormals whatever the floating-point denormal mode.
__device__ __forceinline__ uint32_t f32_key(float v)
{
    uint32_t b = __float_as_uint(v);
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
#endif

}  // namespace skycell
