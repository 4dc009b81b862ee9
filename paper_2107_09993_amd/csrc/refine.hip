// K5: the exact refine of one instance over the whole GPU (the lane loop is in
// refine_core.h).  Work items are in Morton order of their cells and split
// into kNumXcd contiguous shares with one queue each; workgroup b starts on
// share b % kNumXcd (the XCD it is dispatched to), so the waves sharing an L2
// work on neighbouring cells and their cones, and moves on to the other shares
// once its own is empty.  A wave takes `chunk` items per atomic: small chunks
// keep the waves of an XCD on a narrow front of neighbouring cells.
#include <cstdlib>

#include "common.h"
#include "refine_core.h"
#include "refine_mc.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kRefineThreads = 256;

struct XcdFeeder {
    uint32_t *heads;   // kNumXcd queue heads
    uint32_t n_items;
    uint32_t chunk;
    int share;         // wave-uniform
    int shares_left;

    __device__ bool next(uint32_t &lo, uint32_t &hi)
    {
        while (shares_left > 0) {
            const uint32_t s_lo = (uint32_t)(((uint64_t)n_items * share) / kNumXcd);
            const uint32_t s_hi = (uint32_t)(((uint64_t)n_items * (share + 1)) / kNumXcd);
            uint32_t base = 0u;
            if (__lane_id() == 0) base = atomicAdd(&heads[share], chunk);
            base = __shfl(base, 0) + s_lo;
            if (base < s_hi) {
                lo = base;
                hi = base + chunk < s_hi ? base + chunk : s_hi;
                return true;
            }
            share = share + 1 == kNumXcd ? 0 : share + 1;
            --shares_left;
        }
        return false;
    }
};

// Walk records (common.h) of every cell, after the scatter: the record's
// lower-neighbour mask and the bytewise minimum of the screening columns of the
// cell's sorted points, halved into 6-bit fields.  One lane per cell; a cell
// with more than kWrecLanePoints points is reduced by the whole wave together
// (strided loads, then a butterfly of bytewise minima).  Every lane of the
// launch stays active to the end (lanes past the last cell hold no points), so
// the butterfly sees all 64 lanes.
constexpr uint32_t kWrecLanePoints = 32;

// Bytewise minimum of two words of 7-bit bytes.
__device__ __forceinline__ uint64_t bytes_min(uint64_t a, uint64_t b)
{
    const uint64_t ge = ((b | kHigh) - a) & kHigh;  // top bit of a byte: b >= a there
    const uint64_t sel = (ge - (ge >> 7)) | ge;     // 0xFF in those bytes
    return (a & sel) | (b & ~sel);
}

template <int D>
__global__ __launch_bounds__(kRefineThreads) void k_wrec(const uint64_t *__restrict__ rec,
                                                         const uint64_t *__restrict__ fkeys,
                                                         uint64_t *__restrict__ wrec, uint32_t cells)
{
    constexpr uint32_t kAll = (1u << D) - 1u;
    constexpr uint64_t kNone = 0x7F7F7F7F7F7F7F7Full;
    const uint32_t x = blockIdx.x * kRefineThreads + threadIdx.x;
    const bool mine = x < cells;
    const uint64_t r = mine ? rec[x] : 0ull;
    uint32_t s = 0u, c = 0u;
    if (rec_surv(r)) {
        s = rec_start(r);
        c = rec_count(r);
        if (c == kRecCountSat) c = rec_start(rec[x + 1]) - s;
    }
    uint64_t mn = kNone;
    const uint32_t own = c <= kWrecLanePoints ? c : 0u;
    for (uint32_t i = 0; i < own; ++i) mn = bytes_min(mn, fkeys[s + i]);
    uint64_t big = __ballot(c > kWrecLanePoints);
    while (big != 0ull) {
        const int l = __builtin_ctzll(big);
        big &= big - 1ull;
        const uint32_t bs = __builtin_amdgcn_readlane(s, l);
        const uint32_t bc = __builtin_amdgcn_readlane(c, l);
        uint64_t part = kNone;
        for (uint32_t i = __lane_id(); i < bc; i += kWave) part = bytes_min(part, fkeys[bs + i]);
        for (int off = kWave / 2; off > 0; off >>= 1) part = bytes_min(part, __shfl_xor(part, off));
        if (__lane_id() == (unsigned)l) mn = part;
    }
    if (!mine) return;
    uint64_t wv = 0ull;
#pragma unroll
    for (int k = 0; k < D; ++k) wv |= ((mn >> (8 * k + 1)) & 0x3Full) << (7 * k);
    reinterpret_cast<ulonglong2 *>(wrec)[x] = make_ulonglong2(wv | ((uint64_t)(rec_nbr(r) & kAll) << 56), wv);
}

// Fieldwise minimum of two words of 6-bit fields in 7-bit slots (guard bits zero).
__device__ __forceinline__ uint64_t fields_min(uint64_t a, uint64_t b)
{
    constexpr uint64_t kG = wrec_guards();
    const uint64_t ge = ((b | kG) - a) & kG;  // guard bit of a field: b >= a there
    const uint64_t sel = (ge - (ge >> 6)) | ge;
    return (a & sel) | (b & ~sel);
}

// Prefix minimum of the walk records' first words over the first P dimensions
// (word 2x, common.h).  One workgroup per tile: the 2^(P*r) cells that share the
// index bits outside the P dimensions; tile element t has bit b*P + k for index
// bit b*D + k.  Per dimension k and column bit b, in increasing b, every element
// with that bit set takes the minimum with the element that has it cleared and
// dimension k's lower column bits all set: afterwards each element holds the
// minimum over the elements <= it in those dimensions.
template <int D>
__global__ __launch_bounds__(kRefineThreads) void k_wrec_prefix(uint64_t *__restrict__ wrec, int r, int pdims,
                                                                uint32_t cells)
{
    __shared__ uint64_t s_v[1u << kWrecTileBits];
    __shared__ uint8_t s_nb[1u << kWrecTileBits];
    const int tb = pdims * r;
    const uint32_t tsize = 1u << tb;
    uint32_t inmask = 0u;
    for (int b = 0; b < r; ++b)
        for (int k = 0; k < pdims; ++k) inmask |= 1u << (b * D + k);
    // the tile number's bits, in order, at the index bits outside the tile
    const uint32_t outmask = (cells - 1u) & ~inmask;
    uint32_t base = 0u, tile = blockIdx.x;
    for (int p = 0; p < 32 && tile != 0u; ++p) {
        if ((outmask >> p) & 1u) {
            base |= (tile & 1u) << p;
            tile >>= 1;
        }
    }
    const uint32_t lowdims = (1u << pdims) - 1u;
    auto cell_of = [&](uint32_t t) {
        uint32_t xi = base;
        for (int b = 0; b < r; ++b) xi |= ((t >> (b * pdims)) & lowdims) << (b * D);
        return xi;
    };
    for (uint32_t t = threadIdx.x; t < tsize; t += kRefineThreads) {
        const uint64_t w = wrec[2 * (size_t)cell_of(t)];
        s_v[t] = w & kWrecFields;
        s_nb[t] = (uint8_t)(w >> 56);
    }
    __syncthreads();
    for (int k = 0; k < pdims; ++k) {
        uint32_t low = 0u;
        for (int b = 0; b < r; ++b) {
            const int pos = b * pdims + k;
            const uint32_t pbit = 1u << pos;
            for (uint32_t u = threadIdx.x; u < tsize / 2; u += kRefineThreads) {
                const uint32_t t = ((u >> pos) << (pos + 1)) | pbit | (u & (pbit - 1u));
                s_v[t] = fields_min(s_v[t], s_v[(t & ~pbit) | low]);
            }
            __syncthreads();
            low |= pbit;
        }
    }
    for (uint32_t t = threadIdx.x; t < tsize; t += kRefineThreads)
        wrec[2 * (size_t)cell_of(t)] = s_v[t] | ((uint64_t)s_nb[t] << 56);
}

template <int D, int M, bool MC>
__global__ __launch_bounds__(kRefineThreads) void k_refine(const uint32_t *__restrict__ keys,
                                                           const uint64_t *__restrict__ fkeys,
                                                           const int32_t *__restrict__ sidx,
                                                           const uint64_t *__restrict__ rec,
                                                           const uint64_t *__restrict__ wrec,
                                                           const uint2 *__restrict__ items,
                                                           uint32_t *__restrict__ ctr,
                                                           uint8_t *__restrict__ flag, GridDesc gd,
                                                           uint32_t chunk, uint64_t *__restrict__ stats)
{
    __shared__ uint32_t s_mask[kMaxD], s_low[kMaxD];
    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= gd.mask[k];
        s_mask[threadIdx.x] = threadIdx.x < (unsigned)D ? gd.mask[threadIdx.x] : 0u;
        s_low[threadIdx.x] = low;
    }
    __syncthreads();

    const RefineView v{keys, fkeys, sidx, rec, items, flag, s_mask, s_low};
    XcdFeeder feed{ctr + kCtrHead, ctr[kCtrItems], chunk, (int)(blockIdx.x % kNumXcd), kNumXcd};
    uint32_t visits = 0u, tests = 0u;
    if constexpr (MC)
        refine_loop_mc<D, M>(v, wrec, wrec_prefix_dims(D, gd.r), feed, visits, tests);
    else
        refine_loop<D, M>(v, feed, visits, tests);

    if (stats != nullptr) {
        uint64_t v64 = visits, t64 = tests;
        for (int off = 32; off > 0; off >>= 1) {
            v64 += __shfl_xor(v64, off);
            t64 += __shfl_xor(t64, off);
        }
        if (__lane_id() == 0) {
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)v64);
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)t64);
        }
    }
}

// Items a wave takes from its share per atomic (SKYCELL_REFINE_CHUNK overrides
// it for tuning sweeps).
static uint32_t refine_chunk()
{
    static int chunk = -1;
    if (chunk < 0) {
        const char *v = getenv("SKYCELL_REFINE_CHUNK");
        chunk = v ? atoi(v) : 0;
        if (chunk < 1 || chunk > 4096) chunk = 32;
    }
    return (uint32_t)chunk;
}

// Resident workgroups per CU of one instantiation (queried once; the query is
// not a stream operation, but callers that capture graphs resolve it first).
template <int D, int M, bool MC>
static int refine_blocks_per_cu()
{
    static int blocks_per_cu = -1;
    if (blocks_per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_refine<D, M, MC>, kRefineThreads, 0) != hipSuccess ||
            b < 1)
            b = 1;
        // at most 4 resident workgroups per CU: more waves add L1/L2 misses
        // faster than they hide latency (SKYCELL_REFINE_BLOCKS overrides the cap
        // for tuning sweeps)
        const char *v = getenv("SKYCELL_REFINE_BLOCKS");
        const int cap = v ? atoi(v) : 4;
        if (cap >= 1 && cap < b) b = cap;
        blocks_per_cu = b;
    }
    return blocks_per_cu;
}

// Workgroups of a lane-form launch: enough to keep every CU at its resident
// limit, but no more than the items can use.  There are at most n items (each
// holds at least one point), and a wave takes `chunk` items per request, so
// n / (chunk * waves per workgroup) workgroups already give every wave work;
// small instances then leave the rest of the chip to concurrent kernels.
template <int D, int M, bool MC>
static unsigned refine_blocks(int64_t n, int num_cus)
{
    const uint64_t full = (uint64_t)num_cus * (uint64_t)refine_blocks_per_cu<D, M, MC>();
    const uint64_t per_block = (uint64_t)refine_chunk() * (kRefineThreads / kWave);
    const uint64_t need = ((uint64_t)(n > 0 ? n : 1) + per_block - 1) / per_block;
    return (unsigned)(need < full ? need : full);
}

// The lane form with walk records (d <= kWrecMaxD unless the plain lane form
// was asked for).
inline bool lane_mc(const GridDesc &gd) { return gd.d <= kWrecMaxD && gd.plain == 0; }

template <int D, int M>
static hipError_t launch_refine_dm(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                                   int num_cus, hipStream_t st)
{
    constexpr bool kCanMc = D <= kWrecMaxD;
    if (kCanMc && lane_mc(gd)) {
        const unsigned blocks = refine_blocks<D, M, kCanMc>(n, num_cus);
        hipLaunchKernelGGL((k_refine<D, M, kCanMc>), dim3(blocks), dim3(kRefineThreads), 0, st,
                           (const uint32_t *)ws.keys, (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx,
                           (const uint64_t *)ws.rec, (const uint64_t *)ws.wrec, (const uint2 *)ws.items, ws.ctr,
                           ws.flag, gd, refine_chunk(), stats);
        return hipGetLastError();
    }
    const unsigned blocks = refine_blocks<D, M, false>(n, num_cus);
    hipLaunchKernelGGL((k_refine<D, M, false>), dim3(blocks), dim3(kRefineThreads), 0, st,
                       (const uint32_t *)ws.keys, (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx,
                       (const uint64_t *)ws.rec, (const uint64_t *)nullptr, (const uint2 *)ws.items, ws.ctr,
                       ws.flag, gd, refine_chunk(), stats);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_refine_d(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                                  int num_cus, hipStream_t st)
{
    switch (gd.m) {
    case 1:
        return launch_refine_dm<D, 1>(n, gd, ws, stats, num_cus, st);
    case 2:
        return launch_refine_dm<D, 2>(n, gd, ws, stats, num_cus, st);
    case 4:
        return launch_refine_dm<D, 4>(n, gd, ws, stats, num_cus, st);
    default:
        return hipErrorInvalidValue;
    }
}

template <int D, int M>
static void prepare_dm(const GridDesc &gd)
{
    constexpr bool kCanMc = D <= kWrecMaxD;
    if (kCanMc && lane_mc(gd))
        (void)refine_blocks_per_cu<D, M, kCanMc>();
    else
        (void)refine_blocks_per_cu<D, M, false>();
}

template <int D>
static hipError_t prepare_d(const GridDesc &gd)
{
    switch (gd.m) {
    case 1:
        prepare_dm<D, 1>(gd);
        return hipSuccess;
    case 2:
        prepare_dm<D, 2>(gd);
        return hipSuccess;
    case 4:
        prepare_dm<D, 4>(gd);
        return hipSuccess;
    default:
        return hipErrorInvalidValue;
    }
}

// Walk records for the lane form's minimum-corner screen (after the scatter;
// nothing to do for the other forms).
hipError_t launch_walk_records(const GridDesc &gd, const Workspace &ws, hipStream_t st)
{
    if (gd.tile || gd.m == kWaveItemPoints || !lane_mc(gd)) return hipSuccess;
    const unsigned wb = (gd.cells + kRefineThreads - 1) / kRefineThreads;
    const int pdims = wrec_prefix_dims(gd.d, gd.r);
    const unsigned tiles = pdims > 0 ? gd.cells >> (pdims * gd.r) : 0u;
    switch (gd.d) {
#define SKYCELL_WREC_CASE(DD)                                                                              \
    case DD:                                                                                               \
        hipLaunchKernelGGL((k_wrec<DD>), dim3(wb), dim3(kRefineThreads), 0, st, (const uint64_t *)ws.rec,    \
                           (const uint64_t *)ws.fkeys, ws.wrec, gd.cells);                                  \
        if (tiles > 0)                                                                                     \
            hipLaunchKernelGGL((k_wrec_prefix<DD>), dim3(tiles), dim3(kRefineThreads), 0, st, ws.wrec, gd.r, \
                               pdims, gd.cells);                                                           \
        return hipGetLastError();
        SKYCELL_WREC_CASE(1)
        SKYCELL_WREC_CASE(2)
        SKYCELL_WREC_CASE(3)
        SKYCELL_WREC_CASE(4)
        SKYCELL_WREC_CASE(5)
        SKYCELL_WREC_CASE(6)
        SKYCELL_WREC_CASE(7)
        SKYCELL_WREC_CASE(8)
#undef SKYCELL_WREC_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// Resolve every host-side query the refine launch of this grid makes, so that
// the launch itself can be captured into a graph.
hipError_t refine_prepare(const GridDesc &gd)
{
    (void)refine_chunk();
    if (gd.tile) return refine_tile_prepare(gd);
    if (gd.m == kWaveItemPoints) return refine_wave_prepare(gd);
    switch (gd.d) {
#define SKYCELL_PREPARE_CASE(DD) \
    case DD:                     \
        return prepare_d<DD>(gd);
        SKYCELL_PREPARE_CASE(1)
        SKYCELL_PREPARE_CASE(2)
        SKYCELL_PREPARE_CASE(3)
        SKYCELL_PREPARE_CASE(4)
        SKYCELL_PREPARE_CASE(5)
        SKYCELL_PREPARE_CASE(6)
        SKYCELL_PREPARE_CASE(7)
        SKYCELL_PREPARE_CASE(8)
        SKYCELL_PREPARE_CASE(9)
        SKYCELL_PREPARE_CASE(10)
        SKYCELL_PREPARE_CASE(11)
        SKYCELL_PREPARE_CASE(12)
        SKYCELL_PREPARE_CASE(13)
        SKYCELL_PREPARE_CASE(14)
        SKYCELL_PREPARE_CASE(15)
        SKYCELL_PREPARE_CASE(16)
#undef SKYCELL_PREPARE_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_refine(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                         int num_cus, hipStream_t st)
{
    if (gd.tile) return launch_refine_tile(n, gd, ws, stats, num_cus, st);
    if (gd.m == kWaveItemPoints) return launch_refine_wave(n, gd, ws, stats, num_cus, st);
    switch (gd.d) {
#define SKYCELL_REFINE_CASE(DD) \
    case DD:                    \
        return launch_refine_d<DD>(n, gd, ws, stats, num_cus, st);
        SKYCELL_REFINE_CASE(1)
        SKYCELL_REFINE_CASE(2)
        SKYCELL_REFINE_CASE(3)
        SKYCELL_REFINE_CASE(4)
        SKYCELL_REFINE_CASE(5)
        SKYCELL_REFINE_CASE(6)
        SKYCELL_REFINE_CASE(7)
        SKYCELL_REFINE_CASE(8)
        SKYCELL_REFINE_CASE(9)
        SKYCELL_REFINE_CASE(10)
        SKYCELL_REFINE_CASE(11)
        SKYCELL_REFINE_CASE(12)
        SKYCELL_REFINE_CASE(13)
        SKYCELL_REFINE_CASE(14)
        SKYCELL_REFINE_CASE(15)
        SKYCELL_REFINE_CASE(16)
#undef SKYCELL_REFINE_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace skycell
