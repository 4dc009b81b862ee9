// K5: the exact refine of one instance over the whole GPU (the lane loop is in
// refine_core.h).  Work items are in Morton order of their cells and split
// into kNumXcd contiguous shares with one queue each (taken from the top of
// the share down); workgroup b starts on
// share b % kNumXcd (the XCD it is dispatched to), so the waves sharing an L2
// work on neighbouring cells and their cones, and moves on to the other shares
// once its own is empty.  A wave takes `chunk` items per atomic: small chunks
// keep the waves of an XCD on a narrow front of neighbouring cells, but every
// request is a device-scope atomic on one of eight queue heads; 64 items per
// request measured best (8 items per request made the headline refine 1.8x
// slower, 256 about 8% slower).
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
            base = __shfl(base, 0);
            if (base < s_hi - s_lo) {
                // from the top of the share down: the cells with the highest
                // columns, whose cone walks are the longest on average, are
                // handed out first and do not start near the end of the launch
                hi = s_hi - base;
                lo = hi - s_lo > chunk ? hi - chunk : s_lo;
                return true;
            }
            share = share + 1 == kNumXcd ? 0 : share + 1;
            --shares_left;
        }
        return false;
    }
};

template <int D, int M, bool MC>
__global__ __launch_bounds__(kRefineThreads) void k_refine(const uint32_t *__restrict__ keys,
                                                           const uint64_t *__restrict__ fkeys,
                                                           const int32_t *__restrict__ sidx,
                                                           const uint64_t *__restrict__ rec,
                                                           const uint64_t *__restrict__ wrec,
                                                           const uint2 *__restrict__ items,
                                                           uint32_t *__restrict__ ctr,
                                                           uint8_t *__restrict__ flag, GridDesc gd,
                                                           uint32_t chunk, uint32_t n, uint64_t *__restrict__ stats)
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
        refine_loop_mc<D, M>(v, wrec, wrec_prefix_dims(D, gd.r), n, gd.cells, feed, visits, tests);
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
        if (chunk < 1 || chunk > 4096) chunk = 64;
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
                           ws.flag, gd, refine_chunk(), (uint32_t)n, stats);
        return hipGetLastError();
    }
    const unsigned blocks = refine_blocks<D, M, false>(n, num_cus);
    hipLaunchKernelGGL((k_refine<D, M, false>), dim3(blocks), dim3(kRefineThreads), 0, st,
                       (const uint32_t *)ws.keys, (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx,
                       (const uint64_t *)ws.rec, (const uint64_t *)nullptr, (const uint2 *)ws.items, ws.ctr,
                       ws.flag, gd, refine_chunk(), (uint32_t)n, stats);
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
