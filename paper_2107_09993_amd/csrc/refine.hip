// K5: exact refine of the surviving points (SkyCell paper, Algorithm 1,
// RefineSkyline, with the cross-cell correction below).
//
// A point p can only be dominated by a point q whose cell is <= cell(p) in
// every dimension (the column map is non-decreasing).  The paper refines each
// candidate cell on its own, which misses dominators in other candidate cells
// that share a column with cell(p); this kernel instead checks p against every
// surviving point of every non-empty cell in the lower cone of cell(p).  All
// such cells survive the cell-domination prune (a cell below a surviving cell
// cannot be dominated), and pruned points never need to be candidates because
// whatever dominates them also dominates anything they dominate.
//
// Cone walk: the cells y <= x are enumerated as x - delta, delta >= 0, by a
// depth-first walk that lowers dimensions in non-decreasing order (each cell is
// reached by exactly one such path).  A step down in dimension k is taken only
// if the info word of the current cell says that the cone below x - e_k still
// holds a non-empty cell (lower-closure bit), which prunes the empty part of the
// cone.  The walk keeps no stack: delta, packed in fixed-width fields, tells
// which dimension to step back up in.
//
// Mapping: one lane owns one work item (up to M query points of one cell, their
// keys in registers) and walks its cone; lanes whose item ends take new items
// from a global queue, a batch per wave, so that unequal cone sizes do not idle
// the wave.  Every loop turn a lane does one unit of work: test one candidate
// point against its live query points, or one step of the walk.
#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kRefineThreads = 256;
constexpr int kRefillMin = 16;

template <int D>
__global__ __launch_bounds__(kRefineThreads) void k_refine(const uint32_t *__restrict__ keys,
                                                           const int32_t *__restrict__ sidx,
                                                           const uint32_t *__restrict__ info,
                                                           const uint32_t *__restrict__ offs,
                                                           const uint2 *__restrict__ items,
                                                           uint32_t *__restrict__ ctr,
                                                           uint8_t *__restrict__ flag, GridDesc gd,
                                                           uint64_t *__restrict__ stats)
{
    constexpr int M = items_per_group(D);
    __shared__ uint32_t s_stride[kMaxD];
    if (threadIdx.x < kMaxD) s_stride[threadIdx.x] = threadIdx.x < (unsigned)D ? gd.stride[threadIdx.x] : 0u;
    __syncthreads();

    const uint32_t n_items = ctr[kCtrItems];
    const int logw = gd.log_w;
    const int lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    uint32_t q[M][D];
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int k = 0; k < D; ++k) q[t][k] = 0u;
    uint32_t alive = 0u, qstart = 0u;
    uint32_t x = 0u, nb = 0u, cur = 0u, end = 0u;
    uint64_t delta = 0ull;
    int mode = 0;  // 0 idle, 1 testing the points of the current cell, 2 walking the cone
    bool exhausted = false;
    uint64_t visits = 0ull, tests = 0ull;

    for (;;) {
        // ---- refill idle lanes from the global queue, a batch per wave
        const bool wants = (mode == 0) && !exhausted;
        const uint64_t want = __ballot(wants);
        const uint64_t busy = __ballot(mode != 0);
        if (want != 0ull && (__popcll(want) >= kRefillMin || busy == 0ull)) {
            const int leader = __ffsll((unsigned long long)want) - 1;
            uint32_t base = 0u;
            if (lane == leader) base = atomicAdd(&ctr[kCtrHead], (uint32_t)__popcll(want));
            base = __shfl(base, leader);
            if (wants) {
                const uint32_t my = base + (uint32_t)__popcll(want & below);
                if (my < n_items) {
                    const uint2 it = items[my];
                    const uint32_t qc = it.y >> 26;
                    qstart = it.x;
                    x = it.y & ((1u << 26) - 1u);
#pragma unroll
                    for (int t = 0; t < M; ++t)
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            q[t][k] = (t < (int)qc) ? keys[(size_t)(qstart + t) * D + k] : 0u;
                    alive = (1u << qc) - 1u;
                    delta = 0ull;
                    nb = info[x] & kNbrMask;
                    cur = offs[x];
                    end = offs[x + 1];
                    mode = 1;
                    ++visits;
                } else {
                    exhausted = true;
                }
            }
        }
        if (__ballot(mode != 0) == 0ull) break;

        if (mode == 1) {
            // ---- one candidate point against the live query points (Definition 1)
            uint32_t c[D];
#pragma unroll
            for (int k = 0; k < D; ++k) c[k] = keys[(size_t)cur * D + k];
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (alive & (1u << t)) {
                    bool le = true, ne = false;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        le = le && (c[k] <= q[t][k]);
                        ne = ne || (c[k] != q[t][k]);
                    }
                    if (le && ne) alive &= ~(1u << t);
                    ++tests;
                }
            }
            ++cur;
            if (alive == 0u)
                mode = 0;  // every query point of the item is dominated
            else if (cur == end)
                mode = 2;
        } else if (mode == 2) {
            if (nb != 0u) {
                // ---- step down in the lowest allowed dimension
                const int k = __ffs(nb) - 1;
                x -= s_stride[k];
                delta += 1ull << (k << logw);
                const uint32_t inf = info[x];
                nb = inf & kNbrMask & ~((1u << k) - 1u);
                ++visits;
                if (inf & kOccBit) {
                    cur = offs[x];
                    end = offs[x + 1];
                    mode = 1;
                }
            } else if (delta == 0ull) {
                // ---- cone exhausted: the live query points are skyline points
#pragma unroll
                for (int t = 0; t < M; ++t)
                    if (alive & (1u << t)) flag[sidx[qstart + t]] = 1;
                mode = 0;
            } else {
                // ---- step back up along the last lowered dimension
                const int k = (63 - __clzll((long long)delta)) >> logw;
                x += s_stride[k];
                delta -= 1ull << (k << logw);
                nb = info[x] & kNbrMask & ~((2u << k) - 1u);
            }
        }
    }

    if (stats != nullptr) {
        for (int off = 32; off > 0; off >>= 1) {
            visits += __shfl_xor(visits, off);
            tests += __shfl_xor(tests, off);
        }
        if (lane == 0) {
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)visits);
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)tests);
        }
    }
}

template <int D>
static hipError_t launch_refine_d(const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                                  int num_cus, hipStream_t st)
{
    static int blocks_per_cu = -1;
    if (blocks_per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_refine<D>, kRefineThreads, 0) != hipSuccess || b < 1)
            b = 1;
        blocks_per_cu = b;
    }
    const unsigned blocks = (unsigned)(num_cus * blocks_per_cu);
    hipLaunchKernelGGL(k_refine<D>, dim3(blocks), dim3(kRefineThreads), 0, st,
                       (const uint32_t *)ws.keys, (const int32_t *)ws.sidx, (const uint32_t *)ws.info,
                       (const uint32_t *)ws.offs, (const uint2 *)ws.items, ws.ctr, ws.flag, gd, stats);
    return hipGetLastError();
}

hipError_t launch_refine(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                         int num_cus, hipStream_t st)
{
    (void)n;
    switch (gd.d) {
#define SKYCELL_REFINE_CASE(DD) \
    case DD:                    \
        return launch_refine_d<DD>(gd, ws, stats, num_cus, st);
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
