// Grid phase of the skyline path (SkyCell paper, Section III grid structure and
// Section V, Algorithm 1 line 1):
//   K1  quantise every point to its cell (Equation 1), build the occupancy
//       histogram and keep each point's rank inside its cell;
//   K3  lower closure of the occupancy by d prefix-OR passes, then per cell the
//       "dominated" test of Definition 3 and the lower-neighbour mask used by the
//       refine's cone walk;
//   K2  exclusive scan of surviving-cell counts: counting-sort offsets and refine
//       work items;
//   K4  scatter of surviving points, grouped by cell, as order-preserving keys.
#include "cellops.h"
#include "common.h"
#include "scan.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kThreads = 256;

static inline dim3 grid_for(uint64_t count, int per_block = kThreads)
{
    uint64_t b = (count + per_block - 1) / per_block;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(kThreads) void k_init(uint32_t *cnt, uint32_t cells, uint32_t *ctr,
                                                   uint64_t *stats, int32_t g)
{
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t i = gid; i < cells; i += stride) cnt[i] = 0u;
    if (gid < kCtrCount) ctr[gid] = 0u;
    if (stats != nullptr && gid < SKYCELL_NUM_STATS)
        stats[gid] = gid == SKYCELL_STAT_GRID_RES ? (uint64_t)g : 0ull;
}

hipError_t launch_init(const Workspace &ws, const GridDesc &gd, uint64_t *stats, hipStream_t st)
{
    uint32_t blocks = (gd.cells + kThreads * 8 - 1) / (kThreads * 8);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(kThreads), 0, st, ws.cnt, gd.cells, ws.ctr, stats, gd.g);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K1
template <typename T>
__global__ __launch_bounds__(kThreads) void k_quantize_hist(const T *__restrict__ pts, uint32_t n,
                                                            GridDesc gd, int value_bits,
                                                            uint32_t *__restrict__ cell_of,
                                                            uint32_t *__restrict__ rank,
                                                            uint32_t *__restrict__ cnt,
                                                            uint32_t *__restrict__ ctr)
{
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    bool nan = false;
    const uint32_t cell = point_cell(pts, n, i, gd, value_bits, nan);
    cell_of[i] = cell;
    rank[i] = atomicAdd(&cnt[cell], 1u);
    if (nan) atomicOr(&ctr[kCtrErr], 1u);
}

hipError_t launch_quantize_hist(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                                int value_bits, const Workspace &ws, hipStream_t st)
{
    if (dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_quantize_hist<float>, grid_for(n), dim3(kThreads), 0, st,
                           (const float *)pts, (uint32_t)n, gd, value_bits, ws.cell_of, ws.rank,
                           ws.cnt, ws.ctr);
    else
        hipLaunchKernelGGL(k_quantize_hist<uint16_t>, grid_for(n), dim3(kThreads), 0, st,
                           (const uint16_t *)pts, (uint32_t)n, gd, value_bits, ws.cell_of, ws.rank,
                           ws.cnt, ws.ctr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K3
// lc[x] = 1 iff some non-empty cell y has y <= x in every dimension.  Built as
// the occupancy followed by an inclusive prefix-OR along each dimension.
__global__ __launch_bounds__(kThreads) void k_lc_init(const uint32_t *__restrict__ cnt,
                                                      uint8_t *__restrict__ lc, uint32_t cells)
{
    const uint32_t x = blockIdx.x * kThreads + threadIdx.x;
    if (x < cells) lc[x] = cnt[x] != 0u ? 1 : 0;
}

// One thread per line of cells that differ only in the dimension whose index
// bits are `m`; the line is walked from column 0 up to column g-1.
__global__ __launch_bounds__(kThreads) void k_lc_prefix(uint8_t *__restrict__ lc, uint32_t lines,
                                                        uint32_t m, uint32_t all_bits, uint32_t g)
{
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    if (t < lines) lc_prefix_line(lc, t, m, all_bits, g);
}

// Per cell: the high half of the cell record (see cellops.h); the scan fills
// in the low half (first sorted position).
__global__ __launch_bounds__(kThreads) void k_cell_rec(GridDesc gd, const uint32_t *__restrict__ cnt,
                                                       const uint8_t *__restrict__ lc,
                                                       uint64_t *__restrict__ rec,
                                                       uint64_t *__restrict__ stats)
{
    const uint32_t x = blockIdx.x * kThreads + threadIdx.x;
    bool occ = false, surv = false;
    if (x < gd.cells) rec[x] = cell_record(gd, cnt, lc, x, occ, surv);
    if (stats != nullptr) {
        const uint64_t bo = __ballot(occ), bs = __ballot(surv);
        if (__lane_id() == 0) {
            if (bo) atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_NONEMPTY_CELLS],
                              (unsigned long long)__popcll(bo));
            if (bs) atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_SURVIVING_CELLS],
                              (unsigned long long)__popcll(bs));
        }
    }
}

hipError_t launch_cell_prune(const GridDesc &gd, const Workspace &ws, uint64_t *stats, hipStream_t st)
{
    hipLaunchKernelGGL(k_lc_init, grid_for(gd.cells), dim3(kThreads), 0, st, ws.cnt, ws.lc, gd.cells);
    if (gd.g > 1) {
        const uint32_t lines = gd.cells >> gd.r;
        const uint32_t all_bits = gd.cells - 1u;
        for (int k = 0; k < gd.d; ++k)
            hipLaunchKernelGGL(k_lc_prefix, grid_for(lines), dim3(kThreads), 0, st, ws.lc, lines,
                               gd.mask[k], all_bits, (uint32_t)gd.g);
    }
    hipLaunchKernelGGL(k_cell_rec, grid_for(gd.cells), dim3(kThreads), 0, st, gd, ws.cnt, ws.lc,
                       ws.rec, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K2
__global__ void k_cell_scan_total(const uint64_t *block_sums, uint32_t nb, uint32_t cells,
                                  uint64_t *rec, uint32_t *ctr, uint64_t *stats)
{
    const uint64_t tot = block_sums[nb];
    rec[cells] = (uint32_t)tot;  // sentinel: start of "the cell after the last"
    ctr[kCtrSurvPts] = (uint32_t)tot;
    ctr[kCtrItems] = (uint32_t)(tot >> 32);
    if (stats != nullptr) {
        stats[SKYCELL_STAT_SURVIVOR_POINTS] = (uint32_t)tot;
        stats[SKYCELL_STAT_ITEMS] = tot >> 32;
    }
}

hipError_t launch_cell_scan(const GridDesc &gd, const Workspace &ws, uint64_t *stats, hipStream_t st,
                            bool recount)
{
    const uint32_t m = (uint32_t)gd.m;
    CellLoader ld{ws.rec, ws.cnt, m};
    CellEmitter em{(uint32_t *)ws.rec, ws.items, m, recount};
    hipError_t e = enqueue_scan<uint64_t>(ld, em, gd.cells, ws.block_sums, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_scan_total, dim3(1), dim3(1), 0, st, (const uint64_t *)ws.block_sums,
                       scan_tiles(gd.cells), gd.cells, ws.rec, ws.ctr, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K4
// Counting-sort scatter of the points of surviving cells: slot = first sorted
// position of the cell + the point's rank from the histogram atomic, so the
// order inside a cell follows the histogram's (arbitrary) order; the skyline
// does not depend on it.  Writes the exact keys and the packed screening
// columns, and clears the output flag of every point.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(const T *__restrict__ pts, uint32_t n, int d,
                                                      int value_bits,
                                                      const uint32_t *__restrict__ cell_of,
                                                      const uint32_t *__restrict__ rank,
                                                      const uint64_t *__restrict__ rec,
                                                      uint32_t *__restrict__ keys,
                                                      uint64_t *__restrict__ fkeys,
                                                      int32_t *__restrict__ sidx,
                                                      uint8_t *__restrict__ flag)
{
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    flag[i] = 0;
    const uint32_t x = cell_of[i];
    const uint64_t r = rec[x];
    if (!rec_surv(r)) return;
    const uint32_t rk = rank[i];
    if (rk == kRankRemoved) return;
    scatter_point(pts, n, d, value_bits, i, rec_start(r) + rk, keys, fkeys, sidx);
}

hipError_t launch_scatter(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                          const Workspace &ws, int value_bits, hipStream_t st)
{
    if (dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_scatter<float>, grid_for(n), dim3(kThreads), 0, st, (const float *)pts,
                           (uint32_t)n, gd.d, value_bits, ws.cell_of, ws.rank, ws.rec, ws.keys, ws.fkeys,
                           ws.sidx, ws.flag);
    else
        hipLaunchKernelGGL(k_scatter<uint16_t>, grid_for(n), dim3(kThreads), 0, st,
                           (const uint16_t *)pts, (uint32_t)n, gd.d, value_bits, ws.cell_of, ws.rank,
                           ws.rec, ws.keys, ws.fkeys, ws.sidx, ws.flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan partials
__global__ __launch_bounds__(kPartialThreads) void k_scan_partials(uint64_t *block_sums, uint32_t nb)
{
    __shared__ uint64_t s_w[kPartialThreads / kWave];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kPartialThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? block_sums[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t, kPartialThreads>(v, &tot, s_w);
        if (i < nb) block_sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) block_sums[nb] = carry;
}

}  // namespace skycell
