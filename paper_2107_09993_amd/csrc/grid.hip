// Grid phase of the skyline path (SkyCell paper, Section III grid structure and
// Section V, Algorithm 1, whose first step sorts the points by cell):
//   K1  quantise every point to its cell (Equation 1), build the occupancy
//       histogram and keep each point's rank inside its cell;
//   K3  lower closure of the occupancy by d prefix-OR passes, then per cell the
//       "dominated" test of Definition 3 and the lower-neighbour mask used by the
//       refine's cone walk;
//   K2  exclusive scan of surviving-cell counts: counting-sort offsets and refine
//       work items;
//   K4  scatter of surviving points, grouped by cell, as order-preserving keys
//       (one pass below 2^20 points; above, staged by ranges of cells first so
//       that the final writes complete whole cache lines), followed for d <= 8
//       by the walk records of the refine's lane form (refine.hip).
#include <cstdlib>

#include "cellops.h"
#include "common.h"
#include "scan.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kThreads = 256;
// Workgroups per CU of the second scatter pass (SKYCELL_SCATTER_ROW_BLOCKS
// overrides it): few enough that the rows in flight on one XCD target a window
// of destination lines that fits in its L2.
static int scatter_row_blocks()
{
    static int b = -1;
    if (b < 0) {
        const char *v = getenv("SKYCELL_SCATTER_ROW_BLOCKS");
        const int e = v ? atoi(v) : 0;
        b = (e >= 1 && e <= 16) ? e : 1;
    }
    return b;
}

// SKYCELL_SCATTER2=0 keeps the one-pass scatter for every size (comparisons).
static bool scatter_two_pass_enabled()
{
    static int on = -1;
    if (on < 0) {
        const char *v = getenv("SKYCELL_SCATTER2");
        on = (v && v[0] == '0') ? 0 : 1;
    }
    return on != 0;
}

static inline dim3 grid_for(uint64_t count, int per_block = kThreads)
{
    uint64_t b = (count + per_block - 1) / per_block;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(kThreads) void k_init(uint32_t *cnt, uint32_t cells, uint32_t *ctr,
                                                   uint64_t *stats, int32_t g, uint32_t *split_hist)
{
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t i = gid; i < cells; i += stride) cnt[i] = 0u;
    if (split_hist != nullptr)
        for (uint32_t i = gid; i <= (uint32_t)kSplitBins; i += stride) split_hist[i] = 0u;
    if (gid < kCtrCount) ctr[gid] = gid == kCtrSplitThr ? 0x7F800000u : 0u;  // threshold +inf: no cell split
    if (stats != nullptr && gid < SKYCELL_NUM_STATS)
        stats[gid] = gid == SKYCELL_STAT_GRID_RES ? (uint64_t)g : 0ull;
}

__global__ __launch_bounds__(kThreads) void k_zero_words(uint32_t *__restrict__ p, uint32_t count)
{
    for (uint32_t t = blockIdx.x * kThreads + threadIdx.x; t < count; t += gridDim.x * kThreads) p[t] = 0u;
}

hipError_t launch_init(const Workspace &ws, const GridDesc &gd, uint64_t *stats, hipStream_t st)
{
    uint32_t blocks = (gd.cells + kThreads * 8 - 1) / (kThreads * 8);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(kThreads), 0, st, ws.cnt, gd.cells, ws.ctr, stats, gd.g,
                       gd.split ? ws.bcur : nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K1
// Each thread quantises kQuantPer points (strided by the workgroup size, so
// every load is coalesced) and takes each point's rank inside its cell from
// the cell's counter.  Ranks only need to be distinct and below the cell's
// count (the scatter puts a point at the cell's first position plus its rank),
// so points that share a cell can take them together:
//   * lanes of one wave whose points share a cell (common when a few cells
//     hold most points, as on correlated data, where one counter per hot cell
//     would otherwise take every point's atomic in turn) rank among
//     themselves in lane order, and their leader adds their number at once.
//     A round whose lowest pending lane holds its cell alone leaves that lane
//     to its own atomic on the global counter; after kQuantSkips such rounds
//     in a row every lane still pending takes its own atomic, so wholly
//     distinct cells (the anti-correlated headline) pay a few ballot rounds,
//     while a wave that mixes a few hot cells with single ones keeps grouping
//     the hot ones (C2-correlated: 0.485 -> 0.449 ms);
//   * the leaders add into a small table of the workgroup's shared cells in
//     LDS instead of the global counter, and after the workgroup's last point
//     one atomic per table entry reserves the entry's ranks in the global
//     counter.  A cell that finds no free entry in two probes goes to the
//     global counter directly.
constexpr int kQuantPer = 8;
constexpr int kQuantSkips = 6;
constexpr int kHotSlots = 128;
constexpr uint32_t kNoSlot = 0xFFu;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_quantize_hist(const T *__restrict__ pts, uint32_t n,
                                                            GridDesc gd, int value_bits,
                                                            uint32_t *__restrict__ cell_of,
                                                            uint32_t *__restrict__ rank,
                                                            uint32_t *__restrict__ cnt,
                                                            uint32_t *__restrict__ ctr)
{
    __shared__ uint32_t s_key[kHotSlots], s_cnt[kHotSlots], s_base[kHotSlots];
    for (int e = threadIdx.x; e < kHotSlots; e += kThreads) {
        s_key[e] = kEmptyKey;
        s_cnt[e] = 0u;
    }
    __syncthreads();
    const uint32_t lane = __lane_id();
    const uint32_t first = blockIdx.x * (uint32_t)(kThreads * kQuantPer) + threadIdx.x;
    uint32_t rk[kQuantPer], sl[kQuantPer];
    bool nan = false;
#pragma unroll
    for (int p = 0; p < kQuantPer; ++p) {
        const uint32_t i = first + (uint32_t)(p * kThreads);
        const bool live = i < n;
        uint32_t cell = 0u;
        if (live) {
            cell = point_cell<T, D>(pts, n, i, gd, value_bits, nan);
            cell_of[i] = cell;
        }
        uint64_t pend = __ballot(live);
        bool got = false;
        uint32_t r = 0u, slot = kNoSlot;
        int skips = 0;
        while (pend != 0ull && skips < kQuantSkips) {
            const int lead = __builtin_ctzll(pend);
            const uint32_t lc = __builtin_amdgcn_readlane(cell, lead);
            const uint64_t same = __ballot(live && !got && cell == lc);
            const uint32_t k = (uint32_t)__builtin_popcountll(same);
            pend &= ~same;
            if (k < 2u) {
                ++skips;
                continue;
            }
            skips = 0;
            uint32_t base = 0u, ls = kNoSlot;
            if (lane == (uint32_t)lead) {
                uint32_t h = (lc * 0x9E3779B1u) >> 25;  // 7 bits: kHotSlots entries
                for (int probe = 0; probe < 2 && ls == kNoSlot; ++probe) {
                    const uint32_t old = atomicCAS(&s_key[h], kEmptyKey, lc);
                    if (old == kEmptyKey || old == lc) ls = h;
                    h = (h + 1u) & (kHotSlots - 1);
                }
                base = ls != kNoSlot ? atomicAdd(&s_cnt[ls], k) : atomicAdd(&cnt[lc], k);
            }
            base = __builtin_amdgcn_readlane(base, lead);
            ls = __builtin_amdgcn_readlane(ls, lead);
            if ((same >> lane) & 1ull) {
                r = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
                slot = ls;
                got = true;
            }
        }
        if (live && !got) r = atomicAdd(&cnt[cell], 1u);
        if (live && slot == kNoSlot) rank[i] = r;
        rk[p] = r;
        sl[p] = slot;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kHotSlots; e += kThreads)
        if (s_key[e] != kEmptyKey) s_base[e] = atomicAdd(&cnt[s_key[e]], s_cnt[e]);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kQuantPer; ++p) {
        const uint32_t i = first + (uint32_t)(p * kThreads);
        if (i < n && sl[p] != kNoSlot) rank[i] = s_base[sl[p]] + rk[p];
    }
    if (nan) atomicOr(&ctr[kCtrErr], 1u);
}

template <typename T>
static hipError_t launch_quantize_hist_t(const T *pts, int64_t n, const GridDesc &gd, int value_bits,
                                         const Workspace &ws, hipStream_t st)
{
    const dim3 grid = grid_for(n, kThreads * kQuantPer);
    switch (gd.d) {
#define SKYCELL_QH_CASE(DD)                                                                                     \
    case DD:                                                                                                    \
        hipLaunchKernelGGL((k_quantize_hist<T, DD>), grid, dim3(kThreads), 0, st, pts, (uint32_t)n, gd, value_bits, \
                           ws.cell_of, ws.rank, ws.cnt, ws.ctr);                                                \
        break;
        SKYCELL_QH_CASE(1) SKYCELL_QH_CASE(2) SKYCELL_QH_CASE(3) SKYCELL_QH_CASE(4)
        SKYCELL_QH_CASE(5) SKYCELL_QH_CASE(6) SKYCELL_QH_CASE(7) SKYCELL_QH_CASE(8)
        SKYCELL_QH_CASE(9) SKYCELL_QH_CASE(10) SKYCELL_QH_CASE(11) SKYCELL_QH_CASE(12)
        SKYCELL_QH_CASE(13) SKYCELL_QH_CASE(14) SKYCELL_QH_CASE(15) SKYCELL_QH_CASE(16)
#undef SKYCELL_QH_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_quantize_hist(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                                int value_bits, const Workspace &ws, hipStream_t st)
{
    if (dtype == SKYCELL_DTYPE_F32) return launch_quantize_hist_t((const float *)pts, n, gd, value_bits, ws, st);
    return launch_quantize_hist_t((const uint16_t *)pts, n, gd, value_bits, ws, st);
}

// ------------------------------------------------------------------ K3
// Lower closure bitmap: bit x is 1 iff some non-empty cell y has y <= x in
// every dimension.  Built as the occupancy bits (one wave ballot per 64 cells)
// followed by an inclusive prefix-OR along each dimension, one column bit
// level at a time (lc_step_word): the steps inside a word all run in one
// pass; each step above runs as one pass over the 2 MB (2^24 cells) bitmap.
__global__ __launch_bounds__(kThreads) void k_lc_init(const uint32_t *__restrict__ cnt,
                                                      uint64_t *__restrict__ lcb, uint32_t cells)
{
    const uint32_t x = blockIdx.x * kThreads + threadIdx.x;
    const uint64_t b = __ballot(x < cells && cnt[x] != 0u);
    if (__lane_id() == 0 && x < cells) lcb[x >> 6] = b;
}

// Every step whose index bit is inside a word (p < 6), for every dimension in
// order of its column bits.
__global__ __launch_bounds__(kThreads) void k_lc_inword(uint64_t *__restrict__ lcb, uint32_t words, GridDesc gd)
{
    const uint32_t wi = blockIdx.x * kThreads + threadIdx.x;
    if (wi >= words) return;
    uint64_t w = lcb[wi];
    for (int k = 0; k < gd.d; ++k) {
        uint32_t lowk = 0u;
        for (int b = 0; b < gd.r; ++b) {
            const int p = b * gd.d + k;
            if (p >= 6) break;
            w = lc_step_word(w, 0ull, p, lowk);
            lowk |= 1u << p;
        }
    }
    lcb[wi] = w;
}

// One step with index bit p >= 6: word W with bit p - 6 set ORs in word
// (W without that bit) | (lowk >> 6), spread over the low index bits of lowk.
__global__ __launch_bounds__(kThreads) void k_lc_step(uint64_t *__restrict__ lcb, uint32_t words, int p, uint32_t lowk)
{
    const uint32_t wi = blockIdx.x * kThreads + threadIdx.x;
    if (wi >= words || ((wi >> (p - 6)) & 1u) == 0u) return;
    const uint32_t si = (wi & ~(1u << (p - 6))) | (lowk >> 6);
    lcb[wi] = lc_step_word(lcb[wi], lcb[si], p, lowk);
}

// Per cell: the high half of the cell record (see cellops.h); the scan fills
// in the low half (first sorted position).  Grid-stride over the cells, so that
// with statistics on, each workgroup adds its totals with one atomic per
// counter at the end (one atomic per wave on the same two words serialised).
// With `split` (lane form with split slabs): the slab count of every
// surviving cell whose cone-size estimate reaches the picked threshold goes
// into its record (rec_slabs), and the exact work items before the split and
// the items it adds are counted (cell_slabs checks that they fit in n).
constexpr uint32_t kCellRecBlocks = 2048;

template <int D>
__global__ __launch_bounds__(kThreads) void k_cell_rec(GridDesc gd, const uint32_t *__restrict__ cnt,
                                                       const uint64_t *__restrict__ lc,
                                                       uint64_t *__restrict__ rec,
                                                       uint64_t *__restrict__ survbits,
                                                       uint64_t *__restrict__ stats,
                                                       uint32_t *__restrict__ split, uint32_t per_item)
{
    float thr = __builtin_inff();
    if (split != nullptr) thr = __uint_as_float(split[kCtrSplitThr]);
    const uint32_t top = gd.mask[gd.d - 1];
    uint32_t nocc = 0u, nsurv = 0u;  // wave-uniform running totals
    uint64_t items_all = 0ull, extra = 0ull;  // per lane
    for (uint32_t base = blockIdx.x * kThreads; base < gd.cells; base += gridDim.x * kThreads) {
        const uint32_t x = base + threadIdx.x;
        bool occ = false, surv = false;
        uint64_t r = 0ull;
        if (x < gd.cells) r = cell_record<D>(gd, cnt, lc, x, occ, surv);
        if (split != nullptr && surv) {
            const uint32_t items = (cnt[x] + per_item - 1u) / per_item;
            items_all += items;
            const uint32_t c = cell_column(x, top);
            if (c >= 1u && cone_cells<D>(gd, x) >= thr) {
                r |= (uint64_t)(c + 1u) << 55;
                extra += (uint64_t)items * c;
            }
        }
        if (x < gd.cells) rec[x] = r;
        // one bitmap word per wave: the wave's 64 cells start at a multiple of 64
        const uint64_t bs = __ballot(surv);
        if (__lane_id() == 0 && x < gd.cells) survbits[x >> 6] = bs;
        nocc += (uint32_t)__popcll(__ballot(occ));
        nsurv += (uint32_t)__popcll(bs);
    }
    if (split != nullptr) {
        __shared__ uint64_t s_part[2][kThreads / kWave];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            items_all += __shfl_xor(items_all, off);
            extra += __shfl_xor(extra, off);
        }
        if (__lane_id() == 0) {
            s_part[0][threadIdx.x / kWave] = items_all;
            s_part[1][threadIdx.x / kWave] = extra;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t ti = 0ull, te = 0ull;
            for (int w = 0; w < kThreads / kWave; ++w) {
                ti += s_part[0][w];
                te += s_part[1][w];
            }
            // both totals are below n < 2^31 when the split fits; a sum that
            // passes 2^31 marks it as not fitting, for good
            if (ti != 0ull) atomicAdd(&split[kCtrSplitItems], (uint32_t)ti);
            if (te >= (1ull << 31)) {
                atomicOr(&split[kCtrSplitFail], 1u);
            } else if (te != 0ull) {
                const uint32_t old = atomicAdd(&split[kCtrSplitExtra], (uint32_t)te);
                if ((uint64_t)old + te >= (1ull << 31)) atomicOr(&split[kCtrSplitFail], 1u);
            }
        }
    }
    if (stats != nullptr) {
        __shared__ uint32_t s_occ[kThreads / kWave], s_surv[kThreads / kWave];
        if (__lane_id() == 0) {
            s_occ[threadIdx.x / kWave] = nocc;
            s_surv[threadIdx.x / kWave] = nsurv;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t o = 0ull, v = 0ull;
            for (int w = 0; w < kThreads / kWave; ++w) {
                o += s_occ[w];
                v += s_surv[w];
            }
            if (o) atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_NONEMPTY_CELLS], (unsigned long long)o);
            if (v) atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_SURVIVING_CELLS], (unsigned long long)v);
        }
    }
}

uint32_t split_share()
{
    static int share = -1;
    if (share < 0) {
        const char *v = getenv("SKYCELL_SPLIT_SHARE");
        share = v ? atoi(v) : 256;
        if (share < 0) share = 256;
    }
    return (uint32_t)share;
}

// The split's threshold from a sample of the occupied cells: runs of 256
// consecutive cells, one run in `stride` (kSplitSample on grids of more than
// 2^20 cells, else every run; odd, so that the sampled runs take every value
// of the column bits above the run's 8 index bits, not a fixed subset).
// hist[b] takes the work items (per_item points each) of the sampled cells
// with more than one slab whose cone-size bin is b, hist[kSplitBins] those of
// every sampled cell.  (Counting only the cells that survive Definition 3
// picked the same cells on the anti-correlated inputs and cost twice as much.)
constexpr uint32_t kSplitSample = 17;

__global__ __launch_bounds__(kThreads) void k_split_hist(GridDesc gd, const uint32_t *__restrict__ cnt,
                                                         uint32_t per_item, uint32_t stride,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_hist[kSplitBins + 1];
    for (int b = threadIdx.x; b <= kSplitBins; b += kThreads) s_hist[b] = 0u;
    __syncthreads();
    const uint32_t top = gd.mask[gd.d - 1];
    const uint32_t runs = (gd.cells + kThreads - 1u) / kThreads;
    for (uint32_t run = blockIdx.x * stride; run < runs; run += gridDim.x * stride) {
        const uint32_t x = run * kThreads + threadIdx.x;
        const uint32_t m = x < gd.cells ? cnt[x] : 0u;
        if (m != 0u) {
            const uint32_t items = (m + per_item - 1u) / per_item;
            atomicAdd(&s_hist[kSplitBins], items);
            if (cell_column(x, top) >= 1u) atomicAdd(&s_hist[cone_bin(cone_cells(gd, x))], items);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b <= kSplitBins; b += kThreads)
        if (s_hist[b] != 0u) atomicAdd(&hist[b], s_hist[b]);
}

// The highest bin B whose sampled items and above reach 1 / share
// of all items (share 0: as many as the item array's estimated room takes),
// and never more than that room over g - 1 (a split cell's items become at
// most g times as many); the threshold is the smallest cone-size estimate of
// bin B (cells at or above it are split, cellops.h).
__global__ __launch_bounds__(kThreads) void k_split_pick(const uint32_t *__restrict__ hist_g, uint32_t share,
                                                         uint32_t n, uint32_t g, uint32_t stride,
                                                         uint32_t *__restrict__ ctr)
{
    // the histogram and its sums over chunks of 64 bins into LDS first, so that
    // the walk down from the top bin takes few dependent reads
    constexpr int kChunk = 64, kChunks = kSplitBins / kChunk;
    __shared__ uint32_t hist[kSplitBins + 1];
    __shared__ uint64_t csum[kChunks];
    for (int b = threadIdx.x; b <= kSplitBins; b += kThreads) hist[b] = hist_g[b];
    __syncthreads();
    if (threadIdx.x < (unsigned)kChunks) {
        uint64_t t = 0ull;
        for (int b = 0; b < kChunk; ++b) t += hist[threadIdx.x * kChunk + b];
        csum[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const uint64_t total = (uint64_t)hist[kSplitBins] * stride;
    const uint64_t room = total < n ? ((uint64_t)n - total) / (g > 1u ? g - 1u : 1u) : 0ull;
    uint64_t target = share != 0u ? total / share : room;
    if (target > room) target = room;
    target /= stride;  // in sampled items
    // B: the highest bin whose sampled items and above reach the target (at
    // least 1: bin 0 is a cone of one cell); none if the target is 0
    uint32_t b = (uint32_t)kSplitBins;
    if (target != 0ull) {
        uint64_t acc = 0ull;
        int c = kChunks - 1;
        while (c > 0 && acc + csum[c] < target) acc += csum[c--];
        int i = c * kChunk + kChunk - 1;
        while (i > 1 && acc + hist[i] < target) acc += hist[i--];
        b = (uint32_t)i;
    }
    const float thr = b >= (uint32_t)kSplitBins ? __builtin_inff() : exp2f(((float)b - 0.5f) * 0.125f);
    ctr[kCtrSplitThr] = __float_as_uint(thr);
}

hipError_t launch_cell_prune(const GridDesc &gd, const Workspace &ws, int64_t n, uint64_t *stats, hipStream_t st)
{
    hipLaunchKernelGGL(k_lc_init, grid_for(gd.cells), dim3(kThreads), 0, st, ws.cnt, ws.lc, gd.cells);
    if (gd.g > 1) {
        const uint32_t words = (gd.cells + 63u) / 64u;
        hipLaunchKernelGGL(k_lc_inword, grid_for(words), dim3(kThreads), 0, st, ws.lc, words, gd);
        for (int k = 0; k < gd.d; ++k) {
            uint32_t lowk = 0u;
            for (int b = 0; b < gd.r; ++b) {
                const int p = b * gd.d + k;
                if (p >= 6)
                    hipLaunchKernelGGL(k_lc_step, grid_for(words), dim3(kThreads), 0, st, ws.lc, words, p, lowk);
                lowk |= 1u << p;
            }
        }
    }
    dim3 rgrid = grid_for(gd.cells);
    if (rgrid.x > kCellRecBlocks) rgrid.x = kCellRecBlocks;
    const bool split = gd.split != 0;
    if (split) {
        const uint32_t runs = (gd.cells + kThreads - 1u) / kThreads;
        const uint32_t stride = gd.cells > (1u << 20) ? kSplitSample : 1u;
        uint32_t hb = (runs + stride - 1u) / stride;
        if (hb > 512u) hb = 512u;
        hipLaunchKernelGGL(k_split_hist, dim3(hb), dim3(kThreads), 0, st, gd, (const uint32_t *)ws.cnt,
                           (uint32_t)gd.m, stride, ws.bcur);
        // gd.split 2: as many cells as the item array has room for (tests)
        hipLaunchKernelGGL(k_split_pick, dim3(1), dim3(kThreads), 0, st, (const uint32_t *)ws.bcur,
                           gd.split == 2 ? 0u : split_share(), (uint32_t)n, (uint32_t)gd.g, stride, ws.ctr);
    }
    switch (gd.d) {
#define SKYCELL_REC_CASE(DD)                                                                                   \
    case DD:                                                                                                   \
        hipLaunchKernelGGL(k_cell_rec<DD>, rgrid, dim3(kThreads), 0, st, gd, ws.cnt, ws.lc, ws.rec, ws.survbits, \
                           stats, split ? ws.ctr : nullptr, (uint32_t)gd.m);                                   \
        break;
        SKYCELL_REC_CASE(1) SKYCELL_REC_CASE(2) SKYCELL_REC_CASE(3) SKYCELL_REC_CASE(4)
        SKYCELL_REC_CASE(5) SKYCELL_REC_CASE(6) SKYCELL_REC_CASE(7) SKYCELL_REC_CASE(8)
        SKYCELL_REC_CASE(9) SKYCELL_REC_CASE(10) SKYCELL_REC_CASE(11) SKYCELL_REC_CASE(12)
        SKYCELL_REC_CASE(13) SKYCELL_REC_CASE(14) SKYCELL_REC_CASE(15) SKYCELL_REC_CASE(16)
#undef SKYCELL_REC_CASE
    default:
        return hipErrorInvalidValue;
    }
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

hipError_t launch_cell_scan(const GridDesc &gd, const Workspace &ws, int64_t n, uint64_t *stats, hipStream_t st,
                            bool recount)
{
    const uint32_t m = (uint32_t)gd.m;
    const uint32_t *split = gd.split ? ws.ctr : nullptr;
    CellLoader ld{ws.rec, ws.cnt, m, split, (uint32_t)n};
    CellEmitter em{(uint32_t *)ws.rec, ws.items, m, recount, split != nullptr, gd.mask[gd.d - 1], (uint32_t)n};
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
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_scatter(const T *__restrict__ pts, uint32_t n, int value_bits,
                                                      const uint32_t *__restrict__ cell_of,
                                                      const uint32_t *__restrict__ rank,
                                                      const uint64_t *__restrict__ rec,
                                                      uint32_t *__restrict__ keys,
                                                      uint64_t *__restrict__ fkeys,
                                                      int32_t *__restrict__ sidx,
                                                      uint8_t *__restrict__ flag, uint8_t live_flag)
{
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    flag[i] = 0;
    const uint32_t x = cell_of[i];
    const uint32_t rk = rank[i];  // loaded with the cell, not behind its record
    const uint64_t r = rec[x];
    if (!rec_surv(r) || rk == kRankRemoved) return;
    if (live_flag) flag[i] = live_flag;
    scatter_point<T, D>(pts, n, value_bits, i, rec_start(r) + rk, keys, fkeys, sidx);
}

// Output flag the scatter gives each surviving point: the lane form of the
// refine sets the flags of skyline points itself (start 0), the wave form
// clears the flags of dominated points (start 1), because several waves may
// share one point's cone there.
static inline uint8_t scatter_live_flag(const GridDesc &gd) { return gd.m == kWaveItemPoints ? 1 : 0; }

// Two-pass form (large n).  Workgroup w of the counting and staging passes
// carries the label w % 8, the XCD it runs on under round-robin dispatch.
// Inside each bucket's range of sorted positions the staged rows are grouped
// by label, so the runs that workgroups of one XCD append are adjacent and
// their lines are completed in that XCD's L2.
constexpr int kStagePts = 16;  // points per thread in the counting and staging passes

// The cell, rank and survival word of each of a thread's kStagePts points,
// loaded in three batches (indices, then survival words) so that the loads of
// all points are in flight together.  Points past n read as removed, cell 0.
__device__ __forceinline__ void load_stage_ids(uint32_t n, uint32_t i0, const uint32_t *__restrict__ cell_of,
                                               const uint32_t *__restrict__ rank,
                                               const uint64_t *__restrict__ survbits, uint32_t (&cell)[kStagePts],
                                               uint32_t (&rk)[kStagePts], uint64_t (&sw)[kStagePts])
{
#pragma unroll
    for (int j = 0; j < kStagePts; ++j) {
        const uint32_t i = i0 + (uint32_t)j * kThreads;
        cell[j] = i < n ? cell_of[i] : 0u;
        rk[j] = i < n ? rank[i] : kRankRemoved;
    }
#pragma unroll
    for (int j = 0; j < kStagePts; ++j) sw[j] = survbits[cell[j] >> 6];
}

__device__ __forceinline__ bool stage_live(uint32_t cell, uint32_t rk, uint64_t sw)
{
    return ((sw >> (cell & 63u)) & 1ull) != 0ull && rk != kRankRemoved;
}

// Pass 1a: per-workgroup bucket counts of the points that survive (their cell
// survives and the pivot pre-filter kept them), added into lab_cnt[bucket][label].
__global__ __launch_bounds__(kThreads) void k_scatter_count(uint32_t n, uint32_t nb, uint32_t sh,
                                                            const uint32_t *__restrict__ cell_of,
                                                            const uint32_t *__restrict__ rank,
                                                            const uint64_t *__restrict__ survbits,
                                                            uint32_t *__restrict__ lab_cnt)
{
    __shared__ uint32_t s_cnt[kMaxScatterBuckets];
    for (uint32_t t = threadIdx.x; t < nb; t += kThreads) s_cnt[t] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * (uint32_t)(kThreads * kStagePts) + threadIdx.x;
    uint32_t cell[kStagePts], rk[kStagePts];
    uint64_t sw[kStagePts];
    load_stage_ids(n, i0, cell_of, rank, survbits, cell, rk, sw);
#pragma unroll
    for (int j = 0; j < kStagePts; ++j)
        if (stage_live(cell[j], rk[j], sw[j])) atomicAdd(&s_cnt[cell[j] >> sh], 1u);
    __syncthreads();
    const uint32_t lab = blockIdx.x % kNumXcd;
    for (uint32_t t = threadIdx.x; t < nb; t += kThreads)
        if (s_cnt[t] != 0u) atomicAdd(&lab_cnt[t * kNumXcd + lab], s_cnt[t]);
}

// Pass 1b: exclusive scan of lab_cnt in (bucket, label) order, in place: the
// staging cursor of each (bucket, label).  One workgroup of kThreads threads.
__global__ __launch_bounds__(kThreads) void k_scatter_bases(uint32_t *__restrict__ lab_cnt, uint32_t count)
{
    __shared__ uint32_t s_part[kThreads];
    const uint32_t per = (count + kThreads - 1) / kThreads;
    const uint32_t lo = threadIdx.x * per;
    uint32_t sum = 0u;
    for (uint32_t k = lo; k < lo + per && k < count; ++k) sum += lab_cnt[k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0u;
        for (int t = 0; t < kThreads; ++t) {
            const uint32_t v = s_part[t];
            s_part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = s_part[threadIdx.x];
    for (uint32_t k = lo; k < lo + per && k < count; ++k) {
        const uint32_t v = lab_cnt[k];
        lab_cnt[k] = run;
        run += v;
    }
}

// Rows of the staging array: the raw coordinate words, the original index, the
// cell and the rank, padded to a multiple of four words (16-byte aligned rows).
__host__ __device__ constexpr uint32_t stage_row_words(int d) { return ((uint32_t)d + 3u + 3u) & ~3u; }

__device__ __forceinline__ uint32_t raw_word(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t raw_word(uint16_t v) { return (uint32_t)v; }

// Pass 1c: the same points per workgroup as pass 1a; the LDS atomic gives each
// point its slot in the workgroup's run of its bucket, one global atomic per
// (bucket, label) reserves the run.  Clears the output flag of every point.
// Rows are written kStageGroup points at a time, the coordinates of the group
// loaded before any of its rows is stored.
constexpr int kStageGroup = 4;

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_scatter_stage(const T *__restrict__ pts, uint32_t n,
                                                            uint32_t nb, uint32_t sh,
                                                            const uint32_t *__restrict__ cell_of,
                                                            const uint32_t *__restrict__ rank,
                                                            const uint64_t *__restrict__ survbits,
                                                            uint32_t *__restrict__ lab_cur,
                                                            uint32_t *__restrict__ stage,
                                                            uint8_t *__restrict__ flag, uint8_t live_flag)
{
    __shared__ uint32_t s_cnt[kMaxScatterBuckets];
    for (uint32_t t = threadIdx.x; t < nb; t += kThreads) s_cnt[t] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * (uint32_t)(kThreads * kStagePts) + threadIdx.x;
    uint32_t cell[kStagePts], rk[kStagePts], slot[kStagePts];
    {
        uint64_t sw[kStagePts];
        load_stage_ids(n, i0, cell_of, rank, survbits, cell, rk, sw);
#pragma unroll
        for (int j = 0; j < kStagePts; ++j) {
            const uint32_t i = i0 + (uint32_t)j * kThreads;
            const bool live = stage_live(cell[j], rk[j], sw[j]);
            if (i < n) flag[i] = live ? live_flag : (uint8_t)0;
            slot[j] = live ? atomicAdd(&s_cnt[cell[j] >> sh], 1u) : ~0u;
        }
    }
    __syncthreads();
    const uint32_t lab = blockIdx.x % kNumXcd;
    for (uint32_t t = threadIdx.x; t < nb; t += kThreads) {
        const uint32_t c = s_cnt[t];
        s_cnt[t] = c != 0u ? atomicAdd(&lab_cur[t * kNumXcd + lab], c) : 0u;
    }
    __syncthreads();
    constexpr uint32_t rw = stage_row_words(D);
#pragma unroll
    for (int g0 = 0; g0 < kStagePts; g0 += kStageGroup) {
        uint32_t c[kStageGroup][D];
#pragma unroll
        for (int t = 0; t < kStageGroup; ++t) {
            const int j = g0 + t;
            const uint32_t i = i0 + (uint32_t)j * kThreads;
#pragma unroll
            for (int k = 0; k < D; ++k) c[t][k] = slot[j] != ~0u ? raw_word(pts[(size_t)k * n + i]) : 0u;
        }
#pragma unroll
        for (int t = 0; t < kStageGroup; ++t) {
            const int j = g0 + t;
            if (slot[j] == ~0u) continue;
            const uint32_t i = i0 + (uint32_t)j * kThreads;
            uint4 *row = reinterpret_cast<uint4 *>(stage + (size_t)(s_cnt[cell[j] >> sh] + slot[j]) * rw);
            // words 0..D-1 coordinates, D index, D+1 cell, D+2 rank, then zero padding
#pragma unroll
            for (uint32_t q = 0; q < rw / 4u; ++q) {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = (int)(4u * q) + e;
                    w[e] = k < D ? c[t][k < D ? k : 0] : k == D ? i : k == D + 1 ? cell[j] : k == D + 2 ? rk[j] : 0u;
                }
                row[q] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
}

// Pass 2: the XCD with label x sweeps the x-th eighth of the staged rows in
// order, kThreads rows per workgroup and step, and writes each row to its
// sorted position start(cell) + rank.  Each thread loads its next row right
// after the current row's cell record, so that row's HBM latency overlaps the
// record load and the stores (one workgroup per CU keeps the rows in flight
// on an XCD inside about one bucket's window of sorted positions).
template <int RW>
__device__ __forceinline__ void load_stage_row(const uint32_t *__restrict__ stage, uint64_t r, uint32_t (&w)[RW])
{
    const uint4 *row = reinterpret_cast<const uint4 *>(stage + (size_t)r * RW);
#pragma unroll
    for (int q = 0; q < RW / 4; ++q) {
        const uint4 v = row[q];
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
    }
}

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_scatter_rows(int value_bits,
                                                           const uint32_t *__restrict__ stage,
                                                           const uint64_t *__restrict__ rec,
                                                           const uint32_t *__restrict__ ctr,
                                                           uint32_t *__restrict__ keys,
                                                           uint64_t *__restrict__ fkeys,
                                                           int32_t *__restrict__ sidx)
{
    const uint32_t total = ctr[kCtrSurvPts];
    const uint32_t xcd = blockIdx.x % kNumXcd;
    const uint32_t per = gridDim.x / kNumXcd;  // workgroups per XCD
    const uint32_t lo = (uint32_t)(((uint64_t)total * xcd) / kNumXcd);
    const uint32_t hi = (uint32_t)(((uint64_t)total * (xcd + 1)) / kNumXcd);
    constexpr int rw = (int)stage_row_words(D);
    constexpr int d = D;
    constexpr int fw = fine_words(D);
    const uint64_t step = (uint64_t)per * kThreads;
    uint64_t r = (uint64_t)lo + (uint64_t)(blockIdx.x / kNumXcd) * kThreads + threadIdx.x;
    if (r >= hi) return;
    uint32_t w[rw];
    load_stage_row<rw>(stage, r, w);
    for (;;) {
        const uint32_t i = w[d], x = w[d + 1], rk = w[d + 2];
        const uint64_t cr = rec[x];
        const uint64_t rn = r + step;
        const bool more = rn < hi;
        uint32_t wn[rw];
        load_stage_row<rw>(stage, more ? rn : r, wn);  // unconditional: no wait for it at a join
        const uint32_t pos = rec_start(cr) + rk;
        uint32_t *dst = keys + (size_t)pos * d;
        uint64_t *fdst = fkeys + (size_t)pos * fw;
        uint64_t word = 0ull;
        bool nan = false;
        uint32_t kw[D];
#pragma unroll
        for (int k = 0; k < d; ++k) {
            uint32_t f;
            if constexpr (sizeof(T) == 4) {
                const float v = __uint_as_float(w[k]);
                kw[k] = f32_key(v);
                f = column_f32(v, (float)kFineCols, (uint32_t)kFineCols, nan);
            } else {
                kw[k] = w[k];
                f = column_u16((uint16_t)w[k], (uint32_t)kFineCols, value_bits);
            }
            word |= (uint64_t)f << (8 * (k & 7));
            if ((k & 7) == 7 || k == d - 1) {
                fdst[k >> 3] = word;
                word = 0ull;
            }
        }
        store_key_row<D>(dst, kw);
        sidx[pos] = (int32_t)i;
        if (!more) break;
        r = rn;
#pragma unroll
        for (int q = 0; q < rw; ++q) w[q] = wn[q];
    }
}

static uint32_t scatter_buckets_for(int64_t n, uint32_t cells)
{
    static int env = -1;
    if (env < 0) {
        const char *v = getenv("SKYCELL_SCATTER_BUCKETS");
        env = v ? atoi(v) : 0;
    }
    uint32_t nb = scatter_buckets(n, cells);
    if (env >= 64 && env <= (int)kMaxScatterBuckets && (env & (env - 1)) == 0) nb = (uint32_t)env;
    return nb < cells ? nb : cells;
}

template <typename T>
static hipError_t launch_scatter_two_pass(const T *pts, int64_t n, const GridDesc &gd, const Workspace &ws,
                                          int value_bits, int num_cus, hipStream_t st)
{
    const uint32_t nb = scatter_buckets_for(n, gd.cells);
    uint32_t sh = 0u;
    while ((nb << sh) < gd.cells) ++sh;
    const uint32_t labs = nb * (uint32_t)kNumXcd;
    const dim3 pgrid = grid_for((uint64_t)n, kThreads * kStagePts);
    hipLaunchKernelGGL(k_zero_words, grid_for(labs), dim3(kThreads), 0, st, ws.bcur, labs);
    hipLaunchKernelGGL(k_scatter_count, pgrid, dim3(kThreads), 0, st, (uint32_t)n, nb, sh,
                       (const uint32_t *)ws.cell_of, (const uint32_t *)ws.rank, (const uint64_t *)ws.survbits,
                       ws.bcur);
    hipLaunchKernelGGL(k_scatter_bases, dim3(1), dim3(kThreads), 0, st, ws.bcur, labs);
    switch (gd.d) {
#define SKYCELL_STAGE_CASE(DD)                                                                                   \
    case DD:                                                                                                     \
        hipLaunchKernelGGL((k_scatter_stage<T, DD>), pgrid, dim3(kThreads), 0, st, pts, (uint32_t)n, nb, sh,     \
                           (const uint32_t *)ws.cell_of, (const uint32_t *)ws.rank,                               \
                           (const uint64_t *)ws.survbits, ws.bcur, ws.stage, ws.flag, scatter_live_flag(gd));     \
        break;
        SKYCELL_STAGE_CASE(1) SKYCELL_STAGE_CASE(2) SKYCELL_STAGE_CASE(3) SKYCELL_STAGE_CASE(4)
        SKYCELL_STAGE_CASE(5) SKYCELL_STAGE_CASE(6) SKYCELL_STAGE_CASE(7) SKYCELL_STAGE_CASE(8)
        SKYCELL_STAGE_CASE(9) SKYCELL_STAGE_CASE(10) SKYCELL_STAGE_CASE(11) SKYCELL_STAGE_CASE(12)
        SKYCELL_STAGE_CASE(13) SKYCELL_STAGE_CASE(14) SKYCELL_STAGE_CASE(15) SKYCELL_STAGE_CASE(16)
#undef SKYCELL_STAGE_CASE
    default:
        return hipErrorInvalidValue;
    }
    const unsigned blocks = (unsigned)(((num_cus * scatter_row_blocks() + kNumXcd - 1) / kNumXcd) * kNumXcd);
    switch (gd.d) {
#define SKYCELL_ROWS_CASE(DD)                                                                                    \
    case DD:                                                                                                     \
        hipLaunchKernelGGL((k_scatter_rows<T, DD>), dim3(blocks), dim3(kThreads), 0, st, value_bits,             \
                           (const uint32_t *)ws.stage, (const uint64_t *)ws.rec, (const uint32_t *)ws.ctr,        \
                           ws.keys, ws.fkeys, ws.sidx);                                                          \
        break;
        SKYCELL_ROWS_CASE(1) SKYCELL_ROWS_CASE(2) SKYCELL_ROWS_CASE(3) SKYCELL_ROWS_CASE(4)
        SKYCELL_ROWS_CASE(5) SKYCELL_ROWS_CASE(6) SKYCELL_ROWS_CASE(7) SKYCELL_ROWS_CASE(8)
        SKYCELL_ROWS_CASE(9) SKYCELL_ROWS_CASE(10) SKYCELL_ROWS_CASE(11) SKYCELL_ROWS_CASE(12)
        SKYCELL_ROWS_CASE(13) SKYCELL_ROWS_CASE(14) SKYCELL_ROWS_CASE(15) SKYCELL_ROWS_CASE(16)
#undef SKYCELL_ROWS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_scatter_one_pass(const T *pts, int64_t n, const GridDesc &gd, const Workspace &ws,
                                          int value_bits, hipStream_t st)
{
    switch (gd.d) {
#define SKYCELL_ONE_PASS_CASE(DD)                                                                                \
    case DD:                                                                                                     \
        hipLaunchKernelGGL((k_scatter<T, DD>), grid_for(n), dim3(kThreads), 0, st, pts, (uint32_t)n, value_bits, \
                           ws.cell_of, ws.rank, ws.rec, ws.keys, ws.fkeys, ws.sidx, ws.flag,                      \
                           scatter_live_flag(gd));                                                               \
        break;
        SKYCELL_ONE_PASS_CASE(1) SKYCELL_ONE_PASS_CASE(2) SKYCELL_ONE_PASS_CASE(3) SKYCELL_ONE_PASS_CASE(4)
        SKYCELL_ONE_PASS_CASE(5) SKYCELL_ONE_PASS_CASE(6) SKYCELL_ONE_PASS_CASE(7) SKYCELL_ONE_PASS_CASE(8)
        SKYCELL_ONE_PASS_CASE(9) SKYCELL_ONE_PASS_CASE(10) SKYCELL_ONE_PASS_CASE(11) SKYCELL_ONE_PASS_CASE(12)
        SKYCELL_ONE_PASS_CASE(13) SKYCELL_ONE_PASS_CASE(14) SKYCELL_ONE_PASS_CASE(15) SKYCELL_ONE_PASS_CASE(16)
#undef SKYCELL_ONE_PASS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_scatter_points(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                                        const Workspace &ws, int value_bits, int num_cus, hipStream_t st)
{
    if (ws.stage != nullptr && scatter_two_pass_enabled()) {
        if (dtype == SKYCELL_DTYPE_F32)
            return launch_scatter_two_pass<float>((const float *)pts, n, gd, ws, value_bits, num_cus, st);
        return launch_scatter_two_pass<uint16_t>((const uint16_t *)pts, n, gd, ws, value_bits, num_cus, st);
    }
    if (dtype == SKYCELL_DTYPE_F32)
        return launch_scatter_one_pass<float>((const float *)pts, n, gd, ws, value_bits, st);
    return launch_scatter_one_pass<uint16_t>((const uint16_t *)pts, n, gd, ws, value_bits, st);
}

hipError_t launch_scatter(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                          const Workspace &ws, int value_bits, int num_cus, hipStream_t st)
{
    const hipError_t e = launch_scatter_points(pts, dtype, n, gd, ws, value_bits, num_cus, st);
    if (e != hipSuccess) return e;
    return launch_walk_records(gd, ws, n, st);
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
