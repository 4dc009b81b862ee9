// Two grid layers for grids beyond the dense cell budget (Section III: layer
// i+1 splits every cell of layer i in two along each dimension; Cor. 3 in the
// form used here: a non-empty cell of layer i+1 can survive only inside a
// surviving cell of layer i).
//
// The fine layer has g = 2^rho columns and may hold far more cells than a dense
// count table allows (d = 8, g = 16: 2^32 cells); it is kept as one occupancy
// bit per fine cell.  The base layer, g/2 columns, is the dense grid of the
// path: histogram, lower closure, cell records, scan, scatter and refine run on
// it.  Fine cell f = (C << d) | s (C its base cell, bit k of s the lowest bit of
// fine column k) is dominated (Definition 3 at the fine layer) iff a non-empty
// fine cell f' = (C' << d) | t has f' < f in every column, i.e. C' <= C and, in
// the dimensions E where C'_k = C_k, t_k = 0 and s_k = 1.  If C is dominated at
// the base layer every fine cell in it is; if C survives, every non-empty C' in
// its lower cone survives too.  So one lane per surviving base cell walks its
// base cone (the refine's odometer walk) and collects every E whose visited
// cell holds a fine cell t with t & E = 0; fine cell s of C is dominated iff
// one of those E is a subset of s (a superset closure over the 2^d subsets).
// Points of dominated fine cells are then removed before the counting sort, as
// pivot-dominated points are, and the refine on the base grid stays exact.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/skycell.h"
#include "cellops.h"
#include "common.h"
#include "host_internal.h"

namespace skycell {

constexpr int kFineThreads = 256;

static inline dim3 fine_grid(uint64_t count)
{
    const uint64_t b = (count + kFineThreads - 1) / kFineThreads;
    return dim3((unsigned)(b ? b : 1));
}

__global__ __launch_bounds__(kFineThreads) void k_fine_zero(uint32_t *__restrict__ p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kFineThreads + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * kFineThreads)
        p[i] = 0u;
}

// Fine occupancy bit of every point; its sub-cell s goes to rank[i] (the rank
// of the histogram is not used: the counts are taken again after the prune).
template <typename T>
__global__ __launch_bounds__(kFineThreads) void k_fine_occ(const T *__restrict__ pts, uint32_t n, int d, uint32_t gf,
                                                           int value_bits, const uint32_t *__restrict__ cell_of,
                                                           uint32_t *__restrict__ rank, uint32_t *__restrict__ occ)
{
    const uint32_t i = blockIdx.x * kFineThreads + threadIdx.x;
    if (i >= n) return;
    const float gff = (float)gf;
    bool nan = false;
    uint32_t s = 0u;
    for (int k = 0; k < d; ++k) {
        const T v = pts[(size_t)k * n + i];
        uint32_t c;
        if constexpr (sizeof(T) == 4)
            c = column_f32(v, gff, gf, nan);
        else
            c = column_u16(v, gf, value_bits);
        s |= (c & 1u) << k;
    }
    const uint64_t f = ((uint64_t)cell_of[i] << d) | s;
    rank[i] = s;
    atomicOr(&occ[f >> 5], 1u << (f & 31));
}

// The 2^D fine cells of base cell c: bits [c << D, (c + 1) << D) of a bitmap,
// as four 64-bit words (D <= 8; unused high bits zero).
template <int D>
__device__ __forceinline__ void fine_bits(const uint32_t *__restrict__ bm, uint32_t c, uint64_t (&w)[4])
{
    constexpr int kSubs = 1 << D;
    const uint64_t first = (uint64_t)c << D;
    if constexpr (kSubs >= 32) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint64_t v = 0ull;
            if (j * 64 < kSubs) {
                v = bm[(first >> 5) + 2 * j];
                if (j * 64 + 32 < kSubs) v |= (uint64_t)bm[(first >> 5) + 2 * j + 1] << 32;
            }
            w[j] = v;
        }
    } else {
        w[0] = (bm[first >> 5] >> (first & 31)) & ((1u << kSubs) - 1u);
        w[1] = w[2] = w[3] = 0ull;
    }
}

// Subsets t of [0, 256) with t & e = 0, as four words (bit t of word t >> 6).
__device__ __forceinline__ void submasks(uint32_t e, uint64_t (&w)[4])
{
    uint64_t bad = 0ull;
    bad |= (e & 1u) ? 0xAAAAAAAAAAAAAAAAull : 0ull;
    bad |= (e & 2u) ? 0xCCCCCCCCCCCCCCCCull : 0ull;
    bad |= (e & 4u) ? 0xF0F0F0F0F0F0F0F0ull : 0ull;
    bad |= (e & 8u) ? 0xFF00FF00FF00FF00ull : 0ull;
    bad |= (e & 16u) ? 0xFFFF0000FFFF0000ull : 0ull;
    bad |= (e & 32u) ? 0xFFFFFFFF00000000ull : 0ull;
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = ((uint32_t)j & (e >> 6)) ? 0ull : ~bad;
}

// Superset closure over the subsets of D dimensions: bit s set afterwards iff
// some set bit e of the input has e subset of s.
template <int D>
__device__ __forceinline__ void superset_closure(uint64_t (&u)[4])
{
    constexpr uint64_t kLow[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0F0F0F0F0F0F0F0Full,
                                  0x00FF00FF00FF00FFull, 0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
#pragma unroll
    for (int k = 0; k < D && k < 6; ++k) {
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] |= (u[j] & kLow[k]) << (1 << k);
    }
    if (D > 6) {  // bit 6: word j -> word j | 1
        u[1] |= u[0];
        u[3] |= u[2];
    }
    if (D > 7) {  // bit 7: word j -> word j | 2
        u[2] |= u[0];
        u[3] |= u[1];
    }
}

// One lane per base cell: for a surviving cell, the dominated fine cells, into
// `dom` (same layout as `occ`); counts of non-empty and surviving fine cells.
template <int D>
__global__ __launch_bounds__(kFineThreads) void k_fine_dom(GridDesc gd, const uint64_t *__restrict__ rec,
                                                           const uint32_t *__restrict__ occ,
                                                           uint32_t *__restrict__ dom, uint64_t *__restrict__ stats)
{
    constexpr int kSubs = 1 << D;
    constexpr uint32_t kAll = (1u << D) - 1u;
    __shared__ uint32_t s_mask[kMaxD], s_low[kMaxD];
    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= gd.mask[k];
        s_mask[threadIdx.x] = threadIdx.x < (unsigned)D ? gd.mask[threadIdx.x] : 0u;
        s_low[threadIdx.x] = low;
    }
    __syncthreads();
    const uint32_t c = blockIdx.x * kFineThreads + threadIdx.x;
    uint64_t ne_cells = 0ull, surv_cells = 0ull;
    if (c < gd.cells) {
        uint64_t own[4];
        fine_bits<D>(occ, c, own);
        const uint64_t r0 = rec[c];
        ne_cells = (uint64_t)(__popcll(own[0]) + __popcll(own[1]) + __popcll(own[2]) + __popcll(own[3]));
        if (rec_surv(r0)) {
            // collected sets E (bit e of the 2^D-bit set), starting with c itself
            uint64_t got[4] = {0ull, 0ull, 0ull, 0ull};
            uint32_t x = c, y = c;
            uint32_t diag = rec_nbr(r0) & kAll;
            for (;;) {
                uint64_t o[4], m[4];
                fine_bits<D>(occ, y, o);
                uint32_t e = 0u;
#pragma unroll
                for (int k = 0; k < D; ++k) e |= ((y ^ c) & s_mask[k]) == 0u ? (1u << k) : 0u;
                submasks(e, m);
                if ((o[0] & m[0]) | (o[1] & m[1]) | (o[2] & m[2]) | (o[3] & m[3])) {
                    const uint64_t bit = 1ull << (e & 63);
#pragma unroll
                    for (int wj = 0; wj < 4; ++wj) got[wj] |= (e >> 6) == (uint32_t)wj ? bit : 0ull;
                }
                if (diag == 0u) break;
                const int j = __ffs(diag) - 1;
                y = morton_dec((x & ~s_low[j]) | (c & s_low[j]), s_mask[j]);
                const uint32_t lowm = (2u << j) - 1u;
                diag = (diag & ~lowm) | (rec_nbr(rec[y]) & lowm);
                x = y;
            }
            superset_closure<D>(got);
            uint64_t dm[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) dm[j] = got[j] & own[j];
            surv_cells = ne_cells - (uint64_t)(__popcll(dm[0]) + __popcll(dm[1]) + __popcll(dm[2]) + __popcll(dm[3]));
            const uint64_t first = (uint64_t)c << D;
            if constexpr (kSubs >= 32) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j * 64 < kSubs) {
                        dom[(first >> 5) + 2 * j] = (uint32_t)dm[j];
                        if (j * 64 + 32 < kSubs) dom[(first >> 5) + 2 * j + 1] = (uint32_t)(dm[j] >> 32);
                    }
                }
            } else if (dm[0] != 0ull) {
                atomicOr(&dom[first >> 5], (uint32_t)dm[0] << (first & 31));
            }
        }
    }
    if (stats != nullptr) {
        for (int off = 32; off > 0; off >>= 1) {
            ne_cells += __shfl_xor(ne_cells, off);
            surv_cells += __shfl_xor(surv_cells, off);
        }
        if (__lane_id() == 0) {
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_NONEMPTY_CELLS], (unsigned long long)ne_cells);
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_SURVIVING_CELLS], (unsigned long long)surv_cells);
        }
    }
}

// Points of surviving base cells whose fine cell survives are counted again;
// the others are removed.
__global__ __launch_bounds__(kFineThreads) void k_fine_prune(uint32_t n, int d, const uint32_t *__restrict__ cell_of,
                                                             const uint64_t *__restrict__ rec,
                                                             const uint32_t *__restrict__ dom,
                                                             uint32_t *__restrict__ rank, uint32_t *__restrict__ cnt)
{
    const uint32_t i = blockIdx.x * kFineThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = cell_of[i];
    if (!rec_surv(rec[x])) return;
    const uint64_t f = ((uint64_t)x << d) | rank[i];
    const bool removed = (dom[f >> 5] >> (f & 31)) & 1u;
    rank[i] = removed ? kRankRemoved : atomicAdd(&cnt[x], 1u);
}

__global__ __launch_bounds__(kFineThreads) void k_fine_zero_cnt(uint32_t *__restrict__ cnt, uint32_t cells)
{
    for (uint32_t i = blockIdx.x * kFineThreads + threadIdx.x; i < cells; i += gridDim.x * kFineThreads) cnt[i] = 0u;
}

}  // namespace skycell

using namespace skycell;

// Bytes of the fine layer's two bitmaps (occupancy, dominated) for d and rho.
static size_t fine_bitmap_bytes(int d, int rho) { return ((size_t)1 << (rho * d - 3)) + 256; }

int skycell_compute_layered(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t rho, int32_t value_bits,
                            int32_t *out_idx, int32_t *out_count, uint64_t *stats, void *stream)
{
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    if (d < 2 || d > 8) return set_error(SKYCELL_E_INVAL, "d = %d is outside [2, 8]", d);
    if (rho < 2 || (rho - 1) * d > 26 || rho * d > 32)
        return set_error(SKYCELL_E_RANGE, "rho = %d: need rho >= 2, (rho - 1) * d <= 26 and rho * d <= 32", rho);
    int rc = validate(points, dtype, n, d, 1 << (rho - 1), value_bits, out_idx, out_count);
    if (rc != SKYCELL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        SKYCELL_HIP_CHECK(launch_write_zero_count(out_count, st));
        return clear_error();
    }
    const int gb = 1 << (rho - 1);
    const GridDesc gd = pipeline_desc(n, d, gb, dtype);
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    const int cus = device_cus(dev);
    const size_t need = workspace_layout(n, d, gd.cells, nullptr, nullptr);
    const size_t bbytes = fine_bitmap_bytes(d, rho);
    void *wptr = nullptr, *fptr = nullptr;
    if ((rc = cached_buffer(kCacheWorkspace, dev, st, need, &wptr)) != SKYCELL_OK) return rc;
    if ((rc = cached_buffer(kCacheFine, dev, st, 2 * bbytes, &fptr)) != SKYCELL_OK) return rc;
    Workspace ws;
    workspace_layout(n, d, gd.cells, &ws, (char *)wptr);
    uint32_t *occ = (uint32_t *)fptr;
    uint32_t *dom = (uint32_t *)((char *)fptr + bbytes);
    const uint64_t words = ((uint64_t)1 << (rho * d)) / 32 + 1;
    SKYCELL_HIP_CHECK(launch_init(ws, gd, stats, st));
    SKYCELL_HIP_CHECK(launch_quantize_hist(points, dtype, n, gd, value_bits, ws, st));
    const unsigned zb = (unsigned)std::min<uint64_t>(16384, (words + kFineThreads - 1) / kFineThreads);
    hipLaunchKernelGGL(k_fine_zero, dim3(zb ? zb : 1), dim3(kFineThreads), 0, st, occ, words);
    hipLaunchKernelGGL(k_fine_zero, dim3(zb ? zb : 1), dim3(kFineThreads), 0, st, dom, words);
    if (dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_fine_occ<float>, fine_grid(n), dim3(kFineThreads), 0, st, (const float *)points,
                           (uint32_t)n, d, (uint32_t)(1u << rho), value_bits, (const uint32_t *)ws.cell_of, ws.rank, occ);
    else
        hipLaunchKernelGGL(k_fine_occ<uint16_t>, fine_grid(n), dim3(kFineThreads), 0, st, (const uint16_t *)points,
                           (uint32_t)n, d, (uint32_t)(1u << rho), value_bits, (const uint32_t *)ws.cell_of, ws.rank,
                           occ);
    SKYCELL_HIP_CHECK(hipGetLastError());
    SKYCELL_HIP_CHECK(launch_cell_prune(gd, ws, n, nullptr, st));
    switch (d) {
#define SKYCELL_FINE_CASE(DD)                                                                                    \
    case DD:                                                                                                     \
        hipLaunchKernelGGL(k_fine_dom<DD>, fine_grid(gd.cells), dim3(kFineThreads), 0, st, gd,                   \
                           (const uint64_t *)ws.rec, (const uint32_t *)occ, dom, stats);                          \
        break;
        SKYCELL_FINE_CASE(2)
        SKYCELL_FINE_CASE(3)
        SKYCELL_FINE_CASE(4)
        SKYCELL_FINE_CASE(5)
        SKYCELL_FINE_CASE(6)
        SKYCELL_FINE_CASE(7)
        SKYCELL_FINE_CASE(8)
#undef SKYCELL_FINE_CASE
    default:
        return set_error(SKYCELL_E_INVAL, "d = %d", d);
    }
    SKYCELL_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_fine_zero_cnt, dim3(std::min<unsigned>(4096u, (gd.cells + kFineThreads - 1) / kFineThreads)),
                       dim3(kFineThreads), 0, st, ws.cnt, gd.cells);
    hipLaunchKernelGGL(k_fine_prune, fine_grid(n), dim3(kFineThreads), 0, st, (uint32_t)n, d,
                       (const uint32_t *)ws.cell_of, (const uint64_t *)ws.rec, (const uint32_t *)dom, ws.rank, ws.cnt);
    SKYCELL_HIP_CHECK(hipGetLastError());
    SKYCELL_HIP_CHECK(launch_cell_scan(gd, ws, n, stats, st, true));
    SKYCELL_HIP_CHECK(launch_scatter(points, dtype, n, gd, ws, value_bits, cus, st));
    SKYCELL_HIP_CHECK(launch_refine(n, gd, ws, stats, cus, st));
    SKYCELL_HIP_CHECK(launch_output(n, ws, out_idx, out_count, stats, st));
    return clear_error();
}
