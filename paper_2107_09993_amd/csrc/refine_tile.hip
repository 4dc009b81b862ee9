// K5, tile form of the exact refine: a coarse cone walk shared by a workgroup,
// with the candidates of each visited coarse cell staged in LDS and every query
// point screening only those in its own (fine) lower cone.
//
// Two layers of the grid (Section III: layer i+1 splits every cell of layer i
// in two along each dimension).  The fine layer is the call's grid of g = 2^r
// columns; the coarse layer drops the lowest bit of every column, so a coarse
// cell Y holds the 2^d fine cells (Y << d) | t, t in [0, 2^d): bit k of t is
// the lowest bit of the fine column k.  In Morton order the surviving points
// of Y are one contiguous run of the sorted arrays, grouped by t.
//
// A work unit is up to 256 query points of one coarse cell Y (one per thread).
// The workgroup walks the coarse lower cone of Y in odometer order, exactly as
// the lane form walks the fine one (the coarse lower closure of a cell is the
// fine one of its top corner, so empty sub-cones are never entered).  At each
// visited coarse cell C <= Y, let E be the dimensions where C and Y have the
// same coarse column.  A candidate in fine cell (C << d) | t can dominate a
// query in fine cell (Y << d) | s only if t_k <= s_k for k in E (elsewhere the
// coarse column is already smaller), i.e. only if t and F = E & ~s share no
// bit.  The allowed sub-cells are the submasks of ~F: one 64-bit pattern per
// word of the 2^d-bit occupancy of C, ANDed with it.  Each query therefore
// screens exactly the candidates of its fine lower cone (those of the lane
// form), while the walk, the cell starts and the candidates' screening words
// are loaded once per workgroup (coalesced) instead of once per query.
#include <algorithm>
#include <cstdlib>

#include "cellops.h"
#include "common.h"
#include "scan.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kTileThreads = 256;
constexpr int kTileStage = 2048;  // candidates whose screening words fit in LDS
constexpr uint64_t kTHigh = 0x8080808080808080ull;
constexpr uint64_t kTOnes = 0x0101010101010101ull;

// Sub-cells t of one 64-wide word (t in [0, 64)) with t & f = 0, f < 64.
__device__ __forceinline__ uint64_t submask_word(uint32_t f)
{
    uint64_t bad = 0ull;
    bad |= (f & 1u) ? 0xAAAAAAAAAAAAAAAAull : 0ull;
    bad |= (f & 2u) ? 0xCCCCCCCCCCCCCCCCull : 0ull;
    bad |= (f & 4u) ? 0xF0F0F0F0F0F0F0F0ull : 0ull;
    bad |= (f & 8u) ? 0xFF00FF00FF00FF00ull : 0ull;
    bad |= (f & 16u) ? 0xFFFF0000FFFF0000ull : 0ull;
    bad |= (f & 32u) ? 0xFFFFFFFF00000000ull : 0ull;
    return ~bad;
}

// Per coarse cell Y: the run [start, end) of its surviving points in sorted
// order, and its coarse lower-neighbour mask (bit k: coarse column k >= 1 and
// the cone below Y - e_k holds a non-empty cell), from the fine records and
// lower closure.
template <int D>
__global__ __launch_bounds__(256) void k_tile_coarse(GridDesc gd, const uint64_t *__restrict__ rec,
                                                     const uint64_t *__restrict__ lc, uint32_t ccells,
                                                     uint2 *__restrict__ crun, uint32_t *__restrict__ cnbr)
{
    const uint32_t y = blockIdx.x * 256 + threadIdx.x;
    if (y >= ccells) return;
    constexpr uint32_t kSub = (1u << D) - 1u;
    const uint32_t start = rec_start(rec[(size_t)y << D]);
    const uint32_t end = rec_start(rec[(size_t)(y + 1) << D]);
    uint32_t nbr = 0u;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t cm = gd.mask[k] >> D;
        if (y & cm) {
            const uint32_t yk = morton_dec(y, cm);
            if (lc_bit(lc, (yk << D) | kSub)) nbr |= 1u << k;
        }
    }
    crun[y] = make_uint2(start, end);
    cnbr[y] = nbr;
}

// Work units: ceil(points / 256) per coarse cell, in Morton order.
struct UnitLoader {
    const uint2 *crun;
    __device__ uint32_t operator()(uint64_t y) const
    {
        const uint2 r = crun[y];
        return (r.y - r.x + kTileThreads - 1) / kTileThreads;
    }
};

struct UnitEmitter {
    uint2 *units;
    __device__ void operator()(uint64_t y, uint32_t prefix, uint32_t v) const
    {
        for (uint32_t i = 0; i < v; ++i) units[prefix + i] = make_uint2((uint32_t)y, i);
    }
};

__global__ void k_tile_units_total(const uint64_t *block_sums, uint32_t nb, uint32_t *ctr)
{
    ctr[kCtrItems] = (uint32_t)block_sums[nb];
    for (int s = 0; s < kNumXcd; ++s) ctr[kCtrHead + s] = 0u;
}

// Exact Definition 1 test: candidate keys e dominate query keys q.
template <int D>
__device__ __forceinline__ bool exact_dominates(const uint32_t *__restrict__ e, const uint32_t (&q)[D])
{
    uint32_t gt = 0u, ne = 0u;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t ek = e[k];
        gt |= max(ek, q[k]) ^ q[k];
        ne |= ek ^ q[k];
    }
    return gt == 0u && ne != 0u;
}

template <int D>
__global__ __launch_bounds__(kTileThreads) void k_refine_tile(const uint32_t *__restrict__ keys,
                                                              const uint64_t *__restrict__ fkeys,
                                                              const int32_t *__restrict__ sidx,
                                                              const uint64_t *__restrict__ rec,
                                                              const uint2 *__restrict__ crun,
                                                              const uint32_t *__restrict__ cnbr,
                                                              const uint2 *__restrict__ units,
                                                              uint32_t *__restrict__ ctr, uint8_t *__restrict__ flag,
                                                              GridDesc gd, uint64_t *__restrict__ stats)
{
    static_assert(D >= 1 && D <= 8, "tile form holds 2^d <= 256 sub-cells");
    constexpr int kSubs = 1 << D;
    constexpr int kWords = kSubs >= 64 ? kSubs / 64 : 1;
    constexpr uint64_t kPad = (D % 8 == 0) ? 0ull : (~0ull << (8 * (D % 8))) & 0x7F7F7F7F7F7F7F7Full;
    __shared__ uint32_t s_start[kSubs + 1];
    __shared__ uint64_t s_occ[kWords];
    __shared__ uint64_t s_fk[kTileStage];
    __shared__ uint32_t s_cmask[kMaxD], s_clow[kMaxD];
    __shared__ uint32_t s_unit;
    __shared__ int s_live;

    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= gd.mask[k] >> D;
        s_cmask[threadIdx.x] = threadIdx.x < (unsigned)D ? (gd.mask[threadIdx.x] >> D) : 0u;
        s_clow[threadIdx.x] = low;
    }
    const uint32_t n_units = ctr[kCtrItems];
    // the sub-cell bit of a fine column is bit (7 - r) of its 7-bit screening column
    const int sub_shift = 7 - gd.r;
    uint32_t visits = 0u, tests = 0u;
    int share = (int)(blockIdx.x % kNumXcd), shares_left = kNumXcd;

    for (;;) {
        // ---- next unit: the workgroup's XCD share first, then the others
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t u = 0xFFFFFFFFu;
            while (shares_left > 0) {
                const uint32_t s_lo = (uint32_t)(((uint64_t)n_units * share) / kNumXcd);
                const uint32_t s_hi = (uint32_t)(((uint64_t)n_units * (share + 1)) / kNumXcd);
                const uint32_t b = s_lo + atomicAdd(&ctr[kCtrHead + share], 1u);
                if (b < s_hi) {
                    u = b;
                    break;
                }
                share = share + 1 == kNumXcd ? 0 : share + 1;
                --shares_left;
            }
            s_unit = u;
        }
        __syncthreads();
        const uint32_t unit = s_unit;
        if (unit == 0xFFFFFFFFu) break;
        const uint2 uy = units[unit];
        const uint32_t root = uy.x;
        const uint2 rrun = crun[root];
        const uint32_t qi = rrun.x + uy.y * kTileThreads + threadIdx.x;
        bool alive = qi < rrun.y;

        // ---- query point of this thread: exact keys, screening word, sub-cell
        uint32_t q[D];
        uint64_t qf = kTHigh;
        uint32_t s = 0u;
        if (alive) {
#pragma unroll
            for (int k = 0; k < D; ++k) q[k] = keys[(size_t)qi * D + k];
            const uint64_t w = fkeys[qi];
#pragma unroll
            for (int k = 0; k < D; ++k) s |= (uint32_t)((w >> (8 * k + sub_shift)) & 1ull) << k;
            qf = w | kTHigh | kPad;
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) q[k] = 0u;
        }

        // ---- coarse cone walk (the same values in every thread)
        uint32_t x = root;
        uint32_t diag = cnbr[root];
        bool first = true;
        for (;;) {
            uint32_t c;
            if (first) {
                c = root;
                first = false;
            } else {
                if (diag == 0u) break;
                const int j = __ffs(diag) - 1;
                c = morton_dec((x & ~s_clow[j]) | (root & s_clow[j]), s_cmask[j]);
                const uint32_t lowm = (2u << j) - 1u;
                diag = (diag & ~lowm) | (cnbr[c] & lowm);
                x = c;
            }
            const uint2 run = crun[c];
            if (run.y == run.x) continue;
            ++visits;
            // dimensions where c and the root share their coarse column
            uint32_t E = 0u;
#pragma unroll
            for (int k = 0; k < D; ++k) E |= ((c ^ root) & s_cmask[k]) == 0u ? (1u << k) : 0u;
            // stage the cell starts of c and, when they fit, the screening words
            __syncthreads();
            for (int t = threadIdx.x; t <= kSubs; t += kTileThreads)
                s_start[t] = rec_start(rec[((size_t)c << D) + t]);
            const uint32_t len = run.y - run.x;
            const bool staged = len <= (uint32_t)kTileStage;
            if (staged)
                for (uint32_t e = threadIdx.x; e < len; e += kTileThreads) s_fk[e] = fkeys[run.x + e];
            __syncthreads();
            for (int t = threadIdx.x; t < kSubs; t += kTileThreads) {
                const bool occ = s_start[t + 1] > s_start[t];
                const uint64_t b = __ballot(occ);
                if (kSubs >= 64) {
                    if (__lane_id() == 0) s_occ[t >> 6] = b;
                } else if (threadIdx.x == 0) {
                    s_occ[0] = b & ((kSubs == 64) ? ~0ull : ((1ull << kSubs) - 1ull));
                }
            }
            __syncthreads();
            if (alive) {
                const uint32_t F = E & ~s;
#pragma unroll
                for (int wj = 0; wj < kWords; ++wj) {
                    if (!alive) break;
                    if (((uint32_t)wj & (F >> 6)) != 0u) continue;
                    uint64_t wbits = submask_word(F & 63u) & s_occ[wj];
                    while (wbits != 0ull && alive) {
                        const uint32_t t = (uint32_t)wj * 64u + (uint32_t)__ffsll((long long)wbits) - 1u;
                        wbits &= wbits - 1ull;
                        const uint32_t cb = s_start[t], ce = s_start[t + 1];
                        for (uint32_t ci = cb; ci < ce; ++ci) {
                            const uint64_t f = staged ? s_fk[ci - run.x] : fkeys[ci];
                            ++tests;
                            const uint64_t diff = qf - f;
                            const uint64_t nle = ~diff & kTHigh;
                            const uint64_t nlt = ~(diff - kTOnes) & kTHigh;
                            if (nlt == 0ull) {  // smaller in every screening column
                                alive = false;
                                break;
                            }
                            if (nle == 0ull && exact_dominates<D>(keys + (size_t)ci * D, q)) {
                                alive = false;
                                break;
                            }
                        }
                    }
                }
            }
            // stop the walk once every query of the unit is dominated
            if (threadIdx.x == 0) s_live = 0;
            __syncthreads();
            if (alive) s_live = 1;
            __syncthreads();
            if (s_live == 0) break;
        }
        if (alive) flag[sidx[qi]] = 1;
    }

    if (stats != nullptr) {
        uint64_t v64 = __lane_id() == 0 ? visits : 0u, t64 = tests;
        for (int off = 32; off > 0; off >>= 1) {
            v64 += __shfl_xor(v64, off);
            t64 += __shfl_xor(t64, off);
        }
        if (__lane_id() == 0) {
            if (threadIdx.x == 0)
                atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)v64);
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)t64);
        }
    }
}

static int tile_blocks_per_cu_cached[kMaxD + 1];

template <int D>
static int tile_blocks_per_cu()
{
    int &b = tile_blocks_per_cu_cached[D];
    if (b <= 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_refine_tile<D>, kTileThreads, 0) != hipSuccess || v < 1)
            v = 1;
        const char *e = getenv("SKYCELL_TILE_BLOCKS");
        const int cap = e ? atoi(e) : 0;
        if (cap >= 1 && cap < v) v = cap;
        b = v;
    }
    return b;
}

template <int D>
static hipError_t launch_tile_d(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                                hipStream_t st)
{
    const uint32_t ccells = gd.cells >> D;
    // coarse runs and masks in the histogram's memory (not read after the scatter)
    uint2 *crun = reinterpret_cast<uint2 *>(ws.cnt);
    uint32_t *cnbr = reinterpret_cast<uint32_t *>(crun + ccells + 1);
    hipLaunchKernelGGL(k_tile_coarse<D>, dim3((ccells + 255) / 256), dim3(256), 0, st, gd, (const uint64_t *)ws.rec,
                       (const uint64_t *)ws.lc, ccells, crun, cnbr);
    UnitLoader ld{crun};
    UnitEmitter em{ws.items};
    hipError_t e = enqueue_scan<uint32_t>(ld, em, ccells, ws.block_sums, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_units_total, dim3(1), dim3(1), 0, st, (const uint64_t *)ws.block_sums,
                       scan_tiles(ccells), ws.ctr);
    // units <= min(coarse cells, points): no more workgroups than that
    const uint64_t full = (uint64_t)num_cus * (uint64_t)tile_blocks_per_cu<D>();
    const uint64_t bound = std::min<uint64_t>((uint64_t)ccells, (uint64_t)(n > 0 ? n : 1));
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(full, bound));
    hipLaunchKernelGGL(k_refine_tile<D>, dim3(blocks), dim3(kTileThreads), 0, st, (const uint32_t *)ws.keys,
                       (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx, (const uint64_t *)ws.rec,
                       (const uint2 *)crun, (const uint32_t *)cnbr, (const uint2 *)ws.items, ws.ctr, ws.flag, gd,
                       stats);
    return hipGetLastError();
}

// d >= 2 keeps the coarse runs and masks (12 bytes per coarse cell) inside the
// histogram's 4 bytes per fine cell; g <= 128 keeps the sub-cell bit inside the
// 7-bit screening column.
bool tile_form_supported(int d, int g) { return d >= 2 && d <= 8 && g >= 2 && g <= 128 && (g & (g - 1)) == 0; }

hipError_t launch_refine_tile(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                              hipStream_t st)
{
    if (!tile_form_supported(gd.d, gd.g)) return hipErrorInvalidValue;
    switch (gd.d) {
    case 2: return launch_tile_d<2>(n, gd, ws, stats, num_cus, st);
    case 3: return launch_tile_d<3>(n, gd, ws, stats, num_cus, st);
    case 4: return launch_tile_d<4>(n, gd, ws, stats, num_cus, st);
    case 5: return launch_tile_d<5>(n, gd, ws, stats, num_cus, st);
    case 6: return launch_tile_d<6>(n, gd, ws, stats, num_cus, st);
    case 7: return launch_tile_d<7>(n, gd, ws, stats, num_cus, st);
    case 8: return launch_tile_d<8>(n, gd, ws, stats, num_cus, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t refine_tile_prepare(const GridDesc &gd)
{
    switch (gd.d) {
    case 2: (void)tile_blocks_per_cu<2>(); break;
    case 3: (void)tile_blocks_per_cu<3>(); break;
    case 4: (void)tile_blocks_per_cu<4>(); break;
    case 5: (void)tile_blocks_per_cu<5>(); break;
    case 6: (void)tile_blocks_per_cu<6>(); break;
    case 7: (void)tile_blocks_per_cu<7>(); break;
    case 8: (void)tile_blocks_per_cu<8>(); break;
    default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

}  // namespace skycell
