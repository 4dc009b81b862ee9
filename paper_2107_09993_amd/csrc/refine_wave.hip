// K5: exact refine with wave-uniform cone walks (SkyCell paper, Algorithm 1,
// RefineSkyline, with the cross-cell correction below).
//
// A point p can only be dominated by a point q whose cell is <= cell(p) in
// every dimension (the column map is non-decreasing).  The paper refines each
// candidate cell on its own, which misses dominators in other candidate cells
// that share a column with cell(p); here p is checked against every surviving
// point of every non-empty cell in the lower cone of cell(p).  All such cells
// survive the cell-domination prune, and pruned points are never needed as
// candidates: whatever dominates them dominates anything they dominate.
//
// Work unit: a chunk of at most 64 consecutive sorted points (one per lane)
// whose cells lie in one aligned Morton block of 2^b cells.  The wave walks,
// once and in lockstep, the lower cone of the chunk's corner (the largest
// column of its points in every dimension), which contains the cone of every
// point of the chunk.  At each non-empty surviving cell of that cone, the lanes
// whose own cone holds the cell (a packed per-dimension column compare) test
// its points; the cell's points are loaded one per lane and broadcast to the
// wave one at a time, so every test runs on all 64 lanes at once and a wave
// stops as soon as all its points are dominated.
//
// Cone walk.  With c the corner, the cells y <= c are c - delta, delta >= 0,
// visited in odometer order (delta[0] fastest).  From the current cell the
// next one lowers the smallest dimension j that still can be lowered, after
// putting dimensions below j back to c's columns: y = anchor_j - e_j with
// anchor_j = c - (0, .., 0, delta[j], delta[j+1], ..).  The lower closure is
// monotone, so once the cone below anchor_j - e_j is empty every larger
// delta[j] is empty too and the walk carries to j + 1.  Whether anchor_j - e_j
// is worth a visit is bit j of anchor_j's lower-neighbour mask; the walk keeps
// only those d bits, refreshed from the record of every visited cell, so it
// never probes an empty cone, never steps back up and holds O(1) state.
//
// Candidate test.  Each candidate is first screened with its packed 7-bit
// columns: q < p in every screening column proves q < p in every coordinate;
// q <= p in every column leaves the decision to an exact comparison of the
// order-preserving integer keys (Definition 1).
#include <cstdlib>

#include "cellops.h"
#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kWaveRefineThreads = 256;
constexpr int kChunkPoints = kWave;
constexpr uint64_t kFineHigh = 0x8080808080808080ull;
constexpr uint64_t kFineOnes = 0x0101010101010101ull;

// Packed cell columns, one field per dimension, for the "cell y <= cell c in
// every dimension" test: per field (c | top) - y keeps its top bit iff y <= c.
// Fields are wide enough for every column the index budget allows (r*d <= 26).
template <int D>
struct ColPack {
    static constexpr int kBits = D == 1 ? 32 : (D <= 3 ? 16 : 8);
    static constexpr int kPer = 64 / kBits;
    static constexpr int kWords = (D + kPer - 1) / kPer;
    static constexpr uint64_t kTop = kBits == 8 ? 0x8080808080808080ull
                                   : kBits == 16 ? 0x8000800080008000ull : 0x8000000080000000ull;
    static constexpr uint64_t kField = kBits == 32 ? 0xFFFFFFFFull : ((1ull << kBits) - 1ull);
    __host__ __device__ static constexpr int word(int k) { return k / kPer; }
    __host__ __device__ static constexpr int shift(int k) { return (k % kPer) * kBits; }
};

// Binary32 value of an order-preserving key (inverse of f32_key; -0.0 comes
// back as +0.0, which has the same column).
__device__ __forceinline__ float key_to_f32(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ __forceinline__ uint64_t lane64(uint64_t v, uint32_t l)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l) << 32) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
}

struct WaveFeeder {
    uint32_t *heads;   // kNumXcd queue heads
    uint32_t n_items;
    uint32_t chunk;
    int share;
    int shares_left;

    __device__ bool next(uint32_t &lo, uint32_t &hi)
    {
        while (shares_left > 0) {
            const uint32_t s_lo = (uint32_t)(((uint64_t)n_items * share) / kNumXcd);
            const uint32_t s_hi = (uint32_t)(((uint64_t)n_items * (share + 1)) / kNumXcd);
            uint32_t base = 0u;
            if (__lane_id() == 0) base = atomicAdd(&heads[share], chunk);
            base = uniform(__shfl(base, 0)) + s_lo;
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

struct WaveRefineArgs {
    const uint32_t *keys;
    const uint64_t *fkeys;
    const int32_t *sidx;
    const uint64_t *rec;
    const uint2 *items;
    uint32_t *ctr;
    uint8_t *flag;
    uint64_t *stats;
    GridDesc gd;
    uint32_t chunk;
    int32_t dtype;
    int32_t value_bits;
};

template <int D>
__global__ __launch_bounds__(kWaveRefineThreads) void k_refine_wave(WaveRefineArgs a)
{
    constexpr int FW = fine_words(D);
    constexpr uint32_t kAll = (1u << D) - 1u;
    using CP = ColPack<D>;
    constexpr int CW = CP::kWords;
    constexpr uint64_t kPad = (D % 8 == 0) ? 0ull : (~0ull << (8 * (D % 8))) & 0x7F7F7F7F7F7F7F7Full;

    __shared__ uint32_t s_mask[kMaxD], s_low[kMaxD];
    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= a.gd.mask[k];
        s_mask[threadIdx.x] = threadIdx.x < (unsigned)D ? a.gd.mask[threadIdx.x] : 0u;
        s_low[threadIdx.x] = low;
    }
    __syncthreads();

    const uint32_t lane = (uint32_t)__lane_id();
    const float gf = (float)a.gd.g;
    WaveFeeder feed{a.ctr + kCtrHead, a.ctr[kCtrItems], a.chunk, (int)(blockIdx.x % kNumXcd), kNumXcd};
    uint64_t visits = 0u, tests = 0u;

    uint32_t lo = 0u, hi = 0u;
    while (feed.next(lo, hi)) {
        for (uint32_t item = lo; item < hi; ++item) {
            const uint2 it = a.items[item];
            const uint32_t qstart = uniform(it.x), qcnt = uniform(it.y);
            const bool valid = lane < qcnt;
            const uint32_t qpos = qstart + lane;

            // ---- the lane's query point: exact keys, screening columns, cell columns
            uint32_t q[D];
            uint64_t qf[FW];
            uint64_t qc[CW];
            uint32_t col[D];
#pragma unroll
            for (int w = 0; w < FW; ++w) qf[w] = kFineHigh;
#pragma unroll
            for (int w = 0; w < CW; ++w) qc[w] = 0ull;
            if (valid) {
                const uint32_t *p = a.keys + (size_t)qpos * D;
#pragma unroll
                for (int k = 0; k < D; ++k) q[k] = p[k];
                const uint64_t *pf = a.fkeys + (size_t)qpos * FW;
#pragma unroll
                for (int w = 0; w < FW; ++w) qf[w] = pf[w] | kFineHigh;
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) q[k] = 0u;
            }
            qf[FW - 1] |= kPad;
            bool nan = false;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t c = 0u;
                if (valid)
                    c = a.dtype == SKYCELL_DTYPE_F32 ? column_f32(key_to_f32(q[k]), gf, (uint32_t)a.gd.g, nan)
                                                     : column_u16((uint16_t)q[k], (uint32_t)a.gd.g, a.value_bits);
                col[k] = c;
                qc[CP::word(k)] |= (uint64_t)c << CP::shift(k);
            }
#pragma unroll
            for (int k = D; k < CW * CP::kPer; ++k) qc[CP::word(k)] |= (CP::kField >> 1) << CP::shift(k);
#pragma unroll
            for (int w = 0; w < CW; ++w) qc[w] |= CP::kTop;

            // ---- corner: the largest column of the chunk in every dimension
            uint32_t root = 0u;
            uint64_t rootc[CW];
#pragma unroll
            for (int w = 0; w < CW; ++w) rootc[w] = 0ull;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t m = col[k];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor(m, off));
                m = uniform(m);
                root |= deposit_bits(m, s_mask[k]);
                rootc[CP::word(k)] |= (uint64_t)m << CP::shift(k);
            }

            // ---- walk the corner's lower cone
            bool alive = valid;
            uint32_t x = root;
            uint64_t yc[CW];
#pragma unroll
            for (int w = 0; w < CW; ++w) yc[w] = rootc[w];
            uint64_t r = uniform64(a.rec[x]);
            uint32_t diag = rec_nbr(r) & kAll;
            for (;;) {
                ++visits;
                if (rec_surv(r)) {
                    const uint32_t s = rec_start(r);
                    uint32_t c = rec_count(r);
                    if (c == kRecCountSat) c = uniform(rec_start(a.rec[x + 1])) - s;
                    // lanes whose query is alive and whose own cone holds this cell
                    bool in = alive;
#pragma unroll
                    for (int w = 0; w < CW; ++w) in = in && (((qc[w] - yc[w]) & CP::kTop) == CP::kTop);
                    for (uint32_t base = 0; base < c && __ballot(in) != 0ull; base += kChunkPoints) {
                        const uint32_t nt = c - base < (uint32_t)kChunkPoints ? c - base : (uint32_t)kChunkPoints;
                        uint64_t tf[FW];
#pragma unroll
                        for (int w = 0; w < FW; ++w) tf[w] = 0ull;
                        if (lane < nt) {
                            const uint64_t *pf = a.fkeys + (size_t)(s + base + lane) * FW;
#pragma unroll
                            for (int w = 0; w < FW; ++w) tf[w] = pf[w];
                        }
                        for (uint32_t t = 0; t < nt; ++t) {
                            const uint64_t act_mask = __ballot(in);
                            if (act_mask == 0ull) break;
                            const uint32_t cidx = s + base + t;
                            const bool act = in && cidx != qpos;
                            bool le = true, lt = true;
#pragma unroll
                            for (int w = 0; w < FW; ++w) {
                                const uint64_t diff = qf[w] - lane64(tf[w], t);
                                le = le && ((diff & kFineHigh) == kFineHigh);
                                lt = lt && (((diff - kFineOnes) & kFineHigh) == kFineHigh);
                            }
                            tests += (uint64_t)__popcll(__ballot(act));
                            if (act && lt) {
                                alive = false;
                                in = false;
                            }
                            const bool ex = act && le && !lt;
                            if (__ballot(ex) != 0ull) {
                                const uint32_t *pk = a.keys + (size_t)cidx * D;
                                uint32_t e[D];
#pragma unroll
                                for (int k = 0; k < D; ++k) e[k] = uniform(pk[k]);
                                if (ex) {
                                    bool all_le = true, ne = false;
#pragma unroll
                                    for (int k = 0; k < D; ++k) {
                                        all_le = all_le && e[k] <= q[k];
                                        ne = ne || e[k] != q[k];
                                    }
                                    if (all_le && ne) {
                                        alive = false;
                                        in = false;
                                    }
                                }
                            }
                        }
                    }
                }
                if (diag == 0u || __ballot(alive) == 0ull) break;
                const int j = __ffs(diag) - 1;
                x = morton_dec((x & ~s_low[j]) | (root & s_low[j]), s_mask[j]);
#pragma unroll
                for (int w = 0; w < CW; ++w) {
                    const int lo_k = w * CP::kPer;
                    uint64_t lowf = 0ull;
                    if (j >= lo_k + CP::kPer) lowf = ~0ull;
                    else if (j > lo_k) lowf = (1ull << ((j - lo_k) * CP::kBits)) - 1ull;
                    yc[w] = (yc[w] & ~lowf) | (rootc[w] & lowf);
                }
#pragma unroll
                for (int w = 0; w < CW; ++w)
                    if (w == CP::word(j)) yc[w] -= 1ull << CP::shift(j);
                r = uniform64(a.rec[x]);
                const uint32_t lowm = (2u << j) - 1u;
                diag = (diag & ~lowm) | (rec_nbr(r) & lowm);
            }
            if (alive) a.flag[a.sidx[qpos]] = 1;
        }
    }

    if (a.stats != nullptr && lane == 0) {
        atomicAdd((unsigned long long *)&a.stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)visits);
        atomicAdd((unsigned long long *)&a.stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)tests);
    }
}

// Work items a wave takes per atomic (SKYCELL_REFINE_CHUNK overrides it for
// tuning sweeps).
static uint32_t wave_refine_chunk()
{
    static int chunk = -1;
    if (chunk < 0) {
        const char *v = getenv("SKYCELL_REFINE_CHUNK");
        chunk = v ? atoi(v) : 0;
        if (chunk < 1 || chunk > 4096) chunk = 1;
    }
    return (uint32_t)chunk;
}

template <int D>
static int wave_blocks_per_cu()
{
    static int blocks_per_cu = -1;
    if (blocks_per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_refine_wave<D>, kWaveRefineThreads, 0) != hipSuccess ||
            b < 1)
            b = 1;
        blocks_per_cu = b;
    }
    return blocks_per_cu;
}

template <int D>
static hipError_t launch_wave_d(const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                                int dtype, int value_bits, hipStream_t st)
{
    WaveRefineArgs a;
    a.keys = ws.keys;
    a.fkeys = ws.fkeys;
    a.sidx = ws.sidx;
    a.rec = ws.rec;
    a.items = ws.items;
    a.ctr = ws.ctr;
    a.flag = ws.flag;
    a.stats = stats;
    a.gd = gd;
    a.chunk = wave_refine_chunk();
    a.dtype = dtype;
    a.value_bits = value_bits;
    const unsigned blocks = (unsigned)(num_cus * wave_blocks_per_cu<D>());
    hipLaunchKernelGGL(k_refine_wave<D>, dim3(blocks), dim3(kWaveRefineThreads), 0, st, a);
    return hipGetLastError();
}

#define SKYCELL_FOR_EACH_D(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t refine_wave_prepare(const GridDesc &gd)
{
    (void)wave_refine_chunk();
    switch (gd.d) {
#define SKYCELL_PREP(DD) \
    case DD:             \
        (void)wave_blocks_per_cu<DD>(); \
        return hipSuccess;
        SKYCELL_FOR_EACH_D(SKYCELL_PREP)
#undef SKYCELL_PREP
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_refine_wave(const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus, int dtype,
                              int value_bits, hipStream_t st)
{
    switch (gd.d) {
#define SKYCELL_LAUNCH(DD) \
    case DD:               \
        return launch_wave_d<DD>(gd, ws, stats, num_cus, dtype, value_bits, st);
        SKYCELL_FOR_EACH_D(SKYCELL_LAUNCH)
#undef SKYCELL_LAUNCH
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace skycell
