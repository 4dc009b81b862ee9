// Walk records of the lane form of the refine (d <= 8; layout in common.h),
// built after the scatter from the cell records and the sorted points'
// screening columns: per cell the minimum halved screening column of its
// points in every dimension, and those minima's prefix minimum over the first
// few dimensions, with the record's lower-neighbour mask.
#include "cellops.h"
#include "common.h"
#include "refine_core.h"

namespace skycell {

constexpr int kWrecThreads = 256;

// Walk records (common.h) of every cell, after the scatter.  One workgroup per
// tile of cells: the 2^(P*r) cells that share the index bits outside the first
// P dimensions (tile element t has bit b*P + k for index bit b*D + k), or,
// without a prefix (P = 0), 2^tb consecutive cells.
//   1. Per cell, the bytewise minimum of the screening columns of its sorted
//      points, halved into 6-bit fields: the record's second word.  One lane
//      per cell; a cell of more than kWrecLanePoints points is reduced by the
//      whole wave together (strided loads, then a butterfly of minima).
//   2. The fieldwise prefix minimum of those words over the tile's P
//      dimensions, in LDS: per dimension k and column bit b, in increasing b,
//      every element with that bit set takes the minimum with the element that
//      has it cleared and dimension k's lower column bits all set (the
//      bit-level prefix of the lower closure, with min instead of or).  With
//      the record's lower-neighbour mask: the first word.
constexpr uint32_t kWrecLanePoints = 32;
constexpr int kWrecBatch = 4;
constexpr int kWrecRounds = (1 << kWrecTileBits) / (kWrecThreads * kWrecBatch);
static_assert(kWrecRounds * kWrecThreads * kWrecBatch == (1 << kWrecTileBits), "rounds cover a whole tile");

// Bytewise minimum of two words of 7-bit bytes.
__device__ __forceinline__ uint64_t bytes_min(uint64_t a, uint64_t b)
{
    const uint64_t ge = ((b | kHigh) - a) & kHigh;  // top bit of a byte: b >= a there
    const uint64_t sel = (ge - (ge >> 7)) | ge;     // 0xFF in those bytes
    return (a & sel) | (b & ~sel);
}

// Fieldwise minimum of two words of 6-bit fields in 7-bit slots (guard bits zero).
__device__ __forceinline__ uint64_t fields_min(uint64_t a, uint64_t b)
{
    constexpr uint64_t kG = wrec_guards();
    const uint64_t ge = ((b | kG) - a) & kG;  // guard bit of a field: b >= a there
    const uint64_t sel = (ge - (ge >> 6)) | ge;
    return (a & sel) | (b & ~sel);
}

// With slabs (lane form with split cones, cellops.h), the output flags of the
// points of every split cell are set: its slab items clear the flags of the
// points they find dominated.
template <int D>
__global__ __launch_bounds__(kWrecThreads) void k_wrec(const uint64_t *__restrict__ rec,
                                                         const uint64_t *__restrict__ fkeys,
                                                         uint64_t *__restrict__ wrec, int r, int pdims, int tb,
                                                         const uint32_t *__restrict__ ctr_split, uint32_t n,
                                                         const int32_t *__restrict__ sidx,
                                                         uint8_t *__restrict__ flag)
{
    constexpr uint32_t kAll = (1u << D) - 1u;
    constexpr uint64_t kNone = 0x7F7F7F7F7F7F7F7Full;
    __shared__ uint64_t s_v[1u << kWrecTileBits];
    __shared__ uint8_t s_nb[1u << kWrecTileBits];
    const uint32_t tsize = 1u << tb;
    const uint32_t cells = 1u << (r * D);
    uint32_t inmask = 0u;
    if (pdims > 0) {
        for (int b = 0; b < r; ++b)
            for (int k = 0; k < pdims; ++k) inmask |= 1u << (b * D + k);
    } else {
        inmask = tsize - 1u;
    }
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
        if (pdims == 0) return base | t;
        uint32_t xi = base;
        for (int b = 0; b < r; ++b) xi |= ((t >> (b * pdims)) & lowdims) << (b * D);
        return xi;
    };
    // 1. own minima, kWrecBatch cells per thread and round so that their record
    // and first screening-word loads are in flight together; every lane runs
    // every round (lanes past the tile hold no points), so the butterfly of a
    // large cell sees all 64 lanes.  The minima stay in registers until both
    // words of a record are written together.
    uint64_t own[kWrecRounds][kWrecBatch];
#pragma unroll
    for (int rd = 0; rd < kWrecRounds; ++rd) {
        const uint32_t t0 = (uint32_t)rd * kWrecThreads * kWrecBatch;
        if (t0 >= tsize) break;
        uint32_t xi[kWrecBatch], s[kWrecBatch], c[kWrecBatch];
        uint64_t rr[kWrecBatch];
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            const uint32_t t = t0 + (uint32_t)q * kWrecThreads + threadIdx.x;
            xi[q] = t < tsize ? cell_of(t) : 0u;
            rr[q] = t < tsize ? rec[xi[q]] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            s[q] = 0u;
            c[q] = 0u;
            if (rec_surv(rr[q])) {
                s[q] = rec_start(rr[q]);
                c[q] = rec_count(rr[q]);
                if (c[q] == kRecCountSat) c[q] = rec_start(rec[xi[q] + 1]) - s[q];
            }
        }
        bool split[kWrecBatch];
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            split[q] = ctr_split != nullptr && c[q] != 0u && cell_slabs(rr[q], ctr_split, n) > 1u;
            if (split[q] && c[q] <= kWrecLanePoints)
                for (uint32_t i = 0; i < c[q]; ++i) flag[sidx[s[q] + i]] = 1;
        }
        uint64_t mn[kWrecBatch];
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            const bool small = c[q] <= kWrecLanePoints;
            const uint64_t f0 = small && c[q] > 0u ? fkeys[s[q]] : kNone;
            const uint64_t f1 = small && c[q] > 1u ? fkeys[s[q] + 1] : kNone;
            mn[q] = bytes_min(f0, f1);
        }
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            const uint32_t cnt_own = c[q] <= kWrecLanePoints ? c[q] : 0u;
            for (uint32_t i = 2; i < cnt_own; ++i) mn[q] = bytes_min(mn[q], fkeys[s[q] + i]);
            uint64_t big = __ballot(c[q] > kWrecLanePoints);
            while (big != 0ull) {
                const int l = __builtin_ctzll(big);
                big &= big - 1ull;
                const uint32_t bs = __builtin_amdgcn_readlane(s[q], l);
                const uint32_t bc = __builtin_amdgcn_readlane(c[q], l);
                const bool bsplit = __builtin_amdgcn_readlane(split[q] ? 1u : 0u, l) != 0u;
                uint64_t part = kNone;
                for (uint32_t i = __lane_id(); i < bc; i += kWave) {
                    part = bytes_min(part, fkeys[bs + i]);
                    if (bsplit) flag[sidx[bs + i]] = 1;
                }
                for (int off = kWave / 2; off > 0; off >>= 1) part = bytes_min(part, __shfl_xor(part, off));
                if (__lane_id() == (unsigned)l) mn[q] = part;
            }
            uint64_t wv = 0ull;
#pragma unroll
            for (int k = 0; k < D; ++k) wv |= ((mn[q] >> (8 * k + 1)) & 0x3Full) << (7 * k);
            own[rd][q] = wv;
            const uint32_t t = t0 + (uint32_t)q * kWrecThreads + threadIdx.x;
            if (t < tsize) {
                s_v[t] = wv;
                s_nb[t] = (uint8_t)(rec_nbr(rr[q]) & kAll);
            }
        }
    }
    __syncthreads();
    // 2. prefix minima over the first pdims dimensions
    for (int k = 0; k < pdims; ++k) {
        uint32_t low = 0u;
        for (int b = 0; b < r; ++b) {
            const int pos = b * pdims + k;
            const uint32_t pbit = 1u << pos;
            for (uint32_t u = threadIdx.x; u < tsize / 2; u += kWrecThreads) {
                const uint32_t t = ((u >> pos) << (pos + 1)) | pbit | (u & (pbit - 1u));
                s_v[t] = fields_min(s_v[t], s_v[(t & ~pbit) | low]);
            }
            __syncthreads();
            low |= pbit;
        }
    }
#pragma unroll
    for (int rd = 0; rd < kWrecRounds; ++rd) {
#pragma unroll
        for (int q = 0; q < kWrecBatch; ++q) {
            const uint32_t t = (uint32_t)rd * kWrecThreads * kWrecBatch + (uint32_t)q * kWrecThreads + threadIdx.x;
            if (t < tsize)
                reinterpret_cast<ulonglong2 *>(wrec)[cell_of(t)] =
                    make_ulonglong2(s_v[t] | ((uint64_t)s_nb[t] << 56), own[rd][q]);
        }
    }
}

// Walk records for the lane form's minimum-corner screen (after the scatter;
// nothing to do for the other forms).
hipError_t launch_walk_records(const GridDesc &gd, const Workspace &ws, int64_t n, hipStream_t st)
{
    if (gd.tile || gd.m == kWaveItemPoints || !lane_mc(gd)) return hipSuccess;
    const int pdims = wrec_prefix_dims(gd.d, gd.r);
    const int all = gd.r * gd.d;
    const int tb = pdims > 0 ? pdims * gd.r : (all < kWrecTileBits ? all : kWrecTileBits);
    const unsigned tiles = gd.cells >> tb;
    switch (gd.d) {
#define SKYCELL_WREC_CASE(DD)                                                                            \
    case DD:                                                                                             \
        hipLaunchKernelGGL((k_wrec<DD>), dim3(tiles), dim3(kWrecThreads), 0, st, (const uint64_t *)ws.rec, \
                           (const uint64_t *)ws.fkeys, ws.wrec, gd.r, pdims, tb,                         \
                           gd.split ? (const uint32_t *)ws.ctr : nullptr, (uint32_t)n,                             \
                           (const int32_t *)ws.sidx, ws.flag);                                           \
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

}  // namespace skycell
