// Per-element operations of the grid phase, shared by the single-instance
// kernels (one thread per element over the whole GPU) and the batched kernel
// (one workgroup per instance).
#pragma once

#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

// Column of a binary32 value: floor of the binary32 product x*g (round to
// nearest), clamped to [0, g-1].  Non-decreasing in x, which is all that cell
// pruning needs to stay exact.
__device__ __forceinline__ uint32_t column_f32(float v, float gf, uint32_t g, bool &nan)
{
    if (v != v) {
        nan = true;
        return 0u;
    }
    const float f = floorf(__fmul_rn(v, gf));
    if (!(f >= 0.0f)) return 0u;
    if (f >= gf) return g - 1u;
    return (uint32_t)f;
}

__device__ __forceinline__ uint32_t column_u16(uint16_t v, uint32_t g, int bits)
{
    const uint64_t c = ((uint64_t)v * g) >> bits;
    return c > g - 1u ? g - 1u : (uint32_t)c;
}

// Equation 1 for point i of an SoA block: Morton index of its cell.
template <typename T>
__device__ __forceinline__ uint32_t point_cell(const T *__restrict__ pts, uint32_t n, uint32_t i,
                                               const GridDesc &gd, int value_bits, bool &nan)
{
    const float gf = (float)gd.g;
    uint32_t cell = 0u;
    for (int k = 0; k < gd.d; ++k) {
        const T v = pts[(size_t)k * n + i];
        uint32_t c;
        if constexpr (sizeof(T) == 4)
            c = column_f32(v, gf, (uint32_t)gd.g, nan);
        else
            c = column_u16(v, (uint32_t)gd.g, value_bits);
        cell |= deposit_bits(c, gd.mask[k]);
    }
    return cell;
}

// Inclusive prefix-OR of the lower-closure flags along one line of cells that
// differ only in the dimension whose index bits are `m` (line t of all_bits >> r).
__device__ __forceinline__ void lc_prefix_line(uint8_t *__restrict__ lc, uint32_t t, uint32_t m,
                                               uint32_t all_bits, uint32_t g)
{
    uint32_t x = deposit_bits(t, all_bits & ~m);
    uint8_t v = 0;
    // eight columns at a time: all loads of a chunk are issued before its stores
    constexpr uint32_t kChunk = 8;
    for (uint32_t j0 = 0; j0 < g; j0 += kChunk) {
        const uint32_t len = g - j0 < kChunk ? g - j0 : kChunk;
        uint32_t xs[kChunk];
        uint8_t f[kChunk];
#pragma unroll
        for (uint32_t u = 0; u < kChunk; ++u) {
            xs[u] = x;
            f[u] = u < len ? lc[x] : (uint8_t)0;
            if (u + 1 < len) x = morton_inc(x, m);
        }
#pragma unroll
        for (uint32_t u = 0; u < kChunk; ++u) {
            if (u < len) {
                v |= f[u];
                lc[xs[u]] = v;
            }
        }
        if (j0 + kChunk < g) x = morton_inc(x, m);
    }
}

// Cell record without its start (see common.h):
//   dominated(x)  iff  every column of x is >= 1 and lc[x - (1,...,1)] = 1,
//   i.e. a non-empty cell has a smaller column in every dimension (Definition 3);
//   mask bit k    iff  column k of x is >= 1 and lc[x - e_k] = 1, i.e. the cone
//                      below x - e_k still holds a non-empty cell.
__device__ __forceinline__ uint64_t cell_record(const GridDesc &gd, const uint32_t *__restrict__ cnt,
                                                const uint8_t *__restrict__ lc, uint32_t x,
                                                bool &occ, bool &surv)
{
    uint32_t nbr = 0u, diag = x;
    bool all_pos = true;
    for (int k = 0; k < gd.d; ++k) {
        const uint32_t m = gd.mask[k];
        if ((x & m) == 0u) {
            all_pos = false;
        } else {
            if (lc[morton_dec(x, m)]) nbr |= 1u << k;
            diag = morton_dec(diag, m);
        }
    }
    const uint32_t c = cnt[x];
    occ = c != 0u;
    surv = occ && !(all_pos && lc[diag]);
    const uint64_t cs = surv ? (c < kRecCountSat ? c : kRecCountSat) : 0u;
    return ((uint64_t)(surv ? 1u : 0u) << 63) | ((uint64_t)nbr << 47) | (cs << 32);
}

// Scatter of point i of a surviving cell to sorted position pos: exact
// order-preserving keys and packed screening columns.
template <typename T>
__device__ __forceinline__ void scatter_point(const T *__restrict__ pts, uint32_t n, int d,
                                              int value_bits, uint32_t i, uint32_t pos,
                                              uint32_t *__restrict__ keys,
                                              uint64_t *__restrict__ fkeys,
                                              int32_t *__restrict__ sidx)
{
    uint32_t *dst = keys + (size_t)pos * d;
    const int fw = fine_words(d);
    uint64_t *fdst = fkeys + (size_t)pos * fw;
    uint64_t word = 0ull;
    bool nan = false;
    for (int k = 0; k < d; ++k) {
        const T v = pts[(size_t)k * n + i];
        uint32_t f;
        if constexpr (sizeof(T) == 4) {
            dst[k] = f32_key(v);
            f = column_f32(v, (float)kFineCols, (uint32_t)kFineCols, nan);
        } else {
            dst[k] = (uint32_t)v;
            f = column_u16(v, (uint32_t)kFineCols, value_bits);
        }
        word |= (uint64_t)f << (8 * (k & 7));
        if ((k & 7) == 7 || k == d - 1) {
            fdst[k >> 3] = word;
            word = 0ull;
        }
    }
    sidx[pos] = (int32_t)i;
}

// Scan value per cell: surviving points (low 32 bits) and refine work items
// (high 32 bits); a cell with m surviving points gives ceil(m / M) items.
struct CellLoader {
    const uint64_t *rec;
    const uint32_t *cnt;
    uint32_t per_item;
    __device__ uint64_t operator()(uint64_t x) const
    {
        const uint32_t m = rec_surv(rec[x]) ? cnt[x] : 0u;
        const uint32_t it = (m + per_item - 1u) / per_item;
        return (uint64_t)m | ((uint64_t)it << 32);
    }
};

// Writes the first sorted position into the low half of the cell record and
// the cell's work items: (first sorted position, (point count << 26) | cell).
// With `recount`, the record's count field is rewritten from the scanned count.
struct CellEmitter {
    uint32_t *rec_words;
    uint2 *items;
    uint32_t per_item;
    bool recount;
    __device__ void operator()(uint64_t x, uint64_t prefix, uint64_t v) const
    {
        const uint32_t start = (uint32_t)prefix;
        rec_words[2 * x] = start;
        const uint32_t m = (uint32_t)v;
        if (recount) {
            const uint32_t hi = rec_words[2 * x + 1];
            rec_words[2 * x + 1] = (hi & ~kRecCountSat) | (m < kRecCountSat ? m : kRecCountSat);
        }
        const uint32_t it = (uint32_t)(v >> 32);
        const uint32_t ibase = (uint32_t)(prefix >> 32);
        for (uint32_t t = 0; t < it; ++t) {
            const uint32_t first = t * per_item;
            const uint32_t c = (m - first) < per_item ? (m - first) : per_item;
            items[ibase + t] = make_uint2(start + first, (c << 26) | (uint32_t)x);
        }
    }
};

}  // namespace skycell
