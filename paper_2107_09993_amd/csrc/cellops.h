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

// Equation 1 for point i of an SoA block: Morton index of its cell (D > 0:
// gd.d as a compile-time constant).
template <typename T, int D = 0>
__device__ __forceinline__ uint32_t point_cell(const T *__restrict__ pts, uint32_t n, uint32_t i,
                                               const GridDesc &gd, int value_bits, bool &nan)
{
    const float gf = (float)gd.g;
    const int dd = D > 0 ? D : gd.d;
    uint32_t cell = 0u;
#pragma unroll
    for (int k = 0; k < dd; ++k) {
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

// Lower closure as a bitmap: bit x of lcb[x >> 6] is 1 iff some non-empty cell
// is <= x in every dimension.
__device__ __forceinline__ bool lc_bit(const uint64_t *__restrict__ lcb, uint32_t x)
{
    return ((lcb[x >> 6] >> (x & 63u)) & 1ull) != 0ull;
}

// Cells i in [0, 64) of one bitmap word whose index bit q is set.
__host__ __device__ __forceinline__ uint64_t bit_set_pattern(int q)
{
    return q == 0 ? 0xAAAAAAAAAAAAAAAAull
           : q == 1 ? 0xCCCCCCCCCCCCCCCCull
           : q == 2 ? 0xF0F0F0F0F0F0F0F0ull
           : q == 3 ? 0xFF00FF00FF00FF00ull
           : q == 4 ? 0xFFFF0000FFFF0000ull
                    : 0xFFFFFFFF00000000ull;
}

// One step of the prefix-OR along a dimension k, at column bit level b: every
// cell whose column k has bit b set takes the OR of the cell with that bit
// cleared and the lower bits of column k all set.  Applied for b = 0, 1, ...
// this makes x the OR over every cell that differs from x only in a smaller or
// equal column k.  `p` is the index bit of (k, b), `lowk` the index bits of
// column k below b.  Within a word (index bits 0..5) it is a shift of the
// word; above, a word ORs in another word.
__host__ __device__ __forceinline__ uint64_t lc_step_word(uint64_t w, uint64_t src, int p, uint32_t lowk)
{
    const uint32_t lowlo = lowk & 63u;
    uint64_t m = p < 6 ? (w & ~bit_set_pattern(p)) : src;
    for (int q = 0; q < 6; ++q)
        if (lowlo & (1u << q)) m &= bit_set_pattern(q);
    if (p < 6) m <<= (1u << p);
    for (int q = 0; q < 6; ++q)
        if (lowlo & (1u << q)) m |= (m & bit_set_pattern(q)) >> (1u << q);
    return w | m;
}

// Cell record without its start (see common.h):
//   dominated(x)  iff  every column of x is >= 1 and lc(x - (1,...,1)) = 1,
//   i.e. a non-empty cell has a smaller column in every dimension (Definition 3);
//   mask bit k    iff  column k of x is >= 1 and lc(x - e_k) = 1, i.e. the cone
//                      below x - e_k still holds a non-empty cell.
// D > 0: the dimension count as a compile-time constant (gd.d == D).
template <int D = 0>
__device__ __forceinline__ uint64_t cell_record(const GridDesc &gd, const uint32_t *__restrict__ cnt,
                                                const uint64_t *__restrict__ lcb, uint32_t x,
                                                bool &occ, bool &surv)
{
    const int dd = D > 0 ? D : gd.d;
    uint32_t nbr = 0u, diag = x;
    bool all_pos = true;
#pragma unroll
    for (int k = 0; k < dd; ++k) {
        const uint32_t m = gd.mask[k];
        if ((x & m) == 0u) {
            all_pos = false;
        } else {
            if (lc_bit(lcb, morton_dec(x, m))) nbr |= 1u << k;
            diag = morton_dec(diag, m);
        }
    }
    const uint32_t c = cnt[x];
    occ = c != 0u;
    surv = occ && !(all_pos && lc_bit(lcb, diag));
    const uint64_t cs = surv ? (c < kRecCountSat ? c : kRecCountSat) : 0u;
    return ((uint64_t)(surv ? 1u : 0u) << 63) | ((uint64_t)nbr << 47) | (cs << 32);
}

// One point's D key words stored at dst = keys + pos * D (the key array is
// 256-byte aligned), with 16- or 8-byte stores where D makes every row aligned
// to them: fewer, wider scattered stores than one per word.
template <int D>
__device__ __forceinline__ void store_key_row(uint32_t *__restrict__ dst, const uint32_t (&kw)[D])
{
    if constexpr (D % 4 == 0) {
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
#pragma unroll
        for (int q = 0; q < D / 4; ++q) d4[q] = make_uint4(kw[4 * q], kw[4 * q + 1], kw[4 * q + 2], kw[4 * q + 3]);
    } else if constexpr (D % 2 == 0) {
        uint2 *d2 = reinterpret_cast<uint2 *>(dst);
#pragma unroll
        for (int q = 0; q < D / 2; ++q) d2[q] = make_uint2(kw[2 * q], kw[2 * q + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) dst[k] = kw[k];
    }
}

// Scatter of point i of a surviving cell to sorted position pos: exact
// order-preserving keys and packed screening columns.  The D coordinates are
// loaded before the first store, so their loads are in flight together.
template <typename T, int D>
__device__ __forceinline__ void scatter_point(const T *__restrict__ pts, uint32_t n, int value_bits, uint32_t i,
                                              uint32_t pos, uint32_t *__restrict__ keys,
                                              uint64_t *__restrict__ fkeys, int32_t *__restrict__ sidx)
{
    T v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = pts[(size_t)k * n + i];
    uint32_t *dst = keys + (size_t)pos * D;
    constexpr int fw = fine_words(D);
    uint64_t *fdst = fkeys + (size_t)pos * fw;
    uint64_t word = 0ull;
    bool nan = false;
    uint32_t kw[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        uint32_t f;
        if constexpr (sizeof(T) == 4) {
            kw[k] = f32_key(v[k]);
            f = column_f32(v[k], (float)kFineCols, (uint32_t)kFineCols, nan);
        } else {
            kw[k] = (uint32_t)v[k];
            f = column_u16(v[k], (uint32_t)kFineCols, value_bits);
        }
        word |= (uint64_t)f << (8 * (k & 7));
        if ((k & 7) == 7 || k == D - 1) {
            fdst[k >> 3] = word;
            word = 0ull;
        }
    }
    store_key_row<D>(dst, kw);
    sidx[pos] = (int32_t)i;
}

// ---- slabs of long cone walks (walk-record lane form)
// The cost of a lane-form work item is the length of its cell's cone walk,
// which is heavy-tailed (on the anti-correlated headline data the median walk
// is 54 visits, the 99th percentile 1,139, and the longest 1% of items make
// 12% of the visits).  A long walk handed out late holds its wave, and the
// launch, after the other waves are done.  The odometer walk lowers dimension
// d-1 last, so the cone of cell x is the union of its slabs s = 0..c[d-1]:
// the cells whose column d-1 is c[d-1] - s, walked from the corner
// x - s e_{d-1} in dimensions 0..d-2 only.  The slabs are independent walks
// over the same candidates, so a query point is dominated iff some slab finds
// a dominator.  The cells whose cone-size estimate sum_k log2(c_k + 1) (a
// correlation of 0.70 with the log of the walk length on the headline data)
// is in the top bins (k_split_pick) get one work item per (query group, slab),
// next to each other in Morton order, so the slabs run on neighbouring lanes
// at the same time and keep the locality of the cone walks.
constexpr int kSplitBins = 512;

// Column of cell x in the dimension whose index bits are m.
__device__ __forceinline__ uint32_t cell_column(uint32_t x, uint32_t m)
{
    uint32_t c = 0u, bit = 1u;
    while (m != 0u) {
        const uint32_t low = m & (0u - m);
        if (x & low) c |= bit;
        bit <<= 1;
        m ^= low;
    }
    return c;
}

// Cone-size estimate of cell x: prod_k (c_k + 1), the number of cells <= x,
// from the r bit planes of its Morton index (D > 0: gd.d as a constant).
template <int D = 0>
__device__ __forceinline__ float cone_cells(const GridDesc &gd, uint32_t x)
{
    const int dd = D > 0 ? D : gd.d;
    float p = 1.0f;
#pragma unroll
    for (int k = 0; k < dd; ++k) {
        uint32_t c = 0u;
        for (int b = 0; b < gd.r; ++b) c |= ((x >> (b * dd + k)) & 1u) << b;
        p *= (float)(c + 1u);
    }
    return p;
}

// Histogram bin of a cone-size estimate: 8 log2, rounded, below kSplitBins.
__device__ __forceinline__ uint32_t cone_bin(float cells)
{
    const uint32_t b = (uint32_t)(8.0f * __log2f(cells) + 0.5f);
    return b < (uint32_t)kSplitBins ? b : (uint32_t)kSplitBins - 1u;
}

// Slabs of a cell's items from its record (rec_slabs: c[d-1] + 1 for a split
// cell, else 0), or 1 for every cell if the split's added items do not fit in
// the n slots of the item array (the record pass counts both exactly).
__device__ __forceinline__ uint32_t cell_slabs(uint64_t r, const uint32_t *__restrict__ ctr, uint32_t n)
{
    const uint32_t s = rec_slabs(r);
    if (s == 0u) return 1u;
    const uint64_t need = (uint64_t)ctr[kCtrSplitItems] + ctr[kCtrSplitExtra];
    return (ctr[kCtrSplitFail] == 0u && need <= n) ? s : 1u;
}

// Scan value per cell: surviving points (low 32 bits) and refine work items
// (high 32 bits); a cell with m surviving points gives ceil(m / M) items, times
// its slabs when long walks are split (slabs: the per-cell slab bytes, or
// null).
struct CellLoader {
    const uint64_t *rec;
    const uint32_t *cnt;
    uint32_t per_item;
    const uint32_t *ctr;  // with split slabs (else null): the split counters
    uint32_t n;
    __device__ uint64_t operator()(uint64_t x) const
    {
        const uint64_t r = rec[x];
        const uint32_t m = rec_surv(r) ? cnt[x] : 0u;
        uint32_t it = (m + per_item - 1u) / per_item;
        if (ctr != nullptr && m != 0u) it *= cell_slabs(r, ctr, n);
        return (uint64_t)m | ((uint64_t)it << 32);
    }
};

// Writes the first sorted position into the low half of the cell record and
// the cell's work items: (first sorted position, (point count << 26) | cell).
// With `recount`, the record's count field is rewritten from the scanned count.
// With slabs, the items of a split cell are its query groups times its
// slabs, slab-minor: item t is group t / S, slab t % S, rooted at the slab's
// corner and flagged kItemSlab.
struct CellEmitter {
    uint32_t *rec_words;
    uint2 *items;
    uint32_t per_item;
    bool recount;
    bool split;           // the loader may have split cells into slabs
    uint32_t top_mask;    // index bits of dimension d-1
    uint32_t cap;  // slots of the item array (n); never written past
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
        // the loader multiplied the cell's query groups by its slabs
        const uint32_t groups = (m + per_item - 1u) / per_item;
        const uint32_t ns = (split && groups != 0u) ? it / groups : 1u;
        const uint32_t own = it < kLaneItems ? it : kLaneItems;
        for (uint32_t t = 0; t < own; ++t) put(ibase, start, m, (uint32_t)x, t, ns);
        // A cell with more items than one lane writes alone (on correlated data
        // a few cells can hold most of the points, thousands of items each) is
        // finished by every active lane of the wave together, consecutive lanes
        // on consecutive items.  The emitter may be called from a partly active
        // wave (the scan's last tile), so the stride is the active lane count.
        const uint64_t act = __ballot(1);
        uint64_t big = __ballot(it > kLaneItems);
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
        const uint32_t nact = (uint32_t)__builtin_popcountll(act);
        while (big != 0ull) {
            const int l = __builtin_ctzll(big);
            big &= big - 1ull;
            const uint32_t bb = __builtin_amdgcn_readlane(ibase, l);
            const uint32_t bs = __builtin_amdgcn_readlane(start, l);
            const uint32_t bm = __builtin_amdgcn_readlane(m, l);
            const uint32_t bx = __builtin_amdgcn_readlane((uint32_t)x, l);
            const uint32_t bi = __builtin_amdgcn_readlane(it, l);
            const uint32_t bsl = __builtin_amdgcn_readlane(ns, l);
            for (uint32_t t = kLaneItems + pos; t < bi; t += nact) put(bb, bs, bm, bx, t, bsl);
        }
    }
    static constexpr uint32_t kLaneItems = 8;
    __device__ void put(uint32_t ibase, uint32_t start, uint32_t m, uint32_t x, uint32_t t, uint32_t ns) const
    {
        const uint32_t grp = t / ns, slab = t - grp * ns;
        const uint32_t first = grp * per_item;
        const uint32_t c = (m - first) < per_item ? (m - first) : per_item;
        uint32_t root = x, flag = 0u;
        if (ns > 1u) {
            // x - slab * e_{d-1}: a masked subtraction in dimension d-1's bits
            root = (((x & top_mask) - deposit_bits(slab, top_mask)) & top_mask) | (x & ~top_mask);
            flag = kItemSlab;
        }
        if (ibase + t < cap) items[ibase + t] = make_uint2(start + first, (c << 26) | root | flag);
    }
};

}  // namespace skycell
