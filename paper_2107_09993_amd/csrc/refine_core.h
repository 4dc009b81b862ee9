// Lane loop of the exact refine (SkyCell paper, Algorithm 1, RefineSkyline,
// with the cross-cell correction below), shared by the single-instance refine
// kernel and the batched kernel.
//
// A point p can only be dominated by a point q whose cell is <= cell(p) in
// every dimension (the column map is non-decreasing).  The paper refines each
// candidate cell on its own, which misses dominators in other candidate cells
// that share a column with cell(p); this loop instead checks p against every
// surviving point of every non-empty cell in the lower cone of cell(p).  All
// such cells survive the cell-domination prune (a cell below a surviving cell
// cannot be dominated), and pruned points never need to be candidates because
// whatever dominates them also dominates anything they dominate.
//
// Cone walk.  With c the query cell, the cells y <= c are c - delta, delta >= 0,
// visited in odometer order (delta[0] fastest).  From the current cell the next
// one lowers the smallest dimension j that still can be lowered, after putting
// dimensions below j back to c's columns: y = anchor_j - e_j, where anchor_j =
// c - (0, .., 0, delta[j], delta[j+1], ..).  The lower closure is monotone, so
// once the cone below anchor_j - e_j is empty every larger delta[j] is empty
// too and the walk carries to j + 1.  Whether anchor_j - e_j is worth a visit
// is bit j of anchor_j's lower-neighbour mask; the walk only keeps those d bits
// ("diag"), refreshed from the record of every visited cell, so it never probes
// an empty cone, never steps back up and holds O(1) state.
//
// Candidate tests.  Each candidate point is first screened with its packed
// 7-bit columns; only candidates that screening cannot decide are compared
// exactly (Definition 1 on order-preserving integer keys), one turn later.
//
// Mapping.  One lane owns one work item (up to M query points of one cell, in
// registers) and runs its walk; lanes whose item ends take the next item of
// the wave's current range, and the wave asks its feeder for a new range when
// that one is used up, so unequal cone sizes do not idle the wave.  Each loop
// turn issues every load a lane needs (the next cell record, the screening
// columns of up to two candidates, the exact keys of a deferred candidate, a
// new item and its query points) and waits once.
#pragma once

#include "common.h"

namespace skycell {

constexpr uint64_t kHigh = 0x8080808080808080ull;
constexpr uint64_t kOnes = 0x0101010101010101ull;
constexpr int kRefillMin = 8;  // idle lanes that trigger handing out new items

// Hides a value from the optimiser (an empty register constraint, no
// instruction), so that OR-accumulated arithmetic stays arithmetic instead of
// being turned back into per-element compares and lane-mask chains.
__device__ __forceinline__ void opaque(uint32_t &v) { asm("" : "+v"(v)); }

// Exact keys of sorted point i: D words, with 16- or 8-byte vector loads when
// D allows (rows are 4*D bytes apart from a 256-byte aligned base).
template <int D>
__device__ __forceinline__ void load_keys(const uint32_t *__restrict__ keys, uint32_t i, uint32_t (&out)[D])
{
    const uint32_t *p = keys + (size_t)i * D;
    if constexpr (D % 4 == 0) {
        const uint4 *v = reinterpret_cast<const uint4 *>(p);
#pragma unroll
        for (int j = 0; j < D / 4; ++j) {
            const uint4 a = v[j];
            out[4 * j] = a.x;
            out[4 * j + 1] = a.y;
            out[4 * j + 2] = a.z;
            out[4 * j + 3] = a.w;
        }
    } else if constexpr (D % 2 == 0) {
        const uint2 *v = reinterpret_cast<const uint2 *>(p);
#pragma unroll
        for (int j = 0; j < D / 2; ++j) {
            const uint2 a = v[j];
            out[2 * j] = a.x;
            out[2 * j + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) out[k] = p[k];
    }
}

// Screening columns of sorted point i: FW 64-bit words.
template <int FW>
__device__ __forceinline__ void load_fine(const uint64_t *__restrict__ fkeys, uint32_t i, uint64_t (&out)[FW])
{
    const uint64_t *p = fkeys + (size_t)i * FW;
    if constexpr (FW == 2) {
        const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(p);
        out[0] = a.x;
        out[1] = a.y;
    } else {
#pragma unroll
        for (int w = 0; w < FW; ++w) out[w] = p[w];
    }
}

// The sorted data of one instance.  mask/low point to per-wave (or per-block)
// shared memory: mask[k] = index bits of dimension k, low[j] = index bits of
// dimensions below j.
struct RefineView {
    const uint32_t *keys;
    const uint64_t *fkeys;
    const int32_t *sidx;
    const uint64_t *rec;
    const uint2 *items;
    uint8_t *flag;
    const uint32_t *mask;
    const uint32_t *low;
};

// Feeder: `bool next(uint32_t &lo, uint32_t &hi)` is called by the whole wave
// and returns a wave-uniform range of item indices, or false when there is no
// more work for this wave.
template <int D, int M, class Feeder>
__device__ void refine_loop(const RefineView &v, Feeder &feed, uint32_t &visits, uint32_t &tests)
{
    constexpr int FW = fine_words(D);
    constexpr uint32_t kAll = (1u << D) - 1u;
    // bytes of the last screening word beyond dimension D-1: 0x7F in the query
    // word so that they never fail the <= or < byte tests
    constexpr uint64_t kPad = (D % 8 == 0) ? 0ull : (~0ull << (8 * (D % 8))) & 0x7F7F7F7F7F7F7F7Full;
    const int lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    uint32_t q[M][D];
    uint64_t qf[M][FW];
#pragma unroll
    for (int t = 0; t < M; ++t) {
#pragma unroll
        for (int k = 0; k < D; ++k) q[t][k] = 0u;
#pragma unroll
        for (int w = 0; w < FW; ++w) qf[t][w] = kHigh;
    }
    uint32_t alive = 0u, qstart = 0u, qcnt = 0u;
    uint32_t root = 0u, x = 0u, diag = 0u;
    bool walking = false;
    uint32_t cur = 0u, end = 0u, pcur = 0u, pend = 0u;
    uint32_t ex = 0u, exmask = 0u;
    // lane state: 0 idle, 1 item index known (its item is loaded this turn),
    // 2 item known (its cell record and query keys are loaded this turn), 3 active
    int st = 0;
    uint32_t my = 0u;
    // the wave's current range of items [r_next, r_end) (wave-uniform)
    uint32_t r_next = 0u, r_end = 0u;
    bool exhausted = false;

    for (;;) {
        // ---- hand items of the wave's range to idle lanes (in batches, so that
        // the setup turns of many lanes coincide); ask for a new range when empty
        const uint64_t idle = __ballot(st == 0);
        if (idle != 0ull && !exhausted &&
            (__popcll(idle) >= kRefillMin || __ballot(st == 3) == 0ull)) {
            if (r_next >= r_end) {
                uint32_t lo = 0u, hi = 0u;
                if (feed.next(lo, hi)) {
                    r_next = lo;
                    r_end = hi;
                } else {
                    exhausted = true;
                }
            }
            if (r_next < r_end) {
                const uint32_t rank = (uint32_t)__popcll(idle & below);
                if (st == 0 && r_next + rank < r_end) {
                    my = r_next + rank;
                    st = 1;
                }
                const uint32_t took = (uint32_t)__popcll(idle);
                r_next = r_next + took < r_end ? r_next + took : r_end;
            }
        }
        if (__ballot(st != 0) == 0ull) {
            if (exhausted) break;  // the feeder has no more work
            continue;              // take the next range
        }
        const bool active = st == 3;

        // ---- issue this turn's loads
        uint2 it = make_uint2(0u, 0u);
        if (st == 1) it = v.items[my];
        uint64_t r0 = 0ull;
        if (st == 2) {
            r0 = v.rec[root];
            // rows past the item's last point repeat it; only alive bits count
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const uint32_t row = qstart + ((uint32_t)t < qcnt ? (uint32_t)t : qcnt - 1u);
                load_keys<D>(v.keys, row, q[t]);
                load_fine<FW>(v.fkeys, row, qf[t]);
            }
        }
        const bool c0ok = active && cur < end;
        const bool c1ok = active && cur + 1 < end;
        uint64_t f0[FW], f1[FW];
        if (c0ok) load_fine<FW>(v.fkeys, cur, f0);
        if (c1ok) load_fine<FW>(v.fkeys, cur + 1, f1);
        const bool exok = active && exmask != 0u;
        uint32_t e[D];
        if (exok) load_keys<D>(v.keys, ex, e);
        bool stepped = false;
        int j = 0;
        uint32_t y = 0u;
        uint64_t r = 0ull;
        if (active && walking && pcur >= pend) {
            if (diag == 0u) {
                walking = false;
            } else {
                j = __ffs(diag) - 1;
                y = morton_dec((x & ~v.low[j]) | (root & v.low[j]), v.mask[j]);
                r = v.rec[y];
                stepped = true;
            }
        }

        // ---- item setup
        if (st == 1) {
            qcnt = it.y >> 26;
            qstart = it.x;
            root = it.y & ((1u << 26) - 1u);
            st = 2;
        } else if (st == 2) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
#pragma unroll
                for (int w = 0; w < FW; ++w) qf[t][w] |= kHigh;
                qf[t][FW - 1] |= kPad;
            }
            alive = (1u << qcnt) - 1u;
            x = root;
            diag = rec_nbr(r0) & kAll;
            walking = true;
            cur = rec_start(r0);
            uint32_t c = rec_count(r0);
            if (c == kRecCountSat) c = rec_start(v.rec[root + 1]) - cur;
            end = cur + c;
            pcur = pend = 0u;
            exmask = 0u;
            st = 3;
            ++visits;
        }

        // ---- deferred exact test (Definition 1) of one flagged query point per
        // turn, the lowest: e dominates q iff no coordinate of e exceeds q's
        // (max(e,q) ^ q is zero in every dimension) and some coordinate differs.
        // Another flagged point keeps the slot, and the candidate's keys are
        // loaded again, for the next turn.
        if (exok) {
            exmask &= alive;
            const uint32_t tb = exmask & (0u - exmask);
            uint32_t gt = 0u, ne = 0u;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t qv = q[0][k];
#pragma unroll
                for (int t = 1; t < M; ++t) qv = tb == (1u << t) ? q[t][k] : qv;
                uint32_t g = max(e[k], qv) ^ qv, x = e[k] ^ qv;
                opaque(g);
                opaque(x);
                gt |= g;
                ne |= x;
            }
            if (gt == 0u && ne != 0u) alive &= ~tb;
            exmask &= ~tb;
        }

        // ---- screening of up to two candidates.  Per byte, (p | 0x80) - q has its
        // top bit set iff q <= p, and (p | 0x80) - q - 1 iff q < p; no borrow
        // crosses bytes because both columns are below 0x80.  q < p in every
        // screening column already proves q < p in every coordinate; q <= p in
        // every column leaves the exact comparison to decide.  A query point is
        // never screened against itself.
        if (c0ok) {
            uint32_t adv = 0u;
#pragma unroll
            for (int cnd = 0; cnd < 2; ++cnd) {
                if (cnd == 1 && !c1ok) break;
                const uint32_t cidx = cur + (uint32_t)cnd;
                // query points screened: alive, and not the candidate itself
                const uint32_t self = cidx - qstart;
                const uint32_t act = alive & ~(self < (uint32_t)M ? (1u << self) : 0u);
                uint32_t le_bits = 0u, lt_bits = 0u;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    uint64_t nle = 0ull, nlt = 0ull;
#pragma unroll
                    for (int w = 0; w < FW; ++w) {
                        const uint64_t diff = qf[t][w] - (cnd == 0 ? f0[w] : f1[w]);
                        nle |= ~diff & kHigh;
                        nlt |= ~(diff - kOnes) & kHigh;
                    }
                    le_bits |= nle == 0ull ? (1u << t) : 0u;
                    lt_bits |= nlt == 0ull ? (1u << t) : 0u;
                }
                tests += (uint32_t)__popc(act);
                alive &= ~(lt_bits & act);
                uint32_t pass = le_bits & ~lt_bits & act;
                pass &= alive;
                if (pass == 0u) {
                    ++adv;
                    continue;
                }
                if (exmask == 0u) {
                    ex = cidx;
                    exmask = pass;
                    ++adv;
                    continue;
                }
                break;  // the exact slot is taken: screen this candidate again next turn
            }
            cur += adv;
            if (cur >= end && pcur < pend) {
                cur = pcur;
                end = pend;
                pcur = pend = 0u;
            }
        }

        // ---- walk step: take the record of the new cell
        if (stepped) {
            x = y;
            const uint32_t lowm = (2u << j) - 1u;
            diag = (diag & ~lowm) | (rec_nbr(r) & lowm);
            ++visits;
            if (rec_surv(r)) {
                const uint32_t s = rec_start(r);
                uint32_t c = rec_count(r);
                if (c == kRecCountSat) c = rec_start(v.rec[y + 1]) - s;
                if (cur >= end) {
                    cur = s;
                    end = s + c;
                } else {
                    pcur = s;
                    pend = s + c;
                }
            }
        }

        // ---- item end
        if (active) {
            if (alive == 0u) {
                st = 0;  // every query point of the item is dominated
            } else if (!walking && cur >= end && pcur >= pend && exmask == 0u) {
#pragma unroll
                for (int t = 0; t < M; ++t)
                    if (alive & (1u << t)) v.flag[v.sidx[qstart + t]] = 1;
                st = 0;
            }
        }
    }
}

}  // namespace skycell
