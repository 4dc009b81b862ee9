// Lane loop of the exact refine for d <= 8 with minimum-corner screening of
// the cone's cells (SkyCell paper, Algorithm 1, RefineSkyline, with the
// lower-cone correction described in refine_core.h).
//
// The walk over the lower cone of the item's cell is the one of refine_core.h
// (odometer order, lower-neighbour bits, O(1) state), but it reads the cells'
// walk records (common.h): the lower-neighbour mask plus, per dimension, the
// minimum halved screening column of the cell's surviving points, and that
// minimum taken over the cells below it in the first few dimensions.  A point
// q can dominate a query point p only if q <= p in every dimension, so only if
// every minimum of q's cell is <= p's halved column; when that fails for every
// live query point the cell is passed over without touching its points.  On
// the anti-correlated headline data about 7% of the non-empty cells of a cone
// pass, and they hold about 14% of its points.  The walk below a cell reached
// by a step along dimension j stays in dimensions 0..j, so when j is among the
// first dimensions and the cell's prefix minima rule out every live query
// point, that whole part of the cone is skipped (a CPU count on the same data:
// 137 visits per item fall to about 90).
//
// A passing cell's record (first sorted position and count) is loaded on the
// turn after its walk record, and its points go into the lane's candidate
// queue (the current range and one pending range).  The walk steps only while
// the queue can take what the step may add.  Screening (one candidate per
// lane and turn) and the exact test of one deferred candidate are those of
// refine_core.h.  (Running them only when many lanes of the wave hold
// candidates, so that the wave executes that code less often, was slower:
// lanes with full queues stop walking until then.)
//
// A slab item (kItemSlab, cellops.h) walks one slab of its cell's cone: it
// starts at the slab's corner and never steps along dimension D-1.  Its query
// points' flags start set, and it clears those of the points it finds
// dominated; a whole-cone item sets the flags of its surviving points.
#pragma once

#include "common.h"
#include "refine_core.h"

namespace skycell {

// The loop's per-turn loads are raw buffer loads: a 32-bit byte offset against
// a resource that holds the array's base and size, so no 64-bit address
// arithmetic per load, and a lane with nothing to load passes an offset past
// the end (kMcNoLoad), for which the hardware returns zero without touching
// memory, instead of branching around the load.  Every array then has to stay
// below 2^31 bytes: the host uses this loop only for n < kWrecMaxPoints
// (2^26 cells of 16-byte walk records are 2^30 bytes).
constexpr uint32_t kMcNoLoad = 0x80000000u;
constexpr uint32_t kBufferWord3 = 0x00020000u;  // raw 32-bit elements, gfx9 resource format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, (int)kBufferWord3);
}
__device__ __forceinline__ uint64_t buffer_u64(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return ((uint64_t)v[1] << 32) | v[0];
}
__device__ __forceinline__ ulonglong2 buffer_u128(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_ulonglong2(((uint64_t)v[1] << 32) | v[0], ((uint64_t)v[3] << 32) | v[2]);
}

// n: points of the instance (sizes of the item and screening-word arrays),
// cells: its index space (sizes of the cell and walk records).
template <int D, int M, class Feeder>
__device__ void refine_loop_mc(const RefineView &v, const uint64_t *__restrict__ wrec, int pdims, uint32_t n,
                               uint32_t cells, Feeder &feed, uint32_t &visits, uint32_t &tests)
{
    static_assert(D >= 1 && D <= kWrecMaxD, "walk records hold at most kWrecMaxD dimensions");
    constexpr uint32_t kAll = (1u << D) - 1u;
    constexpr uint64_t kPad = (D % 8 == 0) ? 0ull : (~0ull << (8 * (D % 8))) & 0x7F7F7F7F7F7F7F7Full;
    constexpr uint64_t kGuard = wrec_guards();
    const int lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const __amdgpu_buffer_rsrc_t rs_items = raw_buffer(v.items, n * 8u), rs_rec = raw_buffer(v.rec, (cells + 1u) * 8u),
                                 rs_fkeys = raw_buffer(v.fkeys, n * 8u), rs_wrec = raw_buffer(wrec, cells * 16u);

    uint32_t q[M][D];
    uint64_t qf[M], q6[M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
#pragma unroll
        for (int k = 0; k < D; ++k) q[t][k] = 0u;
        qf[t] = kHigh;
        q6[t] = kGuard;
    }
    uint32_t alive = 0u, qstart = 0u, qcnt = 0u;
    bool slab = false;  // the item walks one slab of its cell's cone (cellops.h)
    uint32_t root = 0u, x = 0u, diag = 0u;
    bool walking = false;
    uint32_t cur = 0u, end = 0u, pcur = 0u, pend = 0u;
    uint32_t ex = 0u, exmask = 0u;
    uint32_t rq = 0u;   // cell whose record is loaded this turn (rqv)
    bool rqv = false;
    int st = 0;         // 0 idle, 1 item index known, 2 item known, 3 active
    uint32_t my = 0u;
    uint32_t r_next = 0u, r_end = 0u;
    bool exhausted = false;

    for (;;) {
        // ---- hand out items (as in refine_core.h)
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
            if (exhausted) break;
            continue;
        }
        const bool active = st == 3;

        // ---- the walk may step if the queue can take a passing cell's points
        const uint32_t used = (cur < end ? 1u : 0u) + (pcur < pend ? 1u : 0u) + (rqv ? 1u : 0u);
        const bool can_step = active && walking && used <= 1u;

        // ---- issue this turn's loads
        const uint64_t it64 = buffer_u64(rs_items, st == 1 ? my * 8u : kMcNoLoad);
        const uint2 it = make_uint2((uint32_t)it64, (uint32_t)(it64 >> 32));
        const uint64_t r0 = buffer_u64(rs_rec, st == 2 ? root * 8u : kMcNoLoad);
        if (st == 2) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const uint32_t row = qstart + ((uint32_t)t < qcnt ? (uint32_t)t : qcnt - 1u);
                load_keys<D>(v.keys, row, q[t]);
                qf[t] = v.fkeys[row];
            }
        }
        const bool c0ok = active && cur < end;
        const uint64_t f0 = buffer_u64(rs_fkeys, c0ok ? cur * 8u : kMcNoLoad);
        const bool exok = active && exmask != 0u;
        uint32_t e[D];
        if (exok) load_keys<D>(v.keys, ex, e);
        const bool rqok = active && rqv;
        const uint64_t rr = buffer_u64(rs_rec, rqok ? rq * 8u : kMcNoLoad);
        // the next cell of the walk (computed on every lane: j = -1 when diag
        // is empty reads the last, unused entry of the shared tables)
        if (can_step && diag == 0u) walking = false;
        const bool stepped = can_step && diag != 0u;
        const int j = __ffs(diag) - 1;
        const uint32_t lowj = v.low[j & (kMaxD - 1)];
        const uint32_t y = morton_dec((x & ~lowj) | (root & lowj), v.mask[j & (kMaxD - 1)]);
        const ulonglong2 w = buffer_u128(rs_wrec, stepped ? y * 16u : kMcNoLoad);

        // ---- item setup
        if (st == 1) {
            qcnt = (it.y >> 26) & 31u;
            slab = (it.y & kItemSlab) != 0u;
            qstart = it.x;
            root = it.y & ((1u << 26) - 1u);
            st = 2;
        } else if (st == 2) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                // halved columns in 7-bit fields with the guard bit set (fields
                // past dimension D-1 stay 0 in the walk records: never failing)
                uint64_t h = kGuard;
#pragma unroll
                for (int k = 0; k < D; ++k) h |= ((qf[t] >> (8 * k + 1)) & 0x3Full) << (7 * k);
                q6[t] = h;
                qf[t] |= kHigh | kPad;
            }
            alive = (1u << qcnt) - 1u;
            x = root;
            diag = rec_nbr(r0) & (slab ? kAll >> 1 : kAll);  // a slab stays in dimensions 0..D-2
            walking = true;
            cur = rec_start(r0);
            uint32_t c = rec_count(r0);
            if (c == kRecCountSat) c = rec_start(v.rec[root + 1]) - cur;
            end = cur + c;
            pcur = pend = 0u;
            exmask = 0u;
            rqv = false;
            st = 3;
            ++visits;
        }

        // ---- deferred exact test of one flagged query point (refine_core.h)
        if (exok) {
            exmask &= alive;
            const uint32_t tb = exmask & (0u - exmask);
            uint32_t gt = 0u, ne = 0u;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t qv = q[0][k];
#pragma unroll
                for (int t = 1; t < M; ++t) qv = tb == (1u << t) ? q[t][k] : qv;
                uint32_t g = max(e[k], qv) ^ qv, xx = e[k] ^ qv;
                opaque(g);
                opaque(xx);
                gt |= g;
                ne |= xx;
            }
            if (gt == 0u && ne != 0u) alive &= ~tb;
            exmask &= ~tb;
        }

        // ---- screening of one candidate (as in refine_core.h, which takes up
        // to two per turn: with the walk records a turn's candidate work is
        // rare, and the second screen cost more issue slots than it saved turns)
        if (c0ok) {
            const uint32_t self = cur - qstart;
            const uint32_t act = alive & ~(self < (uint32_t)M ? (1u << self) : 0u);
            uint32_t le_bits = 0u, lt_bits = 0u;
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const uint64_t diff = qf[t] - f0;
                const uint64_t nle = ~diff & kHigh;
                const uint64_t nlt = ~(diff - kOnes) & kHigh;
                le_bits |= nle == 0ull ? (1u << t) : 0u;
                lt_bits |= nlt == 0ull ? (1u << t) : 0u;
            }
            tests += (uint32_t)__popc(act);
            alive &= ~(lt_bits & act);
            const uint32_t pass = le_bits & ~lt_bits & act & alive;
            // a candidate that needs the exact test waits while another holds it
            bool adv = true;
            if (pass != 0u) {
                if (exmask == 0u) {
                    ex = cur;
                    exmask = pass;
                } else {
                    adv = false;
                }
            }
            if (adv) ++cur;
            if (cur >= end && pcur < pend) {
                cur = pcur;
                end = pend;
                pcur = pend = 0u;
            }
        }

        // ---- record of a passing cell: its points join the candidate queue (a
        // slot is free: the step that asked for it left at most one slot used)
        if (rqok) {
            const uint32_t s = rec_start(rr);
            uint32_t c = rec_count(rr);
            if (c == kRecCountSat) c = rec_start(v.rec[rq + 1]) - s;
            if (cur >= end) {
                cur = s;
                end = s + c;
            } else {
                pcur = s;
                pend = s + c;
            }
            rqv = false;
        }

        // ---- walk step: the new cell's neighbour bits and minimum corners.  A
        // step along dimension j < pdims skips the part of the cone below the
        // new cell (lower in dimensions 0..j only) when the minima over the
        // cells <= it in the first pdims dimensions rule out every live query
        // point: no point there is <= one of them in every dimension.
        if (stepped) {
            x = y;
            const uint32_t lowm = (2u << j) - 1u;
            uint32_t nb = (uint32_t)(w.x >> 56);
            ++visits;
            const uint64_t mp = w.x & kWrecFields;
            uint32_t keep = 0u, pm = 0u;
#pragma unroll
            for (int t = 0; t < M; ++t) {
                keep |= ((q6[t] - mp) & kGuard) == kGuard ? (1u << t) : 0u;
                pm |= ((q6[t] - w.y) & kGuard) == kGuard ? (1u << t) : 0u;
            }
            if (j < pdims && (keep & alive) == 0u) nb = 0u;
            diag = (diag & ~lowm) | (nb & lowm);
            if ((pm & alive) != 0u) {
                rq = y;
                rqv = true;
            }
        }

        // ---- item end
        // (a whole-cone item sets the flags of its surviving query points; a
        // slab item, whose points start flagged, clears those it found dominated)
        if (active && (alive == 0u || (!walking && !rqv && cur >= end && pcur >= pend && exmask == 0u))) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const bool live = (alive >> t) & 1u;
                if ((uint32_t)t < qcnt && live != slab) v.flag[v.sidx[qstart + t]] = live ? 1 : 0;
            }
            st = 0;
        }
    }
}

}  // namespace skycell
