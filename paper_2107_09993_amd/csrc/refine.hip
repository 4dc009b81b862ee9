// K5: exact refine of the surviving points (SkyCell paper, Algorithm 1,
// RefineSkyline, with the cross-cell correction below).
//
// A point p can only be dominated by a point q whose cell is <= cell(p) in
// every dimension (the column map is non-decreasing).  The paper refines each
// candidate cell on its own, which misses dominators in other candidate cells
// that share a column with cell(p); this kernel instead checks p against every
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
// 7-bit columns (one 64-bit subtraction per eight dimensions tests q <= p in
// every byte); only candidates that pass are compared exactly (Definition 1 on
// order-preserving integer keys), one turn later.
//
// Mapping.  One lane owns one work item (up to M query points of one cell, in
// registers) and runs its walk; lanes whose item ends take new items from a
// queue, a batch per wave, so unequal cone sizes do not idle the wave.  Each
// loop turn issues every load a lane needs (the next cell record, the screening
// columns of up to two candidates, the exact keys of a deferred candidate) and
// waits once.  Items are in Morton order of their cells and split into
// kNumXcd contiguous shares with one queue each; workgroup b starts on share
// b % kNumXcd (the XCD it is dispatched to), so the waves sharing an L2 work
// on neighbouring cells and their cones, and moves on to the other shares once
// its own is empty.
#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kRefineThreads = 256;
constexpr int kRefillMin = 16;
constexpr uint64_t kHigh = 0x8080808080808080ull;

template <int D>
__global__ __launch_bounds__(kRefineThreads) void k_refine(const uint32_t *__restrict__ keys,
                                                           const uint64_t *__restrict__ fkeys,
                                                           const int32_t *__restrict__ sidx,
                                                           const uint64_t *__restrict__ rec,
                                                           const uint2 *__restrict__ items,
                                                           uint32_t *__restrict__ ctr,
                                                           uint8_t *__restrict__ flag, GridDesc gd,
                                                           uint64_t *__restrict__ stats)
{
    constexpr int M = items_per_group(D);
    constexpr int FW = fine_words(D);
    constexpr uint32_t kAll = (1u << D) - 1u;
    __shared__ uint32_t s_mask[kMaxD], s_low[kMaxD];
    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= gd.mask[k];
        s_mask[threadIdx.x] = threadIdx.x < (unsigned)D ? gd.mask[threadIdx.x] : 0u;
        s_low[threadIdx.x] = low;
    }
    __syncthreads();

    const uint32_t n_items = ctr[kCtrItems];
    int share = (int)(blockIdx.x % kNumXcd);  // wave-uniform
    int shares_left = kNumXcd;
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
    bool active = false, exhausted = false;
    uint64_t visits = 0ull, tests = 0ull;

    for (;;) {
        // ---- refill idle lanes, a batch per wave
        const bool wants = !active && !exhausted;
        const uint64_t want = __ballot(wants);
        const uint64_t busy = __ballot(active);
        if (want != 0ull && (__popcll(want) >= kRefillMin || busy == 0ull)) {
            const int leader = __ffsll((unsigned long long)want) - 1;
            const uint32_t s_lo = (uint32_t)(((uint64_t)n_items * share) / kNumXcd);
            const uint32_t s_hi = (uint32_t)(((uint64_t)n_items * (share + 1)) / kNumXcd);
            uint32_t base = 0u;
            if (lane == leader) base = atomicAdd(&ctr[kCtrHead + share], (uint32_t)__popcll(want));
            base = __shfl(base, leader) + s_lo;
            if (base + (uint32_t)__popcll(want) > s_hi) {
                share = share + 1 == kNumXcd ? 0 : share + 1;
                --shares_left;
            }
            if (wants) {
                const uint32_t my = base + (uint32_t)__popcll(want & below);
                if (my < s_hi) {
                    const uint2 it = items[my];
                    qcnt = it.y >> 26;
                    qstart = it.x;
                    root = it.y & ((1u << 26) - 1u);
                    const uint64_t r = rec[root];
#pragma unroll
                    for (int t = 0; t < M; ++t) {
                        const bool has = t < (int)qcnt;
#pragma unroll
                        for (int k = 0; k < D; ++k) q[t][k] = has ? keys[(size_t)(qstart + t) * D + k] : 0u;
#pragma unroll
                        for (int w = 0; w < FW; ++w)
                            qf[t][w] = (has ? fkeys[(size_t)(qstart + t) * FW + w] : 0ull) | kHigh;
                    }
                    alive = (1u << qcnt) - 1u;
                    x = root;
                    diag = rec_nbr(r) & kAll;
                    walking = true;
                    cur = rec_start(r);
                    uint32_t c = rec_count(r);
                    if (c == kRecCountSat) c = rec_start(rec[root + 1]) - cur;
                    end = cur + c;
                    pcur = pend = 0u;
                    exmask = 0u;
                    active = true;
                    ++visits;
                } else if (shares_left <= 0) {
                    exhausted = true;
                }
            }
        }
        if (__ballot(active) == 0ull) {
            if (__ballot(!exhausted) == 0ull) break;  // every share is empty
            continue;                                  // retry the refill on the next share
        }

        // ---- issue this turn's loads
        const bool c0ok = active && cur < end;
        const bool c1ok = active && cur + 1 < end;
        uint64_t f0[FW], f1[FW];
#pragma unroll
        for (int w = 0; w < FW; ++w) {
            f0[w] = c0ok ? fkeys[(size_t)cur * FW + w] : 0ull;
            f1[w] = c1ok ? fkeys[(size_t)(cur + 1) * FW + w] : 0ull;
        }
        const bool exok = active && exmask != 0u;
        uint32_t e[D];
#pragma unroll
        for (int k = 0; k < D; ++k) e[k] = exok ? keys[(size_t)ex * D + k] : 0u;
        bool stepped = false;
        int j = 0;
        uint32_t y = 0u;
        uint64_t r = 0ull;
        if (active && walking && pcur >= pend) {
            if (diag == 0u) {
                walking = false;
            } else {
                j = __ffs(diag) - 1;
                y = morton_dec((x & ~s_low[j]) | (root & s_low[j]), s_mask[j]);
                r = rec[y];
                stepped = true;
            }
        }

        // ---- deferred exact test (Definition 1)
        if (exok) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if ((exmask & alive) & (1u << t)) {
                    bool le = true, ne = false;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        le = le && (e[k] <= q[t][k]);
                        ne = ne || (e[k] != q[t][k]);
                    }
                    if (le && ne) alive &= ~(1u << t);
                }
            }
            exmask = 0u;
        }

        // ---- screening of up to two candidates
        if (c0ok) {
            uint32_t adv = 0u;
#pragma unroll
            for (int cnd = 0; cnd < 2; ++cnd) {
                if (cnd == 1 && !c1ok) break;
                uint32_t pass = 0u;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    if (alive & (1u << t)) {
                        bool ok = true;
#pragma unroll
                        for (int w = 0; w < FW; ++w) {
                            const uint64_t diff = qf[t][w] - (cnd == 0 ? f0[w] : f1[w]);
                            ok = ok && ((diff & kHigh) == kHigh);
                        }
                        if (ok) pass |= 1u << t;
                        ++tests;
                    }
                }
                if (pass == 0u) {
                    ++adv;
                    continue;
                }
                if (exmask == 0u) {
                    ex = cur + (uint32_t)cnd;
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
            const uint32_t low = (2u << j) - 1u;
            diag = (diag & ~low) | (rec_nbr(r) & low);
            ++visits;
            if (rec_surv(r)) {
                const uint32_t s = rec_start(r);
                uint32_t c = rec_count(r);
                if (c == kRecCountSat) c = rec_start(rec[y + 1]) - s;
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
                active = false;  // every query point of the item is dominated
            } else if (!walking && cur >= end && pcur >= pend && exmask == 0u) {
#pragma unroll
                for (int t = 0; t < M; ++t)
                    if (alive & (1u << t)) flag[sidx[qstart + t]] = 1;
                active = false;
            }
        }
    }

    if (stats != nullptr) {
        for (int off = 32; off > 0; off >>= 1) {
            visits += __shfl_xor(visits, off);
            tests += __shfl_xor(tests, off);
        }
        if (lane == 0) {
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)visits);
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)tests);
        }
    }
}

template <int D>
static hipError_t launch_refine_d(const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                                  int num_cus, hipStream_t st)
{
    static int blocks_per_cu = -1;
    if (blocks_per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_refine<D>, kRefineThreads, 0) != hipSuccess || b < 1)
            b = 1;
        blocks_per_cu = b;
    }
    const unsigned blocks = (unsigned)(num_cus * blocks_per_cu);
    hipLaunchKernelGGL(k_refine<D>, dim3(blocks), dim3(kRefineThreads), 0, st,
                       (const uint32_t *)ws.keys, (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx,
                       (const uint64_t *)ws.rec, (const uint2 *)ws.items, ws.ctr, ws.flag, gd, stats);
    return hipGetLastError();
}

hipError_t launch_refine(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                         int num_cus, hipStream_t st)
{
    (void)n;
    switch (gd.d) {
#define SKYCELL_REFINE_CASE(DD) \
    case DD:                    \
        return launch_refine_d<DD>(gd, ws, stats, num_cus, st);
        SKYCELL_REFINE_CASE(1)
        SKYCELL_REFINE_CASE(2)
        SKYCELL_REFINE_CASE(3)
        SKYCELL_REFINE_CASE(4)
        SKYCELL_REFINE_CASE(5)
        SKYCELL_REFINE_CASE(6)
        SKYCELL_REFINE_CASE(7)
        SKYCELL_REFINE_CASE(8)
        SKYCELL_REFINE_CASE(9)
        SKYCELL_REFINE_CASE(10)
        SKYCELL_REFINE_CASE(11)
        SKYCELL_REFINE_CASE(12)
        SKYCELL_REFINE_CASE(13)
        SKYCELL_REFINE_CASE(14)
        SKYCELL_REFINE_CASE(15)
        SKYCELL_REFINE_CASE(16)
#undef SKYCELL_REFINE_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace skycell
