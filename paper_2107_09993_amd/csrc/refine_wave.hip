// K5, wave form: the exact refine for coarse grids, where a cell holds many
// points (SkyCell paper, Algorithm 1, RefineSkyline, with the lower-cone
// correction described in refine_core.h).
//
// A work item is up to 63 sorted points of one cell, one per lane; all of them
// share the cell's lower cone.  The wave walks that cone once, in lockstep
// (the same odometer walk as the lane form, with wave-uniform state), and at
// every non-empty surviving cell it streams the cell's points 16 or 32 at a time
// through broadcast loads: each candidate is screened against all 63 query
// points at once, lanes whose query is dominated drop out, and the wave moves
// to the next item as soon as every query point of its item is dominated.
// Per candidate this costs a handful of vector instructions for 63 tests,
// against a whole loop turn per (candidate, lane) in the lane form, which is
// what coarse grids (tens to thousands of points per cone cell) need; fine
// grids (a few points per cell) keep the lane form.
#include <cstdlib>

#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kWaveThreads = 256;
constexpr uint64_t kWHigh = 0x8080808080808080ull;
constexpr uint64_t kWOnes = 0x0101010101010101ull;

__device__ __forceinline__ uint32_t wuniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t wuniform64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
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
            base = wuniform(__shfl(base, 0)) + s_lo;
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


// Screening words of candidate i (wave-uniform index) through a vector load
// that every lane issues for the same address: a group's loads then stay in
// flight together in VGPRs, where scalar loads were waited one by one for lack
// of free SGPRs.
template <int FW>
__device__ __forceinline__ void broadcast_fine(const uint64_t *__restrict__ fkeys, uint32_t i, uint64_t (&f)[FW])
{
    asm("" : "+v"(i));
    if constexpr (FW == 2) {
        const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(fkeys + (size_t)i * 2);
        f[0] = a.x;
        f[1] = a.y;
    } else {
#pragma unroll
        for (int w = 0; w < FW; ++w) f[w] = fkeys[(size_t)i * FW + w];
    }
}

// The read-only arrays are separate restrict arguments, so that the compiler
// can serve wave-uniform reads of them from the scalar data cache.
template <int D>
__global__ __launch_bounds__(kWaveThreads) void k_refine_wave(const uint32_t *__restrict__ keys,
                                                              const uint64_t *__restrict__ fkeys,
                                                              const int32_t *__restrict__ sidx,
                                                              const uint64_t *__restrict__ rec,
                                                              const uint2 *__restrict__ items,
                                                              uint32_t *__restrict__ ctr,
                                                              uint8_t *flag,
                                                              uint64_t *__restrict__ stats, GridDesc gd,
                                                              uint32_t chunk)
{
    constexpr int FW = fine_words(D);
    constexpr uint32_t kAll = (1u << D) - 1u;
    constexpr uint64_t kPad = (D % 8 == 0) ? 0ull : (~0ull << (8 * (D % 8))) & 0x7F7F7F7F7F7F7F7Full;
    // candidates per group; up to d = 8 (one screening word per candidate)
    // the next group's words are loaded while a group is screened, above it
    // (two words) the registers of a second buffer cost more than they hide
    constexpr int G = 16;

    __shared__ uint32_t s_mask[kMaxD], s_low[kMaxD];
    if (threadIdx.x < kMaxD) {
        uint32_t low = 0u;
        for (int k = 0; k < (int)threadIdx.x && k < D; ++k) low |= gd.mask[k];
        s_mask[threadIdx.x] = threadIdx.x < (unsigned)D ? gd.mask[threadIdx.x] : 0u;
        s_low[threadIdx.x] = low;
    }
    __syncthreads();

    const uint32_t lane = (uint32_t)__lane_id();
    const uint32_t parts = (uint32_t)gd.parts;
    // work units: (item, part) pairs, unit = item * parts + part
    WaveFeeder feed{ctr + kCtrHead, ctr[kCtrItems] * parts, chunk, (int)(blockIdx.x % kNumXcd), kNumXcd};
    uint64_t visits = 0u, tests = 0u;

    uint32_t lo = 0u, hi = 0u;
    while (feed.next(lo, hi)) {
        for (uint32_t unit = lo; unit < hi; ++unit) {
            const uint32_t item = unit / parts;
            const uint32_t part = unit - item * parts;
            const uint2 it = items[item];
            const uint32_t qstart = wuniform(it.x);
            const uint32_t qcnt = wuniform(it.y >> 26);
            const uint32_t root = wuniform(it.y & ((1u << 26) - 1u));
            const bool valid = lane < qcnt;
            const uint32_t qpos = qstart + (valid ? lane : 0u);
            const uint32_t orig = (uint32_t)sidx[qpos];

            uint32_t q[D];
            uint64_t qf[FW];
#pragma unroll
            for (int k = 0; k < D; ++k) q[k] = keys[(size_t)qpos * D + k];
#pragma unroll
            for (int w = 0; w < FW; ++w) qf[w] = fkeys[(size_t)qpos * FW + w] | kWHigh;
            qf[FW - 1] |= kPad;
            bool alive = valid;
            // the part's share of the cone: every parts-th group of candidates
            // along the walk, starting with group `part`
            uint32_t gsel = 0u;
            uint32_t since_poll = 0u;

            uint32_t x = root;
            uint64_t r = wuniform64(rec[x]);
            uint32_t diag = rec_nbr(r) & kAll;
            for (;;) {
                ++visits;
                if (rec_surv(r)) {
                    const uint32_t s = rec_start(r);
                    uint32_t c = rec_count(r);
                    if (c == kRecCountSat) c = wuniform(rec_start(rec[x + 1])) - s;
                    // this part's groups of the cell are i, i + parts, ...; the
                    // next one's words are loaded while the current one is screened
                    const uint32_t ng = (c + (uint32_t)G - 1u) / (uint32_t)G;
                    uint32_t i = part >= gsel ? part - gsel : part + parts - gsel;
                    gsel = (uint32_t)((gsel + ng) % parts);
                    uint64_t fa[G][FW], fb[FW == 1 ? G : 1][FW];
                    auto load_group = [&](uint64_t (&fv)[G][FW], uint32_t gi) {
                        const uint32_t t = gi * (uint32_t)G;
#pragma unroll
                        for (int u = 0; u < G; ++u) {
                            const uint32_t ci = t + (uint32_t)u < c ? s + t + (uint32_t)u : s + c - 1u;
                            broadcast_fine<FW>(fkeys, ci, fv[u]);
                        }
                    };
                    // screens group gi; false when every point of the item is dominated
                    auto screen_group = [&](const uint64_t (&fv)[G][FW], uint32_t gi) -> bool {
                        const uint32_t t = gi * (uint32_t)G;
                        if (parts > 1u && ++since_poll == 16u) {
                            // points that another part of this item has already
                            // found dominated stop here too
                            since_poll = 0u;
                            alive = alive && *(volatile const uint8_t *)(flag + orig) != 0;
                            if (__ballot(alive) == 0ull) return false;
                        }
                        const bool was = alive;
                        tests += (uint64_t)__popcll(__ballot(alive)) * (c - t < (uint32_t)G ? c - t : (uint32_t)G);
                        uint32_t kill = 0u, need = 0u;
#pragma unroll
                        for (int u = 0; u < G; ++u) {
                            const uint32_t ci = s + t + (uint32_t)u;
                            uint64_t nle = 0ull, nlt = 0ull;
#pragma unroll
                            for (int w = 0; w < FW; ++w) {
                                const uint64_t diff = qf[w] - fv[u][w];
                                nle |= ~diff & kWHigh;
                                nlt |= ~(diff - kWOnes) & kWHigh;
                            }
                            // in range (wave-uniform), and never a point against itself
                            const bool use = t + (uint32_t)u < c && ci != qpos;
                            if (use && nlt == 0ull) kill = 1u;
                            if (use && nle == 0ull && nlt != 0ull) need |= 1u << u;
                        }
                        alive = alive && kill == 0u;
                        need = alive ? need : 0u;
                        // candidates screening cannot decide: exact comparison (Definition 1)
                        if (__ballot(need != 0u) != 0ull) {
#pragma unroll
                            for (int u = 0; u < G; ++u) {
                                if (__ballot((need >> u) & 1u) == 0ull) continue;
                                const uint32_t ci = s + t + (uint32_t)u;
                                uint32_t gt = 0u, ne = 0u;
#pragma unroll
                                for (int k = 0; k < D; ++k) {
                                    const uint32_t e = wuniform(keys[(size_t)ci * D + k]);
                                    gt |= max(e, q[k]) ^ q[k];
                                    ne |= e ^ q[k];
                                }
                                if (((need >> u) & 1u) && gt == 0u && ne != 0u) alive = false;
                            }
                        }
                        // a dominated point's flag is cleared at once (the
                        // scatter set it for every surviving point)
                        if (was && !alive) flag[orig] = 0;
                        return __ballot(alive) != 0ull;
                    };
                    if constexpr (FW == 1) {
                        if (i < ng) {
                            load_group(fa, i);
                            for (;;) {
                                const uint32_t i1 = i + parts;
                                if (i1 < ng) load_group(fb, i1);
                                if (!screen_group(fa, i) || i1 >= ng) break;
                                const uint32_t i2 = i1 + parts;
                                if (i2 < ng) load_group(fa, i2);
                                if (!screen_group(fb, i1) || i2 >= ng) break;
                                i = i2;
                            }
                        }
                    } else {
                        (void)fb;
                        for (; i < ng; i += parts) {
                            load_group(fa, i);
                            if (!screen_group(fa, i)) break;
                        }
                    }
                }
                if (diag == 0u || __ballot(alive) == 0ull) break;
                const int j = __ffs(diag) - 1;
                x = morton_dec((x & ~s_low[j]) | (root & s_low[j]), s_mask[j]);
                r = wuniform64(rec[x]);
                const uint32_t lowm = (2u << j) - 1u;
                diag = (diag & ~lowm) | (rec_nbr(r) & lowm);
            }
        }
    }

    if (stats != nullptr && lane == 0) {
        atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_CELL_VISITS], (unsigned long long)visits);
        atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PAIR_TESTS], (unsigned long long)tests);
    }
}

// Items a wave takes per atomic (SKYCELL_WAVE_CHUNK overrides it for sweeps).
static uint32_t wave_chunk()
{
    static int chunk = -1;
    if (chunk < 0) {
        const char *v = getenv("SKYCELL_WAVE_CHUNK");
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
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_refine_wave<D>, kWaveThreads, 0) != hipSuccess || b < 1)
            b = 1;
        blocks_per_cu = b;
    }
    return blocks_per_cu;
}

// Workgroups of a launch: the resident limit of the chip, or fewer when the
// work units cannot use them.  A cell with m points gives ceil(m / 63) items,
// so there are at most min(n, cells) + n / 63 items and `parts` units per item,
// and a workgroup runs kWaveThreads / 64 units at a time.
template <int D>
static unsigned wave_blocks(int64_t n, const GridDesc &gd, int num_cus)
{
    const uint64_t full = (uint64_t)num_cus * (uint64_t)wave_blocks_per_cu<D>();
    const uint64_t nn = (uint64_t)(n > 0 ? n : 1);
    const uint64_t items = (nn < gd.cells ? nn : (uint64_t)gd.cells) + (nn + kWaveItemPoints - 1) / kWaveItemPoints;
    const uint64_t waves = items * (uint64_t)gd.parts;
    const uint64_t per_block = kWaveThreads / 64;
    const uint64_t need = (waves + per_block - 1) / per_block;
    return (unsigned)(need < full ? need : full);
}

template <int D>
static hipError_t launch_wave_d(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                                hipStream_t st)
{
    const unsigned blocks = wave_blocks<D>(n, gd, num_cus);
    hipLaunchKernelGGL(k_refine_wave<D>, dim3(blocks), dim3(kWaveThreads), 0, st, (const uint32_t *)ws.keys,
                       (const uint64_t *)ws.fkeys, (const int32_t *)ws.sidx, (const uint64_t *)ws.rec,
                       (const uint2 *)ws.items, ws.ctr, ws.flag, stats, gd, wave_chunk());
    return hipGetLastError();
}

#define SKYCELL_WAVE_EACH_D(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t refine_wave_prepare(const GridDesc &gd)
{
    (void)wave_chunk();
    switch (gd.d) {
#define SKYCELL_WAVE_PREP(DD)           \
    case DD:                            \
        (void)wave_blocks_per_cu<DD>(); \
        return hipSuccess;
        SKYCELL_WAVE_EACH_D(SKYCELL_WAVE_PREP)
#undef SKYCELL_WAVE_PREP
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_refine_wave(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats, int num_cus,
                              hipStream_t st)
{
    switch (gd.d) {
#define SKYCELL_WAVE_LAUNCH(DD) \
    case DD:                    \
        return launch_wave_d<DD>(n, gd, ws, stats, num_cus, st);
        SKYCELL_WAVE_EACH_D(SKYCELL_WAVE_LAUNCH)
#undef SKYCELL_WAVE_LAUNCH
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace skycell
