// Pivot pre-filter of the learned path.
//
//   top-k   the k points with the largest scores, largest first, equal scores
//           by ascending index: an exact radix selection of the k-th largest
//           order-preserving score key (three digit passes, largest digit
//           first), then, among the points holding exactly that key, of the
//           index cut (three passes, smallest first), one selection pass and a
//           one-workgroup bitonic sort of the k selected (key, index) pairs;
//   gather  the pivots' exact keys and packed screening columns;
//   gate    a sample of 2^14 points is screened first; the full pass runs only
//           when pivots remove at least 1% of the sampled points of
//           surviving cells (otherwise the pass only counts the points again;
//           the plain path is the fallback and the result is the same);
//   prune   every point of a surviving cell (Definition 3) is tested against
//           the pivots; a pivot v that dominates it (Definition 1) removes it
//           from the refine, as a query and as a candidate.  The skyline is
//           unchanged: a removed point is not a skyline point, and whatever it
//           dominates is also dominated by v (dominance is transitive), so
//           every remaining point keeps an undominated dominator in its lower
//           cone.  The kept points of each surviving cell are counted again,
//           which gives them their slots in the counting sort.
#include "cellops.h"
#include "common.h"
#include "mlp.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kTopkThreads = 256;
constexpr int kDigitBins = 2048;

// state words
enum TopkState {
    kStPrefix = 0,   // key digits fixed so far
    kStMask = 1,     // which key bits are fixed
    kStNeed = 2,     // rank still wanted among the keys that match the prefix
    kStIPrefix = 3,  // index digits fixed so far (tie pass)
    kStIMask = 4,
    kStDone = 5,     // tie pass not needed: take every point with the cut key
    kStCount = 6,    // selected so far
    kStK = 7,
};

__device__ __forceinline__ uint32_t score_key(float s) { return f32_key(s); }

// Digit passes: pass 0..2 over the score key (bits 31..21, 20..10, 9..0),
// pass 3..5 over the index (bits 30..20, 19..10, 9..0) of the points whose key
// equals the cut.
__host__ __device__ constexpr int digit_shift(int pass)
{
    return pass == 0 ? 21 : pass == 1 ? 10 : pass == 2 ? 0 : pass == 3 ? 20 : pass == 4 ? 10 : 0;
}
__host__ __device__ constexpr uint32_t digit_bits(int pass)
{
    return pass == 0 ? 11u : pass == 1 ? 11u : pass == 2 ? 10u : pass == 3 ? 11u : 10u;
}

__global__ __launch_bounds__(kTopkThreads) void k_topk_hist(const float *__restrict__ scores, uint32_t n,
                                                            const uint32_t *__restrict__ state, int pass,
                                                            uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_h[kDigitBins];
    if (pass >= 3 && state[kStDone]) return;
    for (int b = threadIdx.x; b < kDigitBins; b += kTopkThreads) s_h[b] = 0u;
    __syncthreads();
    const uint32_t prefix = state[kStPrefix], mask = state[kStMask];
    const uint32_t iprefix = state[kStIPrefix], imask = state[kStIMask];
    const int shift = digit_shift(pass);
    const uint32_t dmask = (1u << digit_bits(pass)) - 1u;
    for (uint32_t i = blockIdx.x * kTopkThreads + threadIdx.x; i < n; i += gridDim.x * kTopkThreads) {
        const uint32_t key = score_key(scores[i]);
        if ((key & mask) != prefix) continue;
        if (pass < 3) {
            atomicAdd(&s_h[(key >> shift) & dmask], 1u);
        } else if ((i & imask) == iprefix) {
            atomicAdd(&s_h[(i >> shift) & dmask], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kDigitBins; b += kTopkThreads)
        if (s_h[b]) atomicAdd(&hist[b], s_h[b]);
}

// One thread: the digit holding the wanted rank (largest digits first for the
// key, smallest first for the index), then the histogram is cleared.
__global__ __launch_bounds__(kTopkThreads) void k_topk_pick(uint32_t *__restrict__ hist,
                                                            uint32_t *__restrict__ state, int pass)
{
    const bool skip = pass >= 3 && state[kStDone];
    const int nb = 1 << digit_bits(pass);
    if (threadIdx.x == 0 && !skip) {
        uint32_t need = state[kStNeed];
        const int shift = digit_shift(pass);
        int pick = -1;
        uint32_t at = 0u;
        for (int j = 0; j < nb; ++j) {
            const int b = pass < 3 ? nb - 1 - j : j;
            const uint32_t c = hist[b];
            if (need <= c) {
                pick = b;
                at = c;
                break;
            }
            need -= c;
        }
        if (pick < 0) pick = pass < 3 ? 0 : nb - 1;  // unreachable when need <= matching points
        if (pass < 3) {
            state[kStPrefix] |= (uint32_t)pick << shift;
            state[kStMask] |= (uint32_t)(nb - 1) << shift;
            if (pass == 2) state[kStDone] = need == at ? 1u : 0u;
        } else {
            state[kStIPrefix] |= (uint32_t)pick << shift;
            state[kStIMask] |= (uint32_t)(nb - 1) << shift;
        }
        state[kStNeed] = need;
    }
    __syncthreads();
    if (!skip)
        for (int b = threadIdx.x; b < nb; b += kTopkThreads) hist[b] = 0u;
}

__global__ void k_topk_init(uint32_t *__restrict__ hist, uint32_t *__restrict__ state, uint32_t k)
{
    for (int b = threadIdx.x; b < kDigitBins; b += blockDim.x) hist[b] = 0u;
    if (threadIdx.x < 16) state[threadIdx.x] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        state[kStNeed] = k;
        state[kStK] = k;
    }
}

// Keys above the cut, and keys equal to it up to the index cut.
__global__ __launch_bounds__(kTopkThreads) void k_topk_select(const float *__restrict__ scores, uint32_t n,
                                                              uint32_t *__restrict__ state,
                                                              uint64_t *__restrict__ sel)
{
    const uint32_t cut = state[kStPrefix];
    const bool all_ties = state[kStDone] != 0u;
    const uint32_t icut = state[kStIPrefix];
    const uint32_t k = state[kStK];
    for (uint32_t i = blockIdx.x * kTopkThreads + threadIdx.x; i < n; i += gridDim.x * kTopkThreads) {
        const uint32_t key = score_key(scores[i]);
        const bool take = key > cut || (key == cut && (all_ties || i <= icut));
        if (take) {
            const uint32_t slot = atomicAdd(&state[kStCount], 1u);
            if (slot < k) sel[slot] = ((uint64_t)(~key) << 32) | i;
        }
    }
}

constexpr int kSortThreads = 1024;

// Ascending bitonic sort of the k selected pairs (inverted key, index): the
// best score first, equal scores by index.
__global__ __launch_bounds__(kSortThreads) void k_topk_sort(const uint64_t *__restrict__ sel, uint32_t k,
                                                            int32_t *__restrict__ out_idx)
{
    __shared__ uint64_t s[kMaxPivots];
    uint32_t np = 1u;
    while (np < k) np <<= 1;
    for (uint32_t j = threadIdx.x; j < np; j += kSortThreads) s[j] = j < k ? sel[j] : ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= np; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t j = threadIdx.x; j < np; j += kSortThreads) {
                const uint32_t partner = j ^ stride;
                if (partner > j) {
                    const bool up = (j & size) == 0u;
                    const uint64_t a = s[j], b = s[partner];
                    if ((a > b) == up) {
                        s[j] = b;
                        s[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t j = threadIdx.x; j < k; j += kSortThreads) out_idx[j] = (int32_t)(uint32_t)s[j];
}

static inline dim3 stream_blocks(uint32_t n)
{
    uint64_t b = ((uint64_t)n + kTopkThreads * 8 - 1) / (kTopkThreads * 8);
    if (b > 2048) b = 2048;
    return dim3((unsigned)(b ? b : 1));
}

hipError_t launch_topk(const float *scores, uint32_t n, uint32_t k, int32_t *out_idx, const PivotScratch &ps,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, ps.hist, ps.state, k);
    for (int pass = 0; pass < 6; ++pass) {
        hipLaunchKernelGGL(k_topk_hist, stream_blocks(n), dim3(kTopkThreads), 0, st, scores, n,
                           (const uint32_t *)ps.state, pass, ps.hist);
        hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(kTopkThreads), 0, st, ps.hist, ps.state, pass);
    }
    hipLaunchKernelGGL(k_topk_select, stream_blocks(n), dim3(kTopkThreads), 0, st, scores, n, ps.state, ps.sel);
    hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(kSortThreads), 0, st, (const uint64_t *)ps.sel, k, out_idx);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pivot table
__global__ void k_pivot_gather(const float *__restrict__ pts, uint32_t n, int d,
                               const int32_t *__restrict__ idx, uint32_t k, uint32_t *__restrict__ pkeys,
                               uint64_t *__restrict__ pfine, uint32_t *__restrict__ ctr)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const int32_t i = idx[j];
    const int fw = fine_words(d);
    if (i < 0 || (uint32_t)i >= n) {
        // reported as SKYCELL_E_RANGE by the output stage; the entry can
        // dominate nothing (no finite key reaches ~0u)
        atomicOr(&ctr[kCtrErr], 2u);
        for (int t = 0; t < d; ++t) pkeys[(size_t)j * d + t] = ~0u;
        for (int w = 0; w < fw; ++w) pfine[(size_t)j * fw + w] = 0x7F7F7F7F7F7F7F7Full;
        return;
    }
    uint64_t word = 0ull;
    bool nan = false;
    for (int t = 0; t < d; ++t) {
        const float v = pts[(size_t)t * n + (uint32_t)i];
        pkeys[(size_t)j * d + t] = f32_key(v);
        word |= (uint64_t)column_f32(v, (float)kFineCols, (uint32_t)kFineCols, nan) << (8 * (t & 7));
        if ((t & 7) == 7 || t == d - 1) {
            pfine[(size_t)j * fw + (t >> 3)] = word;
            word = 0ull;
        }
    }
}

hipError_t launch_pivot_gather(const float *pts, uint32_t n, int d, const int32_t *idx, uint32_t k,
                               const PivotScratch &ps, uint32_t *ctr, hipStream_t st)
{
    if (k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pivot_gather, dim3((k + 255) / 256), dim3(256), 0, st, pts, n, d, idx, k, ps.pkeys,
                       ps.pfine, ctr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ prune
constexpr int kPruneThreads = 256;
constexpr int kPivotChunk = 1024;
constexpr uint32_t kPivotSample = 16384;  // points screened by the gate of the pre-filter

__global__ void k_zero_u32(uint32_t *__restrict__ p, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Screening words (query side, top bits set, padding 0x7F) and exact keys of
// point i.
template <int D>
__device__ __forceinline__ void query_words(const float *__restrict__ pts, uint32_t n, uint32_t i,
                                            uint32_t (&qk)[D], uint64_t (&qh)[fine_words(D)])
{
    constexpr int FW = fine_words(D);
    constexpr uint64_t H = 0x8080808080808080ull;
    bool nan = false;
#pragma unroll
    for (int w = 0; w < FW; ++w) qh[w] = 0ull;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const float v = pts[(size_t)t * n + i];
        qk[t] = f32_key(v);
        qh[t >> 3] |= (uint64_t)column_f32(v, (float)kFineCols, (uint32_t)kFineCols, nan) << (8 * (t & 7));
    }
#pragma unroll
    for (int t = D; t < 8 * FW; ++t) qh[t >> 3] |= 0x7Full << (8 * (t & 7));
#pragma unroll
    for (int w = 0; w < FW; ++w) qh[w] |= H;
}

// Whether some pivot dominates the calling thread's point (Definition 1),
// scanning the pivots in chunks staged through LDS by the whole workgroup.
// Every thread of the workgroup must call it (alive = false for threads
// without a point); the workgroup leaves early once no thread is alive.
template <int D>
__device__ __forceinline__ bool dominated_by_pivot(bool alive, const uint32_t (&qk)[D],
                                                   const uint64_t (&qh)[fine_words(D)],
                                                   const uint32_t *__restrict__ pkeys,
                                                   const uint64_t *__restrict__ pfine, uint32_t k,
                                                   uint64_t *s_f)
{
    constexpr int FW = fine_words(D);
    constexpr uint64_t H = 0x8080808080808080ull, L1 = 0x0101010101010101ull;
    bool removed = false;
    for (uint32_t base = 0; base < k; base += kPivotChunk) {
        if (__syncthreads_or(alive) == 0) break;
        const uint32_t cnt_c = k - base < (uint32_t)kPivotChunk ? k - base : (uint32_t)kPivotChunk;
        for (uint32_t j = threadIdx.x; j < cnt_c * FW; j += kPruneThreads) s_f[j] = pfine[(size_t)base * FW + j];
        __syncthreads();
        if (alive) {
            for (uint32_t j = 0; j < cnt_c; ++j) {
                bool le = true, lt = true;
#pragma unroll
                for (int w = 0; w < FW; ++w) {
                    const uint64_t diff = qh[w] - s_f[j * FW + w];
                    le &= (diff & H) == H;
                    lt &= ((diff - L1) & H) == H;
                }
                if (!le) continue;
                bool dom = lt;
                if (!dom) {
                    const uint32_t *pk = pkeys + (size_t)(base + j) * D;
                    bool all_le = true, any_lt = false;
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const uint32_t a = pk[t];
                        all_le &= a <= qk[t];
                        any_lt |= a < qk[t];
                    }
                    dom = all_le && any_lt;
                }
                if (dom) {
                    removed = true;
                    break;
                }
            }
            if (removed) alive = false;
        }
        __syncthreads();
    }
    return removed;
}

// Gate of the pre-filter: a sample of the points (every stride-th) of
// surviving cells is screened against the pivots; the full pass below runs
// only when pivots remove at least 1 in 100 of them.
template <int D>
__global__ __launch_bounds__(kPruneThreads) void k_pivot_sample(const float *__restrict__ pts, uint32_t n,
                                                                uint32_t stride, uint32_t nsample,
                                                                const uint32_t *__restrict__ cell_of,
                                                                const uint64_t *__restrict__ rec,
                                                                const uint32_t *__restrict__ pkeys,
                                                                const uint64_t *__restrict__ pfine, uint32_t k,
                                                                uint32_t *__restrict__ ctr)
{
    __shared__ uint64_t s_f[kPivotChunk * fine_words(D)];
    const uint32_t j = blockIdx.x * kPruneThreads + threadIdx.x;
    const uint32_t i = j * stride;
    bool cand = false;
    if (j < nsample && i < n) cand = rec_surv(rec[cell_of[i]]);
    uint32_t qk[D];
    uint64_t qh[fine_words(D)];
    if (cand) query_words<D>(pts, n, i, qk, qh);
    const bool removed = dominated_by_pivot<D>(cand, qk, qh, pkeys, pfine, k, s_f);
    const uint64_t bc = __ballot(cand), br = __ballot(removed);
    if (__lane_id() == 0) {
        if (bc) atomicAdd(&ctr[kCtrPivSampled], (uint32_t)__popcll(bc));
        if (br) atomicAdd(&ctr[kCtrPivHit], (uint32_t)__popcll(br));
    }
}

template <int D>
__global__ __launch_bounds__(kPruneThreads) void k_pivot_prune(const float *__restrict__ pts, uint32_t n,
                                                               const uint32_t *__restrict__ cell_of,
                                                               const uint64_t *__restrict__ rec,
                                                               const uint32_t *__restrict__ pkeys,
                                                               const uint64_t *__restrict__ pfine, uint32_t k,
                                                               uint32_t *__restrict__ rank,
                                                               uint32_t *__restrict__ cnt,
                                                               const uint32_t *__restrict__ ctr,
                                                               uint64_t *__restrict__ stats, int gated)
{
    __shared__ uint64_t s_f[kPivotChunk * fine_words(D)];
    const uint32_t i = blockIdx.x * kPruneThreads + threadIdx.x;
    // the sample decides for the whole grid (the same value in every thread);
    // without the gate every point of a surviving cell is screened
    const bool use = !gated || (uint64_t)ctr[kCtrPivHit] * 100u >= (uint64_t)ctr[kCtrPivSampled];
    uint32_t x = 0u;
    bool cand = false;
    if (i < n) {
        x = cell_of[i];
        cand = rec_surv(rec[x]);
    }
    uint32_t qk[D];
    uint64_t qh[fine_words(D)];
    if (cand && use) query_words<D>(pts, n, i, qk, qh);
    const bool removed = use ? dominated_by_pivot<D>(cand, qk, qh, pkeys, pfine, k, s_f) : false;
    if (cand) rank[i] = removed ? kRankRemoved : atomicAdd(&cnt[x], 1u);
    if (stats != nullptr) {
        const uint64_t b = __ballot(removed);
        if (__lane_id() == 0 && b)
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_PIVOT_REMOVED], (unsigned long long)__popcll(b));
    }
}

hipError_t launch_pivot_prune(const float *pts, uint32_t n, const GridDesc &gd, const Workspace &ws,
                              const PivotScratch &ps, uint32_t k, uint64_t *stats, bool gated, hipStream_t st)
{
    unsigned zb = (gd.cells + 255u) / 256u;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_zero_u32, dim3(zb ? zb : 1), dim3(256), 0, st, ws.cnt, gd.cells);
    const uint32_t nsample = n < kPivotSample ? n : kPivotSample;
    const uint32_t stride = n / nsample;
    const dim3 sgrid((nsample + kPruneThreads - 1) / kPruneThreads);
    const dim3 grid((n + kPruneThreads - 1) / kPruneThreads);
    switch (gd.d) {
#define SKYCELL_PRUNE_CASE(DD)                                                                                  \
    case DD:                                                                                                    \
        if (gated)                                                                                              \
            hipLaunchKernelGGL(k_pivot_sample<DD>, sgrid, dim3(kPruneThreads), 0, st, pts, n, stride, nsample,  \
                               (const uint32_t *)ws.cell_of, (const uint64_t *)ws.rec,                          \
                               (const uint32_t *)ps.pkeys, (const uint64_t *)ps.pfine, k, ws.ctr);              \
        hipLaunchKernelGGL(k_pivot_prune<DD>, grid, dim3(kPruneThreads), 0, st, pts, n,                         \
                           (const uint32_t *)ws.cell_of, (const uint64_t *)ws.rec, (const uint32_t *)ps.pkeys,  \
                           (const uint64_t *)ps.pfine, k, ws.rank, ws.cnt, (const uint32_t *)ws.ctr, stats,    \
                           gated ? 1 : 0);                                                                      \
        break;
        SKYCELL_PRUNE_CASE(1)
        SKYCELL_PRUNE_CASE(2)
        SKYCELL_PRUNE_CASE(3)
        SKYCELL_PRUNE_CASE(4)
        SKYCELL_PRUNE_CASE(5)
        SKYCELL_PRUNE_CASE(6)
        SKYCELL_PRUNE_CASE(7)
        SKYCELL_PRUNE_CASE(8)
        SKYCELL_PRUNE_CASE(9)
        SKYCELL_PRUNE_CASE(10)
        SKYCELL_PRUNE_CASE(11)
        SKYCELL_PRUNE_CASE(12)
        SKYCELL_PRUNE_CASE(13)
        SKYCELL_PRUNE_CASE(14)
        SKYCELL_PRUNE_CASE(15)
        SKYCELL_PRUNE_CASE(16)
#undef SKYCELL_PRUNE_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t pivot_scratch_layout(PivotScratch *ps, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return base ? base + o : nullptr;
    };
    char *h = take(kDigitBins * 4);
    char *s = take(16 * 4);
    char *se = take((size_t)kMaxPivots * 8);
    char *ix = take((size_t)kMaxPivots * 4);
    char *pk = take((size_t)kMaxPivots * kMaxD * 4);
    char *pf = take((size_t)kMaxPivots * 2 * 8);
    if (ps) {
        ps->hist = (uint32_t *)h;
        ps->state = (uint32_t *)s;
        ps->sel = (uint64_t *)se;
        ps->idx = (int32_t *)ix;
        ps->pkeys = (uint32_t *)pk;
        ps->pfine = (uint64_t *)pf;
    }
    return off;
}

}  // namespace skycell
