// Incremental skyline maintenance under inserts and deletes.
//
// The paper argues (Section I, and Section VII-B3 on dynamic data) that SkyCell
// needs no pre-computation, so it stays applicable when points are inserted and
// deleted.  This module keeps a point set resident in HBM together with its
// skyline flags and, after each batch of updates, recomputes only what the
// batch can change, with the exact single-instance path:
//
//   insert B:  a point that some live point dominates stays dominated when
//              points are added, so sky(P + B) = sky(S + B), S = sky(P);
//   delete D:  only deleted skyline points D_S can release other points, and
//              only points they dominate (or equal): with
//              R = { p live, p not in S : some v in D_S has v <= p },
//              sky(P - D) = sky((S - D) + R).  A point outside S and R keeps a
//              dominator in S - D (its old dominator s in S was not deleted,
//              else p would be in R).
//
// Each update compacts the affected ids (ascending), gathers their points into
// a contiguous SoA block, runs the whole path on it and writes the verdicts
// back into the flags.  Point ids are insertion positions; deleted ids are
// never reused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/skycell.h"
#include "common.h"
#include "host_internal.h"
#include "scan.h"

namespace skycell {

constexpr int kDynThreads = 256;
// deleted skyline points screened per LDS chunk by the release test
constexpr int kDynChunk = 256;
// Above this many (live point, deleted skyline point) pairs the release test
// costs more than recomputing every live point, which is done instead.
constexpr double kDynPairBudget = 2.0e10;

static inline dim3 dyn_grid(uint64_t count)
{
    uint64_t b = (count + kDynThreads - 1) / kDynThreads;
    return dim3((unsigned)(b ? b : 1));
}

// Comparable key of one coordinate: order-preserving u32 for binary32 (with
// -0.0 equal to +0.0), the value itself for uint16.
__device__ __forceinline__ uint32_t dyn_key(const float *p, size_t i) { return f32_key(p[i]); }
__device__ __forceinline__ uint32_t dyn_key(const uint16_t *p, size_t i) { return (uint32_t)p[i]; }

// Copy a batch [d][m] into the store at ids first..first+m-1, mark them live,
// and flag a NaN.
template <typename T>
__global__ __launch_bounds__(kDynThreads) void k_dyn_append(const T *__restrict__ in, int64_t m, int d,
                                                            T *__restrict__ pts, int64_t cap, int64_t first,
                                                            uint8_t *__restrict__ alive, uint8_t *__restrict__ sky,
                                                            uint32_t *__restrict__ ctr)
{
    const int64_t j = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    if (j >= m) return;
    bool nan = false;
    for (int k = 0; k < d; ++k) {
        const T v = in[(size_t)k * m + j];
        if constexpr (sizeof(T) == 4) nan |= (v != v);
        pts[(size_t)k * cap + first + j] = v;
    }
    alive[first + j] = 1;
    sky[first + j] = 0;
    if (nan) atomicOr(&ctr[0], 1u);
}

// Candidates of an insert: the current skyline and the new ids.
__global__ __launch_bounds__(kDynThreads) void k_dyn_cand_insert(const uint8_t *__restrict__ sky, int64_t first,
                                                                 int64_t total, uint8_t *__restrict__ cand)
{
    const int64_t i = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    if (i >= total) return;
    cand[i] = (sky[i] || i >= first) ? 1 : 0;
}

// Deletes: a live id becomes dead; a deleted skyline point is copied (as keys)
// into `dels` for the release test.  Ids out of range raise bit 1 of ctr[0].
template <typename T>
__global__ __launch_bounds__(kDynThreads) void k_dyn_delete(const int32_t *__restrict__ ids, int64_t m,
                                                            int64_t count, const T *__restrict__ pts, int64_t cap,
                                                            int d, uint8_t *__restrict__ alive,
                                                            uint8_t *__restrict__ sky, uint32_t *__restrict__ dels,
                                                            uint32_t *__restrict__ ctr)
{
    const int64_t j = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    if (j >= m) return;
    const int64_t id = ids[j];
    if (id < 0 || id >= count) {
        atomicOr(&ctr[0], 2u);
        return;
    }
    // an id repeated in the batch may be taken twice: both copies of its keys
    // then go into `dels`, which changes nothing
    if (!alive[id]) return;
    alive[id] = 0;
    if (sky[id]) {
        sky[id] = 0;
        const uint32_t slot = atomicAdd(&ctr[1], 1u);
        for (int k = 0; k < d; ++k) dels[(size_t)slot * d + k] = dyn_key(pts, (size_t)k * cap + id);
    }
}

// Candidates of a delete: live skyline points, and live non-skyline points that
// some deleted skyline point is <= in every dimension (the points it may have
// been the only dominator of).  `full` makes every live point a candidate.
template <typename T, int D>
__global__ __launch_bounds__(kDynThreads) void k_dyn_cand_delete(const T *__restrict__ pts, int64_t cap,
                                                                 int64_t count, const uint8_t *__restrict__ alive,
                                                                 const uint8_t *__restrict__ sky,
                                                                 const uint32_t *__restrict__ dels,
                                                                 const uint32_t *__restrict__ ctr, int full,
                                                                 uint8_t *__restrict__ cand)
{
    __shared__ uint32_t s_del[kDynChunk * D];
    const int64_t i = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    const bool in = i < count;
    const bool live = in && alive[i];
    bool c = live && (sky[i] || full);
    bool test = live && !c;
    uint32_t q[D];
    if (test)
        for (int k = 0; k < D; ++k) q[k] = dyn_key(pts, (size_t)k * cap + i);
    const uint32_t nd = full ? 0u : ctr[1];
    for (uint32_t c0 = 0; c0 < nd; c0 += kDynChunk) {
        const uint32_t len = nd - c0 < (uint32_t)kDynChunk ? nd - c0 : (uint32_t)kDynChunk;
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < len * D; e += kDynThreads) s_del[e] = dels[(size_t)c0 * D + e];
        __syncthreads();
        if (__ballot(test) == 0ull) continue;
        if (test) {
            for (uint32_t j = 0; j < len; ++j) {
                uint32_t gt = 0u;
#pragma unroll
                for (int k = 0; k < D; ++k) gt |= s_del[j * D + k] > q[k] ? 1u : 0u;
                if (gt == 0u) {
                    c = true;
                    test = false;
                    break;
                }
            }
        }
    }
    if (in) cand[i] = c ? 1 : 0;
}

struct DynFlagLoader {
    const uint8_t *flag;
    __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)flag[i]; }
};

struct DynFlagEmitter {
    int32_t *out;
    __device__ void operator()(uint64_t i, uint32_t prefix, uint32_t v) const
    {
        if (v) out[prefix] = (int32_t)i;
    }
};

__global__ void k_dyn_zero(uint32_t *ctr)
{
    if (threadIdx.x < 16) ctr[threadIdx.x] = 0u;
}

__global__ void k_dyn_total(const uint64_t *block_sums, uint32_t nb, int32_t *out)
{
    *out = (int32_t)block_sums[nb];
}

// Gather the candidates' coordinates into a contiguous [d][k] block; clear
// their skyline flags (the recompute decides them again).
template <typename T>
__global__ __launch_bounds__(kDynThreads) void k_dyn_gather(const T *__restrict__ pts, int64_t cap, int d,
                                                            const int32_t *__restrict__ ids, int64_t k,
                                                            T *__restrict__ out, uint8_t *__restrict__ sky)
{
    const int64_t j = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    if (j >= k) return;
    const int64_t id = ids[j];
    for (int kk = 0; kk < d; ++kk) out[(size_t)kk * k + j] = pts[(size_t)kk * cap + id];
    sky[id] = 0;
}

// Write the recompute's verdicts back: local index t of the block is id ids[t].
__global__ __launch_bounds__(kDynThreads) void k_dyn_apply(const int32_t *__restrict__ local,
                                                           const int32_t *__restrict__ nres,
                                                           const int32_t *__restrict__ ids,
                                                           uint8_t *__restrict__ sky)
{
    const int64_t j = (int64_t)blockIdx.x * kDynThreads + threadIdx.x;
    const int32_t n = *nres;
    if (j >= n) return;
    sky[ids[local[j]]] = 1;
}

}  // namespace skycell

using namespace skycell;

struct skycell_dyn {
    int dev = 0;
    int d = 0;
    int dtype = SKYCELL_DTYPE_F32;
    int value_bits = 16;
    int64_t cap = 0;
    int64_t count = 0;   // ids handed out so far
    size_t esize = 4;
    void *pts = nullptr;       // [d][cap]
    uint8_t *alive = nullptr;  // [cap]
    uint8_t *sky = nullptr;    // [cap]
    uint8_t *cand = nullptr;   // [cap]
    int32_t *ids = nullptr;    // [cap] compacted candidate ids
    int32_t *local = nullptr;  // [cap] skyline of the gathered block (local indices)
    void *block = nullptr;     // [d][cap] gathered candidates
    uint64_t *sums = nullptr;  // scan partials
    uint32_t *ctr = nullptr;   // [16]: 0 error bits, 1 deleted skyline points
    int32_t *counts = nullptr; // [2]: candidates, recompute result
    uint32_t *dels = nullptr;  // [dcap][d] keys of deleted skyline points
    int64_t dcap = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t last_candidates = 0;
    std::mutex mu;
};

static void dyn_free(skycell_dyn *h)
{
    void *bufs[] = {h->pts, h->alive, h->sky, h->cand, h->ids, h->local, h->block, h->sums, h->ctr,
                    h->counts, h->dels, h->ws};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

int skycell_dyn_create(int32_t d, int32_t dtype, int64_t capacity, int32_t value_bits, skycell_dyn_t *out)
{
    if (out == nullptr) return set_error(SKYCELL_E_INVAL, "handle pointer is NULL");
    *out = nullptr;
    if (d < 1 || d > SKYCELL_MAX_D) return set_error(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (capacity < 1 || capacity >= (int64_t)1 << 31)
        return set_error(SKYCELL_E_INVAL, "capacity = %lld is outside [1, 2^31)", (long long)capacity);
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return set_error(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (dtype == SKYCELL_DTYPE_U16 && (value_bits < 1 || value_bits > 16))
        return set_error(SKYCELL_E_INVAL, "value_bits = %d is outside [1, 16]", value_bits);
    skycell_dyn *h = new (std::nothrow) skycell_dyn;
    if (h == nullptr) return set_error(SKYCELL_E_NOMEM, "out of host memory");
    h->d = d;
    h->cap = capacity;
    h->dtype = dtype;
    h->value_bits = dtype == SKYCELL_DTYPE_U16 ? value_bits : 16;
    h->esize = dtype == SKYCELL_DTYPE_F32 ? 4 : 2;
    hipError_t e = hipGetDevice(&h->dev);
    const size_t cap = (size_t)capacity;
    if (e == hipSuccess) e = hipMalloc(&h->pts, cap * d * h->esize);
    if (e == hipSuccess) e = hipMalloc(&h->block, cap * d * h->esize);
    if (e == hipSuccess) e = hipMalloc((void **)&h->alive, cap);
    if (e == hipSuccess) e = hipMalloc((void **)&h->sky, cap);
    if (e == hipSuccess) e = hipMalloc((void **)&h->cand, cap);
    if (e == hipSuccess) e = hipMalloc((void **)&h->ids, cap * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->local, cap * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->sums, ((size_t)scan_tiles(cap) + 1) * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&h->ctr, 16 * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->counts, 2 * 4);
    if (e != hipSuccess) {
        dyn_free(h);
        delete h;
        return set_error(e == hipErrorOutOfMemory ? SKYCELL_E_NOMEM : SKYCELL_E_HIP, "allocation failed: %s",
                         hipGetErrorString(e));
    }
    *out = h;
    return clear_error();
}

int skycell_dyn_destroy(skycell_dyn_t h)
{
    if (h == nullptr) return clear_error();
    (void)hipDeviceSynchronize();
    dyn_free(h);
    delete h;
    return clear_error();
}

int skycell_dyn_size(skycell_dyn_t h, int64_t *ids_used, int64_t *last_candidates)
{
    if (h == nullptr) return set_error(SKYCELL_E_INVAL, "handle is NULL");
    if (ids_used) *ids_used = h->count;
    if (last_candidates) *last_candidates = h->last_candidates;
    return clear_error();
}

// Compact cand[0..total) into h->ids, gather, recompute, apply.  Synchronises
// twice (candidate count, then the recompute's status).
static int dyn_recompute(skycell_dyn *h, int64_t total, hipStream_t st)
{
    DynFlagLoader ld{h->cand};
    DynFlagEmitter em{h->ids};
    SKYCELL_HIP_CHECK((enqueue_scan<uint32_t>(ld, em, (uint64_t)total, h->sums, st)));
    hipLaunchKernelGGL(k_dyn_total, dim3(1), dim3(1), 0, st, (const uint64_t *)h->sums,
                       scan_tiles((uint64_t)total), h->counts);
    SKYCELL_HIP_CHECK(hipGetLastError());
    int32_t k32 = 0;
    SKYCELL_HIP_CHECK(hipMemcpyAsync(&k32, h->counts, 4, hipMemcpyDeviceToHost, st));
    SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
    const int64_t k = k32;
    h->last_candidates = k;
    if (k == 0) return SKYCELL_OK;
    if (h->dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_dyn_gather<float>, dyn_grid(k), dim3(kDynThreads), 0, st, (const float *)h->pts, h->cap,
                           h->d, (const int32_t *)h->ids, k, (float *)h->block, h->sky);
    else
        hipLaunchKernelGGL(k_dyn_gather<uint16_t>, dyn_grid(k), dim3(kDynThreads), 0, st, (const uint16_t *)h->pts,
                           h->cap, h->d, (const int32_t *)h->ids, k, (uint16_t *)h->block, h->sky);
    SKYCELL_HIP_CHECK(hipGetLastError());
    int g = 0;
    int rc = resolve_grid(k, h->d, h->dtype, 0, &g);
    if (rc != SKYCELL_OK) return rc;
    const size_t need = workspace_layout(k, h->d, grid_desc(h->d, g).cells, nullptr, nullptr);
    if (need > h->ws_bytes) {
        SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
        if (h->ws) SKYCELL_HIP_CHECK(hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
        const size_t grow = need + need / 4;
        if (hipMalloc(&h->ws, grow) != hipSuccess) {
            h->ws = nullptr;
            return set_error(SKYCELL_E_NOMEM, "hipMalloc of %zu workspace bytes failed", grow);
        }
        h->ws_bytes = grow;
    }
    rc = run_pipeline(h->block, h->dtype, k, h->d, g, h->value_bits, h->local, h->counts + 1, h->ws, nullptr, st);
    if (rc != SKYCELL_OK) return rc;
    hipLaunchKernelGGL(k_dyn_apply, dyn_grid(k), dim3(kDynThreads), 0, st, (const int32_t *)h->local,
                       (const int32_t *)(h->counts + 1), (const int32_t *)h->ids, h->sky);
    SKYCELL_HIP_CHECK(hipGetLastError());
    int32_t res = 0;
    SKYCELL_HIP_CHECK(hipMemcpyAsync(&res, h->counts + 1, 4, hipMemcpyDeviceToHost, st));
    SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
    if (res < 0) return set_error(res, "the recompute reported error %d", res);
    return SKYCELL_OK;
}

int skycell_dyn_insert(skycell_dyn_t h, const void *points, int64_t m, int64_t *first_id, void *stream)
{
    if (h == nullptr) return set_error(SKYCELL_E_INVAL, "handle is NULL");
    if (m < 0) return set_error(SKYCELL_E_INVAL, "m = %lld is negative", (long long)m);
    if (m > 0 && points == nullptr) return set_error(SKYCELL_E_INVAL, "points is NULL");
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->count + m > h->cap)
        return set_error(SKYCELL_E_NOMEM, "%lld ids used + %lld new exceed the capacity %lld", (long long)h->count,
                         (long long)m, (long long)h->cap);
    if (first_id) *first_id = h->count;
    if (m == 0) return clear_error();
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_dyn_zero, dim3(1), dim3(64), 0, st, h->ctr);
    if (h->dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_dyn_append<float>, dyn_grid(m), dim3(kDynThreads), 0, st, (const float *)points, m, h->d,
                           (float *)h->pts, h->cap, h->count, h->alive, h->sky, h->ctr);
    else
        hipLaunchKernelGGL(k_dyn_append<uint16_t>, dyn_grid(m), dim3(kDynThreads), 0, st, (const uint16_t *)points, m,
                           h->d, (uint16_t *)h->pts, h->cap, h->count, h->alive, h->sky, h->ctr);
    SKYCELL_HIP_CHECK(hipGetLastError());
    uint32_t err = 0;
    SKYCELL_HIP_CHECK(hipMemcpyAsync(&err, h->ctr, 4, hipMemcpyDeviceToHost, st));
    SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
    if (err & 1u) return set_error(SKYCELL_E_NAN, "the batch holds a NaN; nothing was inserted");
    const int64_t total = h->count + m;
    hipLaunchKernelGGL(k_dyn_cand_insert, dyn_grid(total), dim3(kDynThreads), 0, st, (const uint8_t *)h->sky,
                       h->count, total, h->cand);
    SKYCELL_HIP_CHECK(hipGetLastError());
    h->count = total;
    const int rc = dyn_recompute(h, total, st);
    return rc == SKYCELL_OK ? clear_error() : rc;
}

int skycell_dyn_delete(skycell_dyn_t h, const int32_t *ids, int64_t m, void *stream)
{
    if (h == nullptr) return set_error(SKYCELL_E_INVAL, "handle is NULL");
    if (m < 0) return set_error(SKYCELL_E_INVAL, "m = %lld is negative", (long long)m);
    if (m > 0 && ids == nullptr) return set_error(SKYCELL_E_INVAL, "ids is NULL");
    std::lock_guard<std::mutex> lk(h->mu);
    if (m == 0 || h->count == 0) return clear_error();
    hipStream_t st = (hipStream_t)stream;
    if (m > h->dcap) {
        SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
        if (h->dels) SKYCELL_HIP_CHECK(hipFree(h->dels));
        h->dels = nullptr;
        h->dcap = 0;
        if (hipMalloc((void **)&h->dels, (size_t)m * h->d * 4) != hipSuccess) {
            h->dels = nullptr;
            return set_error(SKYCELL_E_NOMEM, "hipMalloc for %lld deleted points failed", (long long)m);
        }
        h->dcap = m;
    }
    hipLaunchKernelGGL(k_dyn_zero, dim3(1), dim3(64), 0, st, h->ctr);
    if (h->dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_dyn_delete<float>, dyn_grid(m), dim3(kDynThreads), 0, st, ids, m, h->count,
                           (const float *)h->pts, h->cap, h->d, h->alive, h->sky, h->dels, h->ctr);
    else
        hipLaunchKernelGGL(k_dyn_delete<uint16_t>, dyn_grid(m), dim3(kDynThreads), 0, st, ids, m, h->count,
                           (const uint16_t *)h->pts, h->cap, h->d, h->alive, h->sky, h->dels, h->ctr);
    SKYCELL_HIP_CHECK(hipGetLastError());
    uint32_t c[2] = {0u, 0u};
    SKYCELL_HIP_CHECK(hipMemcpyAsync(c, h->ctr, 8, hipMemcpyDeviceToHost, st));
    SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
    // ids out of range are reported once the valid ones have been applied
    auto finish = [&](int rc) {
        if (rc != SKYCELL_OK) return rc;
        if (c[0] & 2u)
            return set_error(SKYCELL_E_RANGE, "an id is outside [0, %lld); the valid ids were deleted",
                             (long long)h->count);
        return clear_error();
    };
    if (c[1] == 0u) {
        h->last_candidates = 0;
        return finish(SKYCELL_OK);  // no skyline point was deleted: the skyline stands
    }
    const int full = (double)c[1] * (double)h->count > kDynPairBudget ? 1 : 0;
    switch (h->d) {
#define SKYCELL_DYN_CASE(DD)                                                                                     \
    case DD:                                                                                                     \
        if (h->dtype == SKYCELL_DTYPE_F32)                                                                       \
            hipLaunchKernelGGL((k_dyn_cand_delete<float, DD>), dyn_grid(h->count), dim3(kDynThreads), 0, st,     \
                               (const float *)h->pts, h->cap, h->count, (const uint8_t *)h->alive,               \
                               (const uint8_t *)h->sky, (const uint32_t *)h->dels, (const uint32_t *)h->ctr,     \
                               full, h->cand);                                                                    \
        else                                                                                                     \
            hipLaunchKernelGGL((k_dyn_cand_delete<uint16_t, DD>), dyn_grid(h->count), dim3(kDynThreads), 0, st,  \
                               (const uint16_t *)h->pts, h->cap, h->count, (const uint8_t *)h->alive,            \
                               (const uint8_t *)h->sky, (const uint32_t *)h->dels, (const uint32_t *)h->ctr,     \
                               full, h->cand);                                                                    \
        break;
        SKYCELL_DYN_CASE(1)
        SKYCELL_DYN_CASE(2)
        SKYCELL_DYN_CASE(3)
        SKYCELL_DYN_CASE(4)
        SKYCELL_DYN_CASE(5)
        SKYCELL_DYN_CASE(6)
        SKYCELL_DYN_CASE(7)
        SKYCELL_DYN_CASE(8)
        SKYCELL_DYN_CASE(9)
        SKYCELL_DYN_CASE(10)
        SKYCELL_DYN_CASE(11)
        SKYCELL_DYN_CASE(12)
        SKYCELL_DYN_CASE(13)
        SKYCELL_DYN_CASE(14)
        SKYCELL_DYN_CASE(15)
        SKYCELL_DYN_CASE(16)
#undef SKYCELL_DYN_CASE
    default:
        return set_error(SKYCELL_E_INVAL, "d = %d", h->d);
    }
    SKYCELL_HIP_CHECK(hipGetLastError());
    return finish(dyn_recompute(h, h->count, st));
}

int skycell_dyn_skyline(skycell_dyn_t h, int32_t *out_idx, int32_t *out_count, void *stream)
{
    if (h == nullptr) return set_error(SKYCELL_E_INVAL, "handle is NULL");
    if (out_idx == nullptr || out_count == nullptr) return set_error(SKYCELL_E_INVAL, "output pointer is NULL");
    std::lock_guard<std::mutex> lk(h->mu);
    hipStream_t st = (hipStream_t)stream;
    DynFlagLoader ld{h->sky};
    DynFlagEmitter em{out_idx};
    SKYCELL_HIP_CHECK((enqueue_scan<uint32_t>(ld, em, (uint64_t)h->count, h->sums, st)));
    hipLaunchKernelGGL(k_dyn_total, dim3(1), dim3(1), 0, st, (const uint64_t *)h->sums,
                       scan_tiles((uint64_t)h->count), out_count);
    SKYCELL_HIP_CHECK(hipGetLastError());
    return clear_error();
}
