// Quadrant (dynamic-origin) skyline queries, Section VII-B3: a query point o
// becomes the origin of the data space and only the points in its top-right
// quadrant, { p : p[k] >= o[k] for every k }, take part; the answer is the
// skyline (Definitions 1-2) of that subset.  The paper runs 10,000 such
// queries with random origins on one dataset.
//
// On the GPU the queries become the instances of one batched plan:
//   count   every (tile of 1024 points, chunk of 64 queries) workgroup counts,
//           per query, the tile's points in the query's quadrant;
//   scan    one exclusive scan over the query-major count matrix gives every
//           (query, tile) its first position among the query's points, so
//           each query's subset is laid out in ascending point order;
//   gather  the same workgroups write each subset as an SoA instance block of
//           the batched plan, with its original indices;
//   batched one graph launch computes every instance's skyline;
//   map     local skyline indices become original point indices (ascending,
//           because the subsets are).
// The quadrant test compares order-preserving keys (binary32: -0.0 = +0.0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/skycell.h"
#include "common.h"
#include "host_internal.h"
#include "scan.h"

namespace skycell {

constexpr int kQThreads = 256;
constexpr int kQPer = 4;                          // points per thread
constexpr int kQTile = kQThreads * kQPer;         // points per tile
constexpr int kQChunk = 64;                       // queries per workgroup
constexpr int32_t kMaxQueries = 65535 * kQChunk;  // grid.y holds the query chunks

__device__ __forceinline__ uint32_t q_key(const float *p, size_t i) { return f32_key(p[i]); }
__device__ __forceinline__ uint32_t q_key(const uint16_t *p, size_t i) { return (uint32_t)p[i]; }

// Load the origins of one chunk of queries (as keys) into LDS; flag NaN origins.
template <typename T>
__device__ __forceinline__ void q_load_origins(const T *__restrict__ origins, int32_t nq, int d, int32_t q0,
                                               uint32_t *s_o, uint32_t *err)
{
    for (int e = threadIdx.x; e < kQChunk * d; e += kQThreads) {
        const int qq = e / d, k = e % d;
        uint32_t v = 0xFFFFFFFFu;  // absent query: nothing is >= it
        if (q0 + qq < nq) {
            const T o = origins[(size_t)k * nq + q0 + qq];
            if constexpr (sizeof(T) == 4) {
                if (o != o) atomicOr(err, 1u);
            }
            v = q_key(origins, (size_t)k * nq + q0 + qq);
        }
        s_o[qq * d + k] = v;
    }
}

// Bit s of the result: point tile*kQTile + threadIdx.x*kQPer + s lies in the
// quadrant of query qq of the chunk.
template <typename T, int D>
__device__ __forceinline__ uint32_t q_members(const uint32_t (&key)[kQPer][D], uint32_t valid,
                                              const uint32_t *s_o, int qq)
{
    uint32_t bits = 0u;
#pragma unroll
    for (int s = 0; s < kQPer; ++s) {
        uint32_t lt = 0u;
#pragma unroll
        for (int k = 0; k < D; ++k) lt |= key[s][k] < s_o[qq * D + k] ? 1u : 0u;
        bits |= (lt == 0u && (valid >> s) & 1u) ? (1u << s) : 0u;
    }
    return bits;
}

template <typename T, int D>
__device__ __forceinline__ uint32_t q_load_points(const T *__restrict__ pts, int64_t n, int64_t base,
                                                  uint32_t (&key)[kQPer][D])
{
    uint32_t valid = 0u;
#pragma unroll
    for (int s = 0; s < kQPer; ++s) {
        const int64_t i = base + s;
        const bool ok = i < n;
        valid |= ok ? (1u << s) : 0u;
#pragma unroll
        for (int k = 0; k < D; ++k) key[s][k] = ok ? q_key(pts, (size_t)k * n + i) : 0u;
    }
    return valid;
}

// cnt[q * tiles + t] = points of tile t in the quadrant of query q.
template <typename T, int D>
__global__ __launch_bounds__(kQThreads) void k_quad_count(const T *__restrict__ pts, int64_t n,
                                                          const T *__restrict__ origins, int32_t nq, uint32_t tiles,
                                                          uint32_t *__restrict__ cnt, uint32_t *__restrict__ err)
{
    __shared__ uint32_t s_o[kQChunk * D];
    __shared__ uint32_t s_c[kQChunk];
    const uint32_t tile = blockIdx.x;
    const int32_t q0 = (int32_t)blockIdx.y * kQChunk;
    q_load_origins(origins, nq, D, q0, s_o, err);
    if (threadIdx.x < kQChunk) s_c[threadIdx.x] = 0u;
    uint32_t key[kQPer][D];
    const uint32_t valid = q_load_points<T, D>(pts, n, (int64_t)tile * kQTile + threadIdx.x * kQPer, key);
    __syncthreads();
    for (int qq = 0; qq < kQChunk; ++qq) {
        const uint32_t bits = q_members<T, D>(key, valid, s_o, qq);
        uint32_t c = (uint32_t)__popc(bits);
        // wave sum, then one LDS atomic per wave
        for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
        if (__lane_id() == 0 && c) atomicAdd(&s_c[qq], c);
    }
    __syncthreads();
    if (threadIdx.x < kQChunk && q0 + (int32_t)threadIdx.x < nq)
        cnt[(size_t)(q0 + threadIdx.x) * tiles + tile] = s_c[threadIdx.x];
}

// Writes each query's subset into its instance block: for query q of n_q points
// at element offset poff[q], coordinate k of its t-th point goes to
// block[poff[q] + k * n_q + t], and its original index to ids[ooff[q] + t].
template <typename T, int D>
__global__ __launch_bounds__(kQThreads) void k_quad_gather(const T *__restrict__ pts, int64_t n,
                                                           const T *__restrict__ origins, int32_t nq, uint32_t tiles,
                                                           const uint64_t *__restrict__ pre,
                                                           const int64_t *__restrict__ poff,
                                                           const int64_t *__restrict__ ooff, T *__restrict__ block,
                                                           int32_t *__restrict__ ids, uint32_t *__restrict__ err)
{
    __shared__ uint32_t s_o[kQChunk * D];
    __shared__ uint32_t s_w[kQChunk][kQThreads / kWave];
    __shared__ uint8_t s_bits[kQChunk][kQThreads];
    const uint32_t tile = blockIdx.x;
    const int32_t q0 = (int32_t)blockIdx.y * kQChunk;
    q_load_origins(origins, nq, D, q0, s_o, err);
    uint32_t key[kQPer][D];
    const int64_t base = (int64_t)tile * kQTile + threadIdx.x * kQPer;
    const uint32_t valid = q_load_points<T, D>(pts, n, base, key);
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const int lane = __lane_id();
    // membership of this thread's points per query, kept in LDS between the passes
    for (int qq = 0; qq < kQChunk; ++qq) {
        const uint32_t bits = q_members<T, D>(key, valid, s_o, qq);
        s_bits[qq][threadIdx.x] = (uint8_t)bits;
        uint32_t c = (uint32_t)__popc(bits);
        for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
        if (lane == 0) s_w[qq][w] = c;
    }
    __syncthreads();
    for (int qq = 0; qq < kQChunk; ++qq) {
        const int32_t q = q0 + qq;
        if (q >= nq) break;
        const uint32_t bits = s_bits[qq][threadIdx.x];
        // exclusive prefix of this thread's count inside its wave
        const uint32_t c = (uint32_t)__popc(bits);
        uint32_t inc = c;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t u = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += u;
        }
        if (bits == 0u) continue;
        uint32_t before = inc - c;
        for (int ww = 0; ww < w; ++ww) before += s_w[qq][ww];
        const uint64_t row = pre[(size_t)q * tiles];
        const int64_t nqpts = (int64_t)(pre[(size_t)(q + 1) * tiles] - row);
        int64_t t = (int64_t)(pre[(size_t)q * tiles + tile] - row) + before;
        T *dst = block + poff[q];
        int32_t *idst = ids + ooff[q];
#pragma unroll
        for (int s = 0; s < kQPer; ++s) {
            if (!((bits >> s) & 1u)) continue;
            const int64_t i = base + s;
#pragma unroll
            for (int k = 0; k < D; ++k) dst[(size_t)k * nqpts + t] = pts[(size_t)k * n + i];
            idst[t] = (int32_t)i;
            ++t;
        }
    }
}

struct QCountLoader {
    const uint32_t *cnt;
    __device__ uint64_t operator()(uint64_t i) const { return (uint64_t)cnt[i]; }
};

struct QPrefixEmitter {
    uint64_t *pre;
    __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t) const { pre[i] = prefix; }
};

// The scan's total goes to pre[count] (so row q + 1 of the matrix starts there
// for the last query).
__global__ void k_quad_total(const uint64_t *block_sums, uint32_t nb, uint64_t *pre, uint64_t count)
{
    pre[count] = block_sums[nb];
}

// Local skyline index -> original index, for every written output slot.
__global__ __launch_bounds__(kQThreads) void k_quad_map(const int32_t *__restrict__ local,
                                                        const int32_t *__restrict__ counts,
                                                        const int64_t *__restrict__ ooff, int32_t nq,
                                                        const int32_t *__restrict__ ids, int32_t *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
    if (e >= ooff[nq]) return;
    // query of slot e: the last q with ooff[q] <= e
    int32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (ooff[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    const int64_t t = e - ooff[lo];
    if (t < counts[lo]) out[e] = ids[ooff[lo] + local[e]];
}

// rows[q] = first position of query q's points (q = nq: the total)
__global__ __launch_bounds__(kQThreads) void k_quad_rows(const uint64_t *__restrict__ pre, int32_t nq, uint32_t tiles,
                                                         uint64_t *__restrict__ rows)
{
    const int64_t q = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
    if (q <= nq) rows[q] = pre[(size_t)q * tiles];
}

__global__ void k_quad_zero(uint32_t *err)
{
    if (threadIdx.x == 0) *err = 0u;
}

}  // namespace skycell

using namespace skycell;

struct skycell_quad {
    int dev = 0;
    int d = 0;
    int dtype = SKYCELL_DTYPE_F32;
    int64_t n = 0;
    int32_t nq = 0;
    uint32_t tiles = 0;
    size_t esize = 4;
    std::vector<int64_t> h_poff, h_ooff;
    int64_t total = 0;
    uint32_t *cnt = nullptr;     // [nq * tiles]
    uint64_t *pre = nullptr;     // [nq * tiles + 1]
    uint64_t *sums = nullptr;
    uint32_t *err = nullptr;
    int64_t *poff = nullptr;     // [nq + 1] element offsets of the instance blocks
    int64_t *ooff = nullptr;     // [nq + 1] point offsets
    void *block = nullptr;       // instance blocks
    int32_t *ids = nullptr;      // [total] original index of each gathered point
    int32_t *local = nullptr;    // [total] batched output (local indices)
    skycell_plan_t plan = nullptr;
};

static void quad_free(skycell_quad *h)
{
    if (h->plan) (void)skycell_plan_destroy(h->plan);
    void *bufs[] = {h->cnt, h->pre, h->sums, h->err, h->poff, h->ooff, h->block, h->ids, h->local};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

template <typename T>
static hipError_t quad_launch(bool gather, const skycell_quad *h, const void *points, const void *origins,
                              hipStream_t st)
{
    const dim3 grid(h->tiles, (unsigned)((h->nq + kQChunk - 1) / kQChunk));
    switch (h->d) {
#define SKYCELL_QUAD_CASE(DD)                                                                                    \
    case DD:                                                                                                     \
        if (gather)                                                                                              \
            hipLaunchKernelGGL((k_quad_gather<T, DD>), grid, dim3(kQThreads), 0, st, (const T *)points, h->n,    \
                               (const T *)origins, h->nq, h->tiles, (const uint64_t *)h->pre,                    \
                               (const int64_t *)h->poff, (const int64_t *)h->ooff, (T *)h->block, h->ids,        \
                               h->err);                                                                          \
        else                                                                                                     \
            hipLaunchKernelGGL((k_quad_count<T, DD>), grid, dim3(kQThreads), 0, st, (const T *)points, h->n,     \
                               (const T *)origins, h->nq, h->tiles, h->cnt, h->err);                             \
        break;
        SKYCELL_QUAD_CASE(1)
        SKYCELL_QUAD_CASE(2)
        SKYCELL_QUAD_CASE(3)
        SKYCELL_QUAD_CASE(4)
        SKYCELL_QUAD_CASE(5)
        SKYCELL_QUAD_CASE(6)
        SKYCELL_QUAD_CASE(7)
        SKYCELL_QUAD_CASE(8)
        SKYCELL_QUAD_CASE(9)
        SKYCELL_QUAD_CASE(10)
        SKYCELL_QUAD_CASE(11)
        SKYCELL_QUAD_CASE(12)
        SKYCELL_QUAD_CASE(13)
        SKYCELL_QUAD_CASE(14)
        SKYCELL_QUAD_CASE(15)
        SKYCELL_QUAD_CASE(16)
#undef SKYCELL_QUAD_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t quad_pass(bool gather, const skycell_quad *h, const void *points, const void *origins,
                            hipStream_t st)
{
    return h->dtype == SKYCELL_DTYPE_F32 ? quad_launch<float>(gather, h, points, origins, st)
                                         : quad_launch<uint16_t>(gather, h, points, origins, st);
}

int skycell_quadrant_create(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t value_bits,
                            const void *origins, int32_t nq, skycell_quad_t *out, void *stream)
{
    if (out == nullptr) return set_error(SKYCELL_E_INVAL, "handle pointer is NULL");
    *out = nullptr;
    if (points == nullptr || origins == nullptr) return set_error(SKYCELL_E_INVAL, "points or origins is NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return set_error(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 1 || n >= (int64_t)1 << 31) return set_error(SKYCELL_E_INVAL, "n = %lld is outside [1, 2^31)", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return set_error(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (nq < 1 || nq > kMaxQueries) return set_error(SKYCELL_E_INVAL, "nq = %d is outside [1, %d]", nq, kMaxQueries);
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    if (value_bits < 1 || value_bits > 16) return set_error(SKYCELL_E_RANGE, "value_bits = %d outside [1, 16]", value_bits);
    skycell_quad *h = new (std::nothrow) skycell_quad;
    if (h == nullptr) return set_error(SKYCELL_E_NOMEM, "out of host memory");
    h->d = d;
    h->dtype = dtype;
    h->n = n;
    h->nq = nq;
    h->esize = dtype == SKYCELL_DTYPE_F32 ? 4 : 2;
    h->tiles = (uint32_t)((n + kQTile - 1) / kQTile);
    hipStream_t st = (hipStream_t)stream;
    const uint64_t cells = (uint64_t)nq * h->tiles;
    auto bail = [&](int code, const char *what, hipError_t e) {
        quad_free(h);
        delete h;
        return set_error(code, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipGetDevice(&h->dev);
    if (e == hipSuccess) e = hipMalloc((void **)&h->cnt, cells * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->pre, (cells + 1) * 8);
    if (e == hipSuccess)
        e = hipMalloc((void **)&h->sums, (std::max<size_t>((size_t)scan_tiles(cells), (size_t)nq) + 1) * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&h->err, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->poff, ((size_t)nq + 1) * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&h->ooff, ((size_t)nq + 1) * 8);
    if (e != hipSuccess) return bail(SKYCELL_E_NOMEM, "allocating the query tables", e);
    hipLaunchKernelGGL(k_quad_zero, dim3(1), dim3(64), 0, st, h->err);
    if ((e = quad_pass(false, h, points, origins, st)) != hipSuccess) return bail(SKYCELL_E_HIP, "count pass", e);
    QCountLoader ld{h->cnt};
    QPrefixEmitter em{h->pre};
    if ((e = enqueue_scan<uint64_t>(ld, em, cells, h->sums, st)) != hipSuccess) return bail(SKYCELL_E_HIP, "scan", e);
    hipLaunchKernelGGL(k_quad_total, dim3(1), dim3(1), 0, st, (const uint64_t *)h->sums, scan_tiles(cells), h->pre,
                       cells);
    // row starts (and the total) back on the host, through the scan partials
    // (no longer needed, and at least nq + 1 entries long)
    std::vector<uint64_t> rows((size_t)nq + 1);
    hipLaunchKernelGGL(k_quad_rows, dim3((unsigned)((nq + kQThreads) / kQThreads)), dim3(kQThreads), 0, st,
                       (const uint64_t *)h->pre, nq, h->tiles, h->sums);
    e = hipMemcpyAsync(rows.data(), h->sums, ((size_t)nq + 1) * 8, hipMemcpyDeviceToHost, st);
    uint32_t err = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&err, h->err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(SKYCELL_E_HIP, "reading the query sizes", e);
    if (err & 1u) {
        quad_free(h);
        delete h;
        return set_error(SKYCELL_E_NAN, "an origin holds a NaN");
    }
    h->total = (int64_t)rows[nq];
    if (h->total >= (int64_t)1 << 31) {
        quad_free(h);
        delete h;
        return set_error(SKYCELL_E_RANGE, "the quadrants hold %lld points in total, 2^31 or more", (long long)h->total);
    }
    std::vector<int64_t> ns((size_t)nq);
    std::vector<int32_t> ds((size_t)nq, d);
    for (int32_t q = 0; q < nq; ++q) ns[q] = (int64_t)(rows[q + 1] - rows[q]);
    int rc = skycell_batched_plan_create(nq, ns.data(), ds.data(), dtype, value_bits, nullptr, &h->plan);
    if (rc != SKYCELL_OK) {
        h->plan = nullptr;
        quad_free(h);
        delete h;
        return rc;
    }
    h->h_poff.resize((size_t)nq + 1);
    h->h_ooff.resize((size_t)nq + 1);
    (void)skycell_batched_offsets(h->plan, h->h_poff.data(), h->h_ooff.data(), nullptr);
    const size_t tot = (size_t)std::max<int64_t>(h->total, 1);
    e = hipMemcpy(h->poff, h->h_poff.data(), ((size_t)nq + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->ooff, h->h_ooff.data(), ((size_t)nq + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&h->block, (size_t)std::max<int64_t>(h->h_poff[nq], 1) * h->esize);
    if (e == hipSuccess) e = hipMalloc((void **)&h->ids, tot * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&h->local, tot * 4);
    if (e != hipSuccess) return bail(SKYCELL_E_NOMEM, "allocating the instance blocks", e);
    *out = h;
    return clear_error();
}

int skycell_quadrant_offsets(skycell_quad_t h, int64_t *out_off)
{
    if (h == nullptr || out_off == nullptr) return set_error(SKYCELL_E_INVAL, "handle or out_off is NULL");
    for (int32_t q = 0; q <= h->nq; ++q) out_off[q] = h->h_ooff[q];
    return clear_error();
}

int skycell_quadrant_run(skycell_quad_t h, const void *points, const void *origins, int32_t *out_idx,
                         int32_t *out_count, void *stream)
{
    if (h == nullptr) return set_error(SKYCELL_E_INVAL, "handle is NULL");
    if (points == nullptr || origins == nullptr || out_idx == nullptr || out_count == nullptr)
        return set_error(SKYCELL_E_INVAL, "points, origins or an output is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(SKYCELL_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != h->dev) return set_error(SKYCELL_E_INVAL, "created on device %d, current is %d", h->dev, dev);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_quad_zero, dim3(1), dim3(64), 0, st, h->err);
    SKYCELL_HIP_CHECK(quad_pass(true, h, points, origins, st));
    const int rc = skycell_batched_run(h->plan, h->block, h->local, out_count, stream);
    if (rc != SKYCELL_OK) return rc;
    if (h->total > 0) {
        const unsigned blocks = (unsigned)((h->total + kQThreads - 1) / kQThreads);
        hipLaunchKernelGGL(k_quad_map, dim3(blocks), dim3(kQThreads), 0, st, (const int32_t *)h->local,
                           (const int32_t *)out_count, (const int64_t *)h->ooff, h->nq, (const int32_t *)h->ids,
                           out_idx);
        SKYCELL_HIP_CHECK(hipGetLastError());
    }
    return clear_error();
}

int skycell_quadrant_destroy(skycell_quad_t h)
{
    if (h == nullptr) return clear_error();
    (void)hipDeviceSynchronize();
    quad_free(h);
    delete h;
    return clear_error();
}
