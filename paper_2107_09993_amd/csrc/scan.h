// Device-wide exclusive scan in three launches (reduce tiles, scan the tile
// sums in one block, rescan each tile and hand every element its prefix to an
// emitter).  Used to turn per-cell counts into the counting-sort offsets of the
// surviving points and refine work items, and skyline flags into the ascending
// output index list.
#pragma once

#include "common.h"

namespace skycell {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kPartialThreads = 1024;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread across a block of NT threads.
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total, T *s_w)
{
    const T inc = wave_inclusive_scan(v);
    const int w = threadIdx.x / kWave;
    if (__lane_id() == kWave - 1) s_w[w] = inc;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
        const T s = s_w[i];
        before += (i < w) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

template <typename T, typename Loader>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Loader ld, uint64_t count,
                                                              uint64_t *block_sums)
{
    __shared__ T s_w[kScanThreads / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const uint64_t i = base + (uint64_t)j * kScanThreads + threadIdx.x;
        if (i < count) s += ld(i);
    }
    T tot;
    block_exclusive_scan<T, kScanThreads>(s, &tot, s_w);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = (uint64_t)tot;
}

// In-place exclusive scan of `nb` tile sums; block_sums[nb] receives the total.
__global__ __launch_bounds__(kPartialThreads) void k_scan_partials(uint64_t *block_sums, uint32_t nb);

// Rescan of one tile: values are loaded lane-contiguous (coalesced) into LDS,
// each thread scans its own run of kScanPer consecutive elements there and
// overwrites them with their exclusive prefixes (the element after the tile
// gets the tile's end), and the emitter is then called lane-contiguous with
// prefix p[e] and value p[e+1] - p[e], so its per-element writes coalesce.
template <typename T, typename Loader, typename Emitter>
__global__ __launch_bounds__(kScanThreads) void k_scan_emit(Loader ld, Emitter em, uint64_t count,
                                                            const uint64_t *block_sums)
{
    __shared__ T s_w[kScanThreads / kWave];
    __shared__ T s_v[kScanTile + 1];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int e = j * kScanThreads + (int)threadIdx.x;
        const uint64_t i = base + (uint64_t)e;
        s_v[e] = (i < count) ? ld(i) : T(0);
    }
    __syncthreads();
    const int own = (int)threadIdx.x * kScanPer;
    T v[kScanPer];
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = s_v[own + j];
        s += v[j];
    }
    T tot;
    T run = block_exclusive_scan<T, kScanThreads>(s, &tot, s_w) + (T)block_sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        s_v[own + j] = run;
        run += v[j];
    }
    if (threadIdx.x == kScanThreads - 1) s_v[kScanTile] = run;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int e = j * kScanThreads + (int)threadIdx.x;
        const uint64_t i = base + (uint64_t)e;
        if (i < count) {
            const T p = s_v[e];
            em(i, p, (T)(s_v[e + 1] - p));
        }
    }
}

inline uint32_t scan_tiles(uint64_t count) { return (uint32_t)((count + kScanTile - 1) / kScanTile); }

// Enqueue the three launches.  block_sums needs scan_tiles(count) + 1 entries.
template <typename T, typename Loader, typename Emitter>
hipError_t enqueue_scan(Loader ld, Emitter em, uint64_t count, uint64_t *block_sums, hipStream_t st)
{
    const uint32_t nb = scan_tiles(count);
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kPartialThreads), 0, st, block_sums, 0u);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_scan_reduce<T, Loader>), dim3(nb), dim3(kScanThreads), 0, st, ld, count,
                       block_sums);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kPartialThreads), 0, st, block_sums, nb);
    hipLaunchKernelGGL((k_scan_emit<T, Loader, Emitter>), dim3(nb), dim3(kScanThreads), 0, st, ld,
                       em, count, (const uint64_t *)block_sums);
    return hipGetLastError();
}

}  // namespace skycell
