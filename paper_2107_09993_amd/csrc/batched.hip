// Batched skyline: many independent instances of uneven n and d in one
// persistent launch (captured into a hipGraph by the plan).
//
// Stage A (one workgroup per instance): a workgroup claims the next instance
// in the plan's order (largest estimated work first), runs every grid phase
// of it with block-wide barriers (histogram, lower closure, cell records,
// scan, scatter) and publishes a ready flag with release semantics.
//
// Stage B (one wave per chunk): once no instance is left to claim, each wave
// takes refine chunks (a range of one instance's work items) from a global
// queue, waits until that instance is ready (its preparer is a running
// workgroup: every instance was claimed before any wave got here, and
// preparing never waits on anything), and runs the shared lane loop
// (refine_core.h) for the instance's d.  The wave that finishes the last chunk
// of an instance writes its output.  The last wave of the launch resets the
// control words so the captured graph can be replayed.
//
// No task ever waits for work that has not started, so the launch completes
// whatever number of workgroups is resident.
#include "cellops.h"
#include "common.h"
#include "refine_core.h"
#include "scan.h"
#include "../../include/skycell.h"
#include "batched.h"

namespace skycell {

constexpr int kBatchThreads = 256;
constexpr int kBatchWaves = kBatchThreads / kWave;

// Block-wide grid phases of one instance.
template <typename T>
__device__ void prepare_instance(const T *__restrict__ pts, const BatchInst &I, uint32_t *ic,
                                 int value_bits, uint64_t *s_w)
{
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const GridDesc &gd = I.gd;
    const uint32_t n = I.n, cells = gd.cells;

    for (uint32_t x = tid; x < cells; x += nt) I.cnt[x] = 0u;
    __syncthreads();
    bool nan = false;
    for (uint32_t i = tid; i < n; i += nt) {
        const uint32_t cell = point_cell(pts, n, i, gd, value_bits, nan);
        I.cell_of[i] = cell;
        I.rank[i] = atomicAdd(&I.cnt[cell], 1u);
    }
    if (nan) atomicOr(&ic[kInstErr], 1u);
    __syncthreads();
    for (uint32_t x = tid; x < cells; x += nt) I.lc[x] = I.cnt[x] != 0u ? 1 : 0;
    __syncthreads();
    if (gd.g > 1) {
        const uint32_t lines = cells >> gd.r;
        for (int k = 0; k < gd.d; ++k) {
            for (uint32_t t = tid; t < lines; t += nt) lc_prefix_line(I.lc, t, gd.mask[k], cells - 1u, (uint32_t)gd.g);
            __syncthreads();
        }
    }
    for (uint32_t x = tid; x < cells; x += nt) {
        bool occ, surv;
        I.rec[x] = cell_record(gd, I.cnt, I.lc, x, occ, surv);
    }
    __syncthreads();

    // exclusive scan of the cells: first sorted positions and work items
    const CellLoader ld{I.rec, I.cnt, (uint32_t)gd.m};
    const CellEmitter em{(uint32_t *)I.rec, I.items, (uint32_t)gd.m};
    uint64_t carry = 0ull;
    for (uint32_t base = 0; base < cells; base += kScanTile) {
        uint64_t v[kScanPer];
        uint64_t s = 0ull;
        const uint32_t first = base + tid * kScanPer;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const uint32_t x = first + (uint32_t)j;
            v[j] = x < cells ? ld(x) : 0ull;
            s += v[j];
        }
        uint64_t tot;
        uint64_t run = block_exclusive_scan<uint64_t, kBatchThreads>(s, &tot, s_w) + carry;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const uint32_t x = first + (uint32_t)j;
            if (x < cells) em(x, run, v[j]);
            run += v[j];
        }
        carry += tot;
    }
    if (tid == 0) {
        I.rec[cells] = (uint32_t)carry;  // sentinel start after the last cell
        ic[kInstItems] = (uint32_t)(carry >> 32);
    }
    __syncthreads();

    for (uint32_t i = tid; i < n; i += nt) {
        I.flag[i] = 0;
        const uint64_t r = I.rec[I.cell_of[i]];
        if (rec_surv(r)) scatter_point(pts, n, gd.d, value_bits, i, rec_start(r) + I.rank[i], I.keys, I.fkeys, I.sidx);
    }
}

// Wave-wide ordered output of one instance: indices local to the instance.
__device__ void write_output_wave(const BatchInst &I, const uint32_t *ic, int32_t *__restrict__ out_idx,
                                  int32_t *__restrict__ out_count)
{
    const int lane = __lane_id();
    int32_t *out = out_idx + I.out_off;
    uint32_t count = 0u;
    for (uint32_t base = 0; base < I.n; base += 4u * kWave) {
        const uint32_t i0 = base + 4u * (uint32_t)lane;
        uint32_t f[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) f[t] = (i0 + t < I.n) ? (uint32_t)I.flag[i0 + t] : 0u;
        const uint32_t c = f[0] + f[1] + f[2] + f[3];
        const uint32_t inc = wave_inclusive_scan(c);
        uint32_t pos = count + inc - c;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (f[t]) out[pos++] = (int32_t)(i0 + t);
        count += __shfl(inc, kWave - 1);
    }
    if (lane == 0) *out_count = ic[kInstErr] ? (int32_t)SKYCELL_E_NAN : (int32_t)count;
}

struct OnceFeeder {
    uint32_t lo, hi;
    bool used;
    __device__ bool next(uint32_t &a, uint32_t &b)
    {
        if (used) return false;
        used = true;
        a = lo;
        b = hi;
        return true;
    }
};

template <int D>
__device__ __attribute__((noinline)) void refine_chunk(const RefineView &v, uint32_t lo, uint32_t hi, uint32_t &visits, uint32_t &tests)
{
    OnceFeeder f{lo, hi, false};
    refine_loop<D, items_per_group(D)>(v, f, visits, tests);
}

template <typename T>
// At least 4 waves per SIMD: the refine chunks are latency-bound (the 16
// instantiations of the lane loop would otherwise need 178 VGPRs).
__global__ __launch_bounds__(kBatchThreads, 4) void k_batched(const T *__restrict__ pts,
                                                           const BatchInst *__restrict__ inst,
                                                           const uint32_t *__restrict__ prep_order,
                                                           uint32_t num_inst,
                                                           const uint32_t *__restrict__ chunk_inst,
                                                           uint32_t num_chunks, uint32_t chunk_items,
                                                           uint32_t *__restrict__ ctl,
                                                           uint32_t *__restrict__ ictl,
                                                           int32_t *__restrict__ out_idx,
                                                           int32_t *__restrict__ out_count,
                                                           int value_bits)
{
    __shared__ uint64_t s_w[kBatchWaves];
    __shared__ uint32_t s_b;
    __shared__ uint32_t s_mask[kBatchWaves][kMaxD], s_low[kBatchWaves][kMaxD];
    const int lane = __lane_id();
    const int wv = threadIdx.x / kWave;

    // ---- stage A: prepare instances, one per workgroup at a time
    for (;;) {
        if (threadIdx.x == 0) s_b = atomicAdd(&ctl[kBatchNextPrep], 1u);
        __syncthreads();
        const uint32_t slot = s_b;
        __syncthreads();
        if (slot >= num_inst) break;
        const uint32_t b = prep_order[slot];
        uint32_t *ic = ictl + kInstWords * b;
        prepare_instance<T>(pts + inst[b].pts_off, inst[b], ic, value_bits, s_w);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(&ic[kInstReady], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- stage B: refine chunks, one wave at a time
    uint32_t visits = 0u, tests = 0u;
    for (;;) {
        uint32_t c = 0u;
        if (lane == 0) c = atomicAdd(&ctl[kBatchNextChunk], 1u);
        c = __shfl(c, 0);
        if (c >= num_chunks) break;
        const uint32_t b = chunk_inst[c];
        uint32_t *ic = ictl + kInstWords * b;
        if (lane == 0) {
            while (__hip_atomic_load(&ic[kInstReady], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                __builtin_amdgcn_s_sleep(8);
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        const BatchInst &I = inst[b];
        const uint32_t n_items = __hip_atomic_load(&ic[kInstItems], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t lo = (c - I.chunk0) * chunk_items;
        const uint32_t hi = lo + chunk_items < n_items ? lo + chunk_items : n_items;
        if (lo < hi) {
            const int d = I.gd.d;
            if (lane < kMaxD) {
                uint32_t low = 0u;
                for (int k = 0; k < lane && k < d; ++k) low |= I.gd.mask[k];
                s_mask[wv][lane] = lane < d ? I.gd.mask[lane] : 0u;
                s_low[wv][lane] = low;
            }
            const RefineView v{I.keys, I.fkeys, I.sidx, I.rec, I.items, I.flag, s_mask[wv], s_low[wv]};
            switch (d) {
#define SKYCELL_BATCH_CASE(DD) \
    case DD:                   \
        refine_chunk<DD>(v, lo, hi, visits, tests); \
        break;
                SKYCELL_BATCH_CASE(1)
                SKYCELL_BATCH_CASE(2)
                SKYCELL_BATCH_CASE(3)
                SKYCELL_BATCH_CASE(4)
                SKYCELL_BATCH_CASE(5)
                SKYCELL_BATCH_CASE(6)
                SKYCELL_BATCH_CASE(7)
                SKYCELL_BATCH_CASE(8)
                SKYCELL_BATCH_CASE(9)
                SKYCELL_BATCH_CASE(10)
                SKYCELL_BATCH_CASE(11)
                SKYCELL_BATCH_CASE(12)
                SKYCELL_BATCH_CASE(13)
                SKYCELL_BATCH_CASE(14)
                SKYCELL_BATCH_CASE(15)
                SKYCELL_BATCH_CASE(16)
#undef SKYCELL_BATCH_CASE
            default:
                break;
            }
        }
        // the flags written by this wave must be visible to the wave that writes the output
        __threadfence();
        uint32_t done = 0u;
        if (lane == 0)
            done = __hip_atomic_fetch_add(&ic[kInstDone], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        done = __shfl(done, 0);
        if (done == I.nchunks) {
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            write_output_wave(I, ic, out_idx, out_count + b);
        }
    }

    // ---- the last wave resets the control words for the next launch
    const uint32_t total = gridDim.x * kBatchWaves;
    uint32_t fin = 0u;
    if (lane == 0) fin = __hip_atomic_fetch_add(&ctl[kBatchFinished], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    fin = __shfl(fin, 0);
    if (fin == total) {
        for (uint32_t w = (uint32_t)lane; w < kInstWords * num_inst; w += kWave) ictl[w] = 0u;
        if (lane == 0) {
            ctl[kBatchNextPrep] = 0u;
            ctl[kBatchNextChunk] = 0u;
            ctl[kBatchFinished] = 0u;
        }
        __threadfence();
    }
    (void)visits;
    (void)tests;
}

int batched_blocks_per_cu(int dtype)
{
    int b = 0;
    hipError_t e = dtype == SKYCELL_DTYPE_F32
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_batched<float>, kBatchThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_batched<uint16_t>, kBatchThreads, 0);
    return (e != hipSuccess || b < 1) ? 1 : b;
}

hipError_t launch_batched(const BatchLaunch &L, hipStream_t st)
{
    if (L.dtype == SKYCELL_DTYPE_F32)
        hipLaunchKernelGGL(k_batched<float>, dim3(L.blocks), dim3(kBatchThreads), 0, st, (const float *)L.points,
                           L.inst, L.prep_order, L.num_inst, L.chunk_inst, L.num_chunks, L.chunk_items, L.ctl,
                           L.ictl, L.out_idx, L.out_count, L.value_bits);
    else
        hipLaunchKernelGGL(k_batched<uint16_t>, dim3(L.blocks), dim3(kBatchThreads), 0, st,
                           (const uint16_t *)L.points, L.inst, L.prep_order, L.num_inst, L.chunk_inst,
                           L.num_chunks, L.chunk_items, L.ctl, L.ictl, L.out_idx, L.out_count, L.value_bits);
    return hipGetLastError();
}

const void *batched_kernel(int dtype)
{
    return dtype == SKYCELL_DTYPE_F32 ? reinterpret_cast<const void *>(&k_batched<float>)
                                      : reinterpret_cast<const void *>(&k_batched<uint16_t>);
}

int batched_threads() { return kBatchThreads; }

}  // namespace skycell
