// K6: ordered output.  The per-point skyline flags (indexed by original point
// index) are scanned; every flagged index is written at its prefix, which gives
// the skyline as ascending indices (Definition 2), and the count goes to the
// device-side out_count (or SKYCELL_E_NAN if the input held a NaN).
#include "common.h"
#include "scan.h"
#include "../../include/skycell.h"

namespace skycell {

struct FlagLoader {
    const uint8_t *flag;
    __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)flag[i]; }
};

struct FlagEmitter {
    int32_t *out;
    __device__ void operator()(uint64_t i, uint32_t prefix, uint32_t v) const
    {
        if (v) out[prefix] = (int32_t)i;
    }
};

__global__ void k_output_total(const uint64_t *block_sums, uint32_t nb, const uint32_t *ctr,
                               int32_t *out_count, uint64_t *stats)
{
    const uint64_t tot = block_sums[nb];
    const uint32_t err = ctr[kCtrErr];
    *out_count = (err & 1u) ? (int32_t)SKYCELL_E_NAN : (err & 2u) ? (int32_t)SKYCELL_E_RANGE : (int32_t)tot;
    if (stats != nullptr) stats[SKYCELL_STAT_SKYLINE] = tot;
}

hipError_t launch_output(int64_t n, const Workspace &ws, int32_t *out_idx, int32_t *out_count,
                         uint64_t *stats, hipStream_t st)
{
    FlagLoader ld{ws.flag};
    FlagEmitter em{out_idx};
    hipError_t e = enqueue_scan<uint32_t>(ld, em, (uint64_t)n, ws.block_sums, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_output_total, dim3(1), dim3(1), 0, st, (const uint64_t *)ws.block_sums,
                       scan_tiles((uint64_t)n), (const uint32_t *)ws.ctr, out_count, stats);
    return hipGetLastError();
}

__global__ void k_write_zero(int32_t *out_count) { *out_count = 0; }

hipError_t launch_write_zero_count(int32_t *out_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_write_zero, dim3(1), dim3(1), 0, st, out_count);
    return hipGetLastError();
}

}  // namespace skycell
