// Allocation-free entry point: the exact skyline of skycell_compute_ws with
// its workspace in a fixed device array of this library instead of caller or
// library allocations, for callers that cannot allocate device memory (code
// under graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable: each GPU the library runs on
// holds its own copy, at its own device address, from the time the module is
// loaded on that GPU until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory, so the device address is
// looked up once per device (hipGetSymbolAddress with that device current) and
// only that address is passed to kernels.
//
// Every call on one GPU uses that GPU's single array: the path clears what it
// needs (counters, histogram, flags) with its own kernels at the start of each
// call, so the previous call's contents do no harm, but two calls that overlap
// in time on one GPU race on the array and give undefined results.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/skycell.h"
#include "common.h"
#include "host_internal.h"

namespace skycell {

static_assert(SKYCELL_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[SKYCELL_STATIC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on device `dev` (the current device), looked up
// at the first call on that device.
static int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(SKYCELL_E_NODEV, "device %d is beyond the %d devices the static scratch supports", dev,
                         kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return set_error(SKYCELL_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
        if (((uintptr_t)p & 255u) != 0u)
            return set_error(SKYCELL_E_HIP, "static scratch on device %d is not 256-byte aligned", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SKYCELL_OK;
}

}  // namespace skycell

using namespace skycell;

extern "C" int skycell_compute_static(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res,
                                      int32_t value_bits, int32_t *out_idx, int32_t *out_count, uint64_t *stats,
                                      void *stream)
{
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    int rc = validate(points, dtype, n, d, grid_res, value_bits, out_idx, out_count);
    if (rc != SKYCELL_OK) return rc;
    int g = 0;
    if ((rc = resolve_grid(n, d, dtype, grid_res, &g)) != SKYCELL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        SKYCELL_HIP_CHECK(launch_write_zero_count(out_count, st));
        return clear_error();
    }
    const size_t need = workspace_layout(n, d, grid_desc(d, g).cells, nullptr, nullptr);
    if (need > (size_t)SKYCELL_STATIC_SCRATCH_BYTES)
        return set_error(SKYCELL_E_NOMEM,
                         "n = %lld, d = %d on a grid of %d needs %zu workspace bytes, over the static scratch of %zu",
                         (long long)n, d, g, need, (size_t)SKYCELL_STATIC_SCRATCH_BYTES);
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    void *ptr = nullptr;
    if ((rc = scratch_address(dev, &ptr)) != SKYCELL_OK) return rc;
    return run_pipeline(points, dtype, n, d, g, value_bits, out_idx, out_count, ptr, stats, st);
}
