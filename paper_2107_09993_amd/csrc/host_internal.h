// Host helpers shared by the C ABI translation units.
#pragma once

#include <stdint.h>

#include "common.h"
#include "mlp.h"

namespace skycell {

#define SKYCELL_HIP_CHECK(expr)                                                                   \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return set_error(SKYCELL_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Pivots for the pre-filter of run_pipeline: k indices into the points (device
// memory) and the scratch their table is built in.
struct PivotArgs {
    const int32_t *idx;
    uint32_t k;
    PivotScratch ps;
};

int set_error(int code, const char *fmt, ...);  // records the thread's error text, returns code
int clear_error();                               // clears it, returns SKYCELL_OK
uint64_t grid_cells(int g, int d);               // 2^(r*d), saturated above the cell budget
GridDesc grid_desc(int d, int g);
// grid_desc with the refine form chosen for an instance of n points
GridDesc pipeline_desc(int64_t n, int d, int g, int dtype);
int choose_grid_batched(int64_t n, int d, int dtype);
int device_cus(int dev);
// Enqueue the whole single-instance path (n > 0) on `st` with a workspace of
// workspace_layout(n, d, cells) bytes; no allocation, no synchronisation.
// With pivots (binary32 points only), points of surviving cells that a pivot
// dominates are dropped before the counting sort.
int run_pipeline(const void *points, int32_t dtype, int64_t n, int32_t d, int g, int32_t value_bits,
                 int32_t *out_idx, int32_t *out_count, void *workspace, uint64_t *stats, hipStream_t st,
                 const PivotArgs *piv = nullptr);
int validate(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res, int32_t value_bits,
             const int32_t *out_idx, const int32_t *out_count);
int resolve_grid(int64_t n, int32_t d, int32_t dtype, int32_t grid_res, int *g_out);
size_t workspace_layout(int64_t n, int d, uint32_t cells, Workspace *ws, char *base);
// Library-owned device buffer per (slot, device, stream), grown on demand
// (the stream is synchronised before an old buffer is freed).
enum CacheSlot { kCacheWorkspace = 0, kCachePivots = 1, kCacheCount = 2 };
int cached_buffer(int slot, int dev, hipStream_t st, size_t need, void **ptr);

}  // namespace skycell
