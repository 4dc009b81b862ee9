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

struct TreeScratch;
int set_error(int code, const char *fmt, ...);  // records the thread's error text, returns code
int clear_error();                               // clears it, returns SKYCELL_OK
uint64_t grid_cells(int g, int d);               // 2^(r*d), saturated above the cell budget
GridDesc grid_desc(int d, int g);
// grid_desc with the refine form chosen for an instance of n points (from the
// tuning table's rows for input class cls first, when cls >= 0)
GridDesc pipeline_desc(int64_t n, int d, int g, int dtype, int cls = -1);
int choose_grid_batched(int64_t n, int d, int dtype);
int device_cus(int dev);
// Enqueue the whole single-instance path (n > 0) on `st` with a workspace of
// workspace_layout(n, d, cells) bytes; no allocation, no synchronisation.
// With pivots (binary32 points only), points of surviving cells that a pivot
// dominates are dropped before the counting sort.
// With tree (grid g = 2^rho), the survivors are the tree form's instead of
// the prefix-OR prune's.
int run_pipeline(const void *points, int32_t dtype, int64_t n, int32_t d, int g, int32_t value_bits,
                 int32_t *out_idx, int32_t *out_count, void *workspace, uint64_t *stats, hipStream_t st,
                 const PivotArgs *piv = nullptr, const TreeScratch *tree = nullptr, int cls = -1);
// Input class of the points (SKYCELL_CLASS_*) from a sample's moments
// (input_class.hip): the launch, its buffer size, and the host-side decision.
size_t class_moments_bytes(int d);
hipError_t launch_class_moments(const void *pts, int dtype, int64_t n, int d, double *out, hipStream_t st);
int class_from_moments(const double *part, int d, int64_t n);
int validate(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res, int32_t value_bits,
             const int32_t *out_idx, const int32_t *out_count);
int resolve_grid(int64_t n, int32_t d, int32_t dtype, int32_t grid_res, int *g_out, int cls = -1);
size_t workspace_layout(int64_t n, int d, uint32_t cells, Workspace *ws, char *base);
// Library-owned device buffer per (slot, device, stream), grown on demand
// (the stream is synchronised before an old buffer is freed).
enum CacheSlot { kCacheWorkspace = 0, kCachePivots = 1, kCacheTree = 2, kCacheFine = 3, kCacheClass = 4, kCacheCount = 5 };

// Scratch of the paper's tree-form cell prune (Algorithm 3 per layer) for
// grids of cells = 2^(rho*d) cells.
struct TreeScratch {
    uint64_t *occ;      // occupancy pyramid, layers 0..rho
    uint64_t *cand[2];  // candidate bitmaps of the previous and the current layer
    uint32_t *leaf;     // [cells] leaves in the current rotation's order
    uint32_t *lptr;     // [cells] l pointer of each cell
    uint32_t *U, *Lv;   // tree levels
    uint64_t *sums;     // scan partials
    uint32_t *count;    // [1] leaves of the current layer
};
size_t tree_scratch_layout(uint32_t cells, int d, int rho, TreeScratch *ts, char *base);
// Layers 1..rho of the tree form on the histogram of layer rho; optional
// copies of every layer's key and candidate bitmaps.
hipError_t run_shrink_tree(const uint32_t *cnt, int d, int rho, const TreeScratch &ts, uint64_t *key_out,
                           uint64_t *cand_out, hipStream_t st);
// Survivor bits of the records and the scatter's bitmap from the tree's layer-rho result.
hipError_t apply_shrink_tree(const TreeScratch &ts, int rho, const Workspace &ws, uint32_t cells, uint64_t *stats,
                             hipStream_t st);
// Process-wide cell prune form: 0 prefix-OR, 1 the tree form (skycell_set_cell_prune).
int cell_prune_form();
int cached_buffer(int slot, int dev, hipStream_t st, size_t need, void **ptr);

}  // namespace skycell
