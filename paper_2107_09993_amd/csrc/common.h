// Shared definitions of the gfx950 skyline kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace skycell {

constexpr int kMaxD = 16;
constexpr uint32_t kMaxCells = 1u << 26;
constexpr int kWave = 64;

// Bit of a cell-info word marking a surviving non-empty cell: it holds points
// and no non-empty cell has a smaller column in every dimension (Definition 3).
constexpr uint32_t kOccBit = 1u << 31;
// Low kMaxD bits of the info word: bit k set iff the cell one column lower in
// dimension k exists and some non-empty cell lies in its lower cone.
constexpr uint32_t kNbrMask = (1u << kMaxD) - 1u;

// Query points per refine work item, by dimensionality.
__host__ __device__ constexpr int items_per_group(int d) { return d <= 8 ? 4 : 2; }

// Regular grid of g columns per dimension, cells numbered in mixed radix with
// dimension 0 fastest: x = sum_k c[k] * g^k.
struct GridDesc {
    int32_t d;
    int32_t g;
    uint32_t cells;            // g^d
    uint32_t stride[kMaxD];    // g^k
    uint32_t diag;             // sum_k g^k: x - diag is the cell one column lower everywhere
    int32_t log_w;             // log2 of the bit width of one lane-cone offset field
};

// Device scratch carved out of one workspace allocation.
struct Workspace {
    uint32_t *cell_of;    // [n]     cell of each input point
    uint32_t *cnt;        // [cells] points per cell; later the scatter cursor
    uint8_t *lc;          // [cells] lower closure: some non-empty cell <= this one
    uint32_t *info;       // [cells] kOccBit | lower-neighbour mask
    uint32_t *offs;       // [cells + 1] first sorted position of each surviving cell
    uint32_t *keys;       // [n * d] order-preserving keys of surviving points, AoS, sorted by cell
    int32_t *sidx;        // [n]     original index of each sorted surviving point
    uint2 *items;         // [n]     refine work items
    uint8_t *flag;        // [n]     1 = skyline, by original index
    uint64_t *block_sums; // scan partials
    uint32_t *ctr;        // small counters, see CtrIndex
};

enum CtrIndex {
    kCtrHead = 0,      // refine work-queue head
    kCtrItems = 1,     // number of refine work items
    kCtrErr = 2,       // nonzero: NaN seen in the input
    kCtrSurvPts = 3,   // number of surviving points
    kCtrCount = 8      // number of 32-bit counters reserved
};

size_t workspace_layout(int64_t n, int d, uint32_t cells, Workspace *ws, char *base);

// ---- launchers (all enqueue on `st`; return hipSuccess or the launch error) ----
hipError_t launch_init(const Workspace &ws, const GridDesc &gd, uint64_t *stats, hipStream_t st);
hipError_t launch_quantize_hist(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                                int value_bits, const Workspace &ws, hipStream_t st);
hipError_t launch_cell_prune(const GridDesc &gd, const Workspace &ws, uint64_t *stats, hipStream_t st);
hipError_t launch_cell_scan(const GridDesc &gd, const Workspace &ws, uint64_t *stats, hipStream_t st);
hipError_t launch_scatter(const void *pts, int dtype, int64_t n, const GridDesc &gd,
                          const Workspace &ws, hipStream_t st);
hipError_t launch_refine(int64_t n, const GridDesc &gd, const Workspace &ws, uint64_t *stats,
                         int num_cus, hipStream_t st);
hipError_t launch_output(int64_t n, const Workspace &ws, int32_t *out_idx, int32_t *out_count,
                         uint64_t *stats, hipStream_t st);
hipError_t launch_write_zero_count(int32_t *out_count, hipStream_t st);

// ---- device helpers ----
#if defined(__HIPCC__)
// Order-preserving key of a binary32 value: key(a) < key(b) iff a < b, with
// -0.0 mapped to the key of +0.0.  Comparing keys as integers is exact for
// subnormals whatever the floating-point denormal mode.
__device__ __forceinline__ uint32_t f32_key(float v)
{
    uint32_t b = __float_as_uint(v);
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
#endif

}  // namespace skycell
