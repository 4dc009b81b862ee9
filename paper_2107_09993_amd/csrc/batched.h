// Device-side description of a batched plan (see batched.hip).
#pragma once

#include "common.h"

namespace skycell {

// One instance: its points (an SoA block of the batch's points buffer), its
// grid, its slice of the output and its workspace buffers.
struct BatchInst {
    uint64_t pts_off;   // element offset of the [d][n] block in the points buffer
    uint32_t n;
    uint32_t out_off;   // first output slot of the instance
    uint32_t chunk0;    // first refine chunk of the instance in the chunk table
    uint32_t nchunks;   // refine chunks reserved for it (ceil(n / chunk_items), at least 1)
    GridDesc gd;
    uint32_t *cell_of;
    uint32_t *rank;
    uint32_t *cnt;
    uint8_t *lc;
    uint64_t *rec;
    uint32_t *keys;
    uint64_t *fkeys;
    int32_t *sidx;
    uint2 *items;
    uint8_t *flag;
};

// Global control words (zero between launches).
enum BatchCtl { kBatchNextPrep = 0, kBatchNextChunk = 1, kBatchFinished = 2, kBatchCtlWords = 4 };
// Per-instance control words (zero between launches).
enum InstCtl { kInstReady = 0, kInstItems = 1, kInstDone = 2, kInstErr = 3, kInstWords = 4 };

struct BatchLaunch {
    int dtype;
    const void *points;
    const BatchInst *inst;
    const uint32_t *prep_order;
    uint32_t num_inst;
    const uint32_t *chunk_inst;
    uint32_t num_chunks;
    uint32_t chunk_items;
    uint32_t *ctl;
    uint32_t *ictl;
    int32_t *out_idx;
    int32_t *out_count;
    int value_bits;
    unsigned blocks;
};

hipError_t launch_batched(const BatchLaunch &L, hipStream_t st);
const void *batched_kernel(int dtype);
int batched_blocks_per_cu(int dtype);
int batched_threads();

}  // namespace skycell
