// Host helpers shared by the C ABI translation units.
#pragma once

#include <stdint.h>

#include "common.h"

namespace skycell {

int set_error(int code, const char *fmt, ...);  // records the thread's error text, returns code
int clear_error();                               // clears it, returns SKYCELL_OK
uint64_t grid_cells(int g, int d);               // 2^(r*d), saturated above the cell budget
GridDesc grid_desc(int d, int g);
int choose_grid_batched(int64_t n, int d, int dtype);
int device_cus(int dev);
// Enqueue the whole single-instance path (n > 0) on `st` with a workspace of
// workspace_layout(n, d, cells) bytes; no allocation, no synchronisation.
int run_pipeline(const void *points, int32_t dtype, int64_t n, int32_t d, int g, int32_t value_bits,
                 int32_t *out_idx, int32_t *out_count, void *workspace, uint64_t *stats, hipStream_t st);

}  // namespace skycell
