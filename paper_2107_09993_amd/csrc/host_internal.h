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

}  // namespace skycell
