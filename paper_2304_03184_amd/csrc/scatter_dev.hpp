// Binned table-gradient scatter (scatter.hip).
#pragma once
#include "grid_dev.hpp"

namespace nvr {

int scatter_tiles(const GridParams &p);
size_t scatter_ws_bytes(const GridParams &p, int64_t cap);
nvr_status scatter_check(const GridParams &p);
// dtable (acc) += binned scatter of w * dfeat; dx_parts: planar -> [8][cap][3]
// partials, row-major -> [n][3] (acc, via atomics); nullable.
nvr_status launch_scatter(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                          const float *x, const void *table, const float *dfeat, float *dtable,
                          float *dx_parts, bool planar, void *ws, hipStream_t st);

}  // namespace nvr
