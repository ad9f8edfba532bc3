// Binned table-gradient scatter (scatter.hip).
#pragma once
#include "grid_dev.hpp"

namespace nvr {

// Optional second stream for a scatter's accumulate and reduce launches: they
// wait (fork event recorded on the caller's stream) for the launches before
// them, and the caller joins the stream back before it reads the table
// gradient; the work after the emit pass (which forms the position gradient)
// then overlaps with them.
struct ScatterTail {
    hipStream_t stream;
    hipEvent_t fork;
};

int scatter_tiles(const GridParams &p);
size_t scatter_ws_bytes(const GridParams &p, int64_t cap);
nvr_status scatter_check(const GridParams &p);
// The tile counter inside a scatter workspace, and a launch that zeroes it.
TileCounter scatter_counter(const GridParams &p, void *ws);
nvr_status launch_counter_reset(const GridParams &p, void *ws, hipStream_t st);
// dtable (acc) += binned scatter of w * dfeat, dfeat in the level-group-planar
// layout [8][cap][2 lpg] (level g + 8 m at [g][s][2m, 2m+1]); dx_parts
// (nullable) receives the [8][cap][3] per-group position-gradient partials.
// counted: the tile counts in ws were already formed (zeroed, then counted by
// the forward gather over the same positions); otherwise they are counted here.
// jac (nullable): the spatial derivatives the forward gather stored for these
// positions (launch_encode_fwd); with it the position gradient reads them
// instead of the table's corner values.
nvr_status launch_scatter(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                          const float *x, const void *table, const float *dfeat, float *dtable,
                          float *dx_parts, void *ws, hipStream_t st,
                          bool counted = false, int emit_chunks = 0, int emit_block = 0,
                          const uint32_t *jac = nullptr, const ScatterTail *tail = nullptr);
// The deterministic variant: same records, order fixed by the inputs (tile
// counts formed by its own pass; no launch-shape choices).
size_t scatter_det_ws_bytes(const GridParams &p, int64_t cap);
nvr_status launch_scatter_det(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                              const float *x, const void *table, const float *dfeat,
                              float *dtable, float *dx_parts, void *ws, hipStream_t st,
                              const uint32_t *jac = nullptr);
// Row-major feature gradients [cap][2L] (regrouped first), device-side count;
// det selects the deterministic scatter.
size_t scatter_rows_ws_bytes(const GridParams &p, int64_t cap, bool det);
nvr_status launch_scatter_rows(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                               const float *x, const float *dfeat, float *dtable, void *ws,
                               hipStream_t st, bool det);
// the scan and emit passes alone (tile counts already formed), for tuning
nvr_status launch_scatter_emit_only(const GridParams &p, int64_t n, const int32_t *n_dev,
                                    int64_t cap, const float *x, const void *table,
                                    const float *dfeat, void *ws, hipStream_t st,
                                    int emit_chunks, int emit_block);

}  // namespace nvr
