// Pose-conditioned deformation network inside the training step (deform.hip):
// the same kernels as nvr_deform_fwd / nvr_deform_bwd over the first *n_dev
// (at most cap) points.
#pragma once
#include "common.hpp"

namespace nvr {

// Every check of the calls below for grid g and capacity cap.
nvr_status deform_check(const nvr_grid_desc *g, int64_t cap);
// One-time launch attributes on the current device (call before any capture).
nvr_status deform_setup();
// Workspace bytes (256-byte aligned base) for capacity cap; matrix_cores picks
// the fp16 / bf16 matrix-core kernels, det the deterministic table scatter.
size_t deform_ws_bytes(const nvr_grid_desc *g, int64_t cap, bool matrix_cores, bool det);
// table: fp32 master (float32 kernels); table_half: its fp16 copy (matrix-core
// kernels).  train: a training forward (the backward will follow on the same
// workspace, and reuses its encoding and tile counts).
nvr_status deform_fwd_dev(const nvr_grid_desc *g, bool matrix_cores, const int32_t *n_dev,
                          int64_t cap, const float *x, const float *theta, const float *table,
                          const void *table_half, const float *params, float *x_can, bool train,
                          bool det, void *ws, hipStream_t st);
// After a training forward on the same workspace.  dparams, dtable, dx and
// dtheta accumulate; dx and dtheta nullable.
struct ScatterTail;
// tail (nullable): second stream for the table gradient's accumulate (matrix
// cores, non-deterministic scatter only)
nvr_status deform_bwd_dev(const nvr_grid_desc *g, bool matrix_cores, const int32_t *n_dev,
                          int64_t cap, const float *x, const float *theta, const float *table,
                          const void *table_half, const float *params, const float *dx_can,
                          float *dparams, float *dtable, float *dx, float *dtheta, bool det,
                          void *ws, hipStream_t st, const ScatterTail *tail = nullptr);
int64_t deform_param_count();
// dst [cap][3] = sum of `parts` arrays src + p stride over the first *n_dev rows
nvr_status launch_sum_parts(const int32_t *n_dev, int64_t cap, int parts, int64_t stride,
                            const float *src, float *dst, hipStream_t st);

}  // namespace nvr
