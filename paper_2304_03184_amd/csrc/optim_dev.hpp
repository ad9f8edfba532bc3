// Optimiser launchers (optim.hip).
#pragma once
#include "common.hpp"

namespace nvr {

struct AdamParams {
    float lr, b1, b2, eps;
    float log2_decay;   // log2 of the per-update learning-rate factor (0: constant)
};
// AdamParams of a descriptor (lr_decay <= 0 or 1: constant learning rate)
AdamParams adam_params(const nvr_adam_desc &a);

nvr_status launch_state_begin(nvr_train_state *s, hipStream_t st);
nvr_status launch_state_end(nvr_train_state *s, hipStream_t st);
nvr_status launch_check_finite(int64_t n, const float *g, nvr_train_state *s, hipStream_t st);
nvr_status launch_adam(const AdamParams &a, int64_t n, float *p, float *m, float *v, float *grad,
                       int skip_zero, const nvr_train_state *s, void *copy, nvr_dtype copy_dtype,
                       hipStream_t st);
nvr_status launch_convert(int64_t n, const float *p, void *out, nvr_dtype dt, hipStream_t st);

}  // namespace nvr
