// Internal launchers shared between the kernel files and the step driver.
#pragma once
#include "common.hpp"
#include "grid_dev.hpp"
#include "mlp_dev.hpp"
#include "composite_dev.hpp"
#include "optim_dev.hpp"

namespace nvr {

// march.hip
struct MarchParams;
nvr_status march_desc_check(const nvr_march_desc *m);
size_t march_ws_bytes(int64_t n_rays);
nvr_status run_march(const nvr_march_desc *m, int64_t n_rays, int64_t begin, int64_t end,
                     const float *o, const float *d, const uint32_t *occ, int64_t capacity,
                     int32_t *off, int32_t *ray_id, float *t, float *dt, float *x, int32_t *n_dev,
                     int32_t *ws, hipStream_t st);

// warp.hip
struct WarpParams;
nvr_status run_warp_fwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t cap,
                        const int32_t *n_dev, const float *x, float *xc, hipStream_t st);
nvr_status run_warp_bwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t cap,
                        const int32_t *n_dev, const float *x, const float *gz, int n_parts,
                        int64_t part_stride, float *d_dq, float *d_bones, hipStream_t st);

// mlp_plain.hip
struct PlainView {
    float *p;
    int64_t su, ss;
};
size_t plain_workspace(const Net &net, int64_t cap);
nvr_status plain_fwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, PlainView F,
                     const float *dirs, const int32_t *ray_id, const float *params, float *sigma,
                     float *rgb, float *ws, hipStream_t st);
nvr_status plain_bwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, PlainView F,
                     const float *params, const float *sigma, const float *rgb,
                     const float *dsigma, const float *drgb, float *dparams, PlainView dF,
                     bool want_dfeat, float *ws, hipStream_t st);

// mlp_mfma.hip
struct MfmaNet;
nvr_status mfma_check(const Net &net);
size_t mfma_ws_bytes(const Net &net, int64_t cap);
// blocks: workgroups of the persistent network kernels (0: default; the
// backward's is capped by its workspace); dparams == nullptr skips the final
// reduction of the per-workgroup weight-gradient partials.
// f16: fp16 forward (feat fp16, params the fp32 masters); otherwise bf16
// forward (feat bf16, params the bf16 copy).  Backward products are bf16.
// sh_rays: the per-ray SH coefficients of launch_sh_rays for the same rays as
// dirs (ray_id indexes both), or nullptr to evaluate them per sample.
nvr_status mfma_fwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap,
                    const uint16_t *feat, bool planar, const float *dirs, const int32_t *ray_id,
                    const void *params, bool f16, float *sigma, float *rgb, hipStream_t st,
                    int blocks = 0, const float *sh_rays = nullptr);
nvr_status mfma_bwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap,
                    const uint16_t *feat, bool planar, const float *dirs, const int32_t *ray_id,
                    const void *params, bool f16, const float *dsigma, const float *drgb,
                    float *dparams, float *dfeat, void *ws, hipStream_t st, int blocks = 0,
                    const float *sh_rays = nullptr);
// out[n_rays][16] = SH coefficients of each ray's direction (0 past the
// network's coefficient count), 16-byte aligned.
nvr_status launch_sh_rays(const Net &net, int64_t n_rays, const float *dirs, float *out,
                          hipStream_t st);

}  // namespace nvr
