// Volume-rendering compositing (forward, closed-form backward), the colour /
// depth loss, and the fused per-ray "composite -> loss -> composite backward"
// kernel used by the training step.  A group of 16 lanes composites one ray:
// its samples are loaded 16 at a time (coalesced), transmittance is
// exp(-prefix sum of tau) in fp32 from a scan over the group's lanes, and the
// backward's suffix sums come from a second scan.  A ray with samples in both
// fields' lists (merged by t, ties: the first list) is walked by the group's
// first lane in t order.
#include "common.hpp"
#include "composite_dev.hpp"

namespace nvr {

// Totals of ray r on every lane of its group.
__device__ __forceinline__ RayAcc group_ray_forward(const nvr_samples &a, const nvr_samples &b,
                                                    bool has_b, int64_t r, int gl, float t_stop) {
    const int64_t ia = a.off[r], iae = a.off[r + 1];
    const int64_t jb = has_b ? b.off[r] : 0, jbe = has_b ? b.off[r + 1] : 0;
    if (ia < iae && jb < jbe) {
        RayAcc acc{{0.f, 0.f, 0.f}, 0.f, 0.f};
        if (gl == 0) acc = ray_forward(a, b, has_b, r, t_stop);
        for (int k = 0; k < 3; ++k) acc.c[k] = group_bcast(acc.c[k], 0);
        acc.d = group_bcast(acc.d, 0);
        acc.tau = group_bcast(acc.tau, 0);
        return acc;
    }
    if (jb < jbe) return group_forward(b, jb, jbe, gl, t_stop);
    return group_forward(a, ia, iae, gl, t_stop);
}

__device__ __forceinline__ void group_ray_backward(const nvr_samples &a, const nvr_samples &b,
                                                   bool has_b, int64_t r, int gl, const float *C,
                                                   float D, const float *gc, float gd, float *dsa,
                                                   float *dra, float *dsb, float *drb) {
    const int64_t ia = a.off[r], iae = a.off[r + 1];
    const int64_t jb = has_b ? b.off[r] : 0, jbe = has_b ? b.off[r + 1] : 0;
    if (ia < iae && jb < jbe) {
        if (gl == 0) ray_backward(a, b, has_b, r, C, D, gc, gd, dsa, dra, dsb, drb);
    } else if (jb < jbe) {
        group_backward(b, jb, jbe, gl, C, D, gc, gd, dsb, drb);
    } else {
        group_backward(a, ia, iae, gl, C, D, gc, gd, dsa, dra);
    }
}

__global__ void __launch_bounds__(256)
composite_fwd_kernel(int64_t n_rays, nvr_samples a, nvr_samples b, bool has_b, float t_stop,
                     float *__restrict__ C, float *__restrict__ D, float *__restrict__ TN) {
    const int gl = threadIdx.x % kGroup;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kGroup);
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kGroup; r < n_rays;
         r += stride) {   // r is the same on the whole group
        RayAcc acc = group_ray_forward(a, b, has_b, r, gl, t_stop);
        if (gl == 0) {
            if (C) {
                C[3 * r] = acc.c[0];
                C[3 * r + 1] = acc.c[1];
                C[3 * r + 2] = acc.c[2];
            }
            if (D) D[r] = acc.d;
            if (TN) TN[r] = expf(-acc.tau);
        }
    }
}

__global__ void __launch_bounds__(256)
composite_bwd_kernel(int64_t n_rays, nvr_samples a, nvr_samples b, bool has_b,
                     const float *__restrict__ C, const float *__restrict__ D,
                     const float *__restrict__ dC, const float *__restrict__ dD,
                     float *__restrict__ dsa, float *__restrict__ dra, float *__restrict__ dsb,
                     float *__restrict__ drb) {
    const int gl = threadIdx.x % kGroup;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kGroup);
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kGroup; r < n_rays;
         r += stride) {   // r is the same on the whole group
        const float cc[3] = {C[3 * r], C[3 * r + 1], C[3 * r + 2]};
        const float gc[3] = {dC[3 * r], dC[3 * r + 1], dC[3 * r + 2]};
        group_ray_backward(a, b, has_b, r, gl, cc, D[r], gc, dD ? dD[r] : 0.f, dsa, dra, dsb, drb);
    }
}

__global__ void fill_zero(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

__device__ __forceinline__ void block_sum_atomic(float v, float *out) {
    __shared__ float red[8];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += red[i];
        unsafeAtomicAdd(out, s);
    }
}

// Block sum to partials[blockIdx.x] (plain store), summed later in a fixed order.
__device__ __forceinline__ void block_sum_store(float v, float *partials) {
    __shared__ float red[8];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += red[i];
        partials[blockIdx.x] = s;
    }
}

// out[0] = sum of partials[0, n) in a fixed order (one workgroup of 256).
__global__ void __launch_bounds__(256)
sum_in_order(int n, const float *__restrict__ partials, float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__device__ __forceinline__ float ray_loss(int64_t r, const float *C, float Dv, const float *C_t,
                                          const float *D_t, const float *mask, float lambda_d,
                                          float inv_R, float S, float *gc, float *gd) {
    const float m = mask ? mask[r] : 1.f;
    float e[3], l = 0.f;
    for (int k = 0; k < 3; ++k) {
        e[k] = C[k] - C_t[3 * r + k];
        l += e[k] * e[k];
        gc[k] = S * 2.f * m * e[k] * inv_R;
    }
    const float ed = D_t ? Dv - D_t[r] : Dv;
    l += lambda_d * ed * ed;
    *gd = S * 2.f * lambda_d * m * ed * inv_R;
    return m * l * inv_R;
}

__global__ void __launch_bounds__(256)
loss_kernel(int64_t n_rays, const float *__restrict__ C, const float *__restrict__ D,
            const float *__restrict__ C_t, const float *__restrict__ D_t,
            const float *__restrict__ mask, float lambda_d, const float *__restrict__ scale,
            float *__restrict__ loss, float *__restrict__ dC, float *__restrict__ dD) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float l = 0.f;
    if (r < n_rays) {
        const float S = scale ? *scale : 1.f;
        float gc[3], gd;
        l = ray_loss(r, C + 3 * r, D[r], C_t, D_t, mask, lambda_d, 1.f / (float)n_rays, S, gc, &gd);
        for (int k = 0; k < 3; ++k) dC[3 * r + k] = gc[k];
        dD[r] = gd;
    }
    block_sum_atomic(l, loss);
}

// Training-step fusion: forward walk, loss, backward walk of the same ray.
__global__ void __launch_bounds__(256)
composite_loss_fused(int64_t n_rays, nvr_samples a, nvr_samples b, bool has_b,
                     const float *__restrict__ C_t, const float *__restrict__ D_t,
                     const float *__restrict__ mask, float lambda_d,
                     const nvr_train_state *__restrict__ state, float *__restrict__ loss,
                     float *__restrict__ C_out, float *__restrict__ D_out,
                     float *__restrict__ dsa, float *__restrict__ dra, float *__restrict__ dsb,
                     float *__restrict__ drb, float *__restrict__ partials) {
    const int gl = threadIdx.x % kGroup;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kGroup);
    float l = 0.f;
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kGroup; r < n_rays;
         r += stride) {   // r is the same on the whole group
        RayAcc acc = group_ray_forward(a, b, has_b, r, gl, 0.f);
        const float S = state ? state->loss_scale : 1.f;
        float gc[3], gd;
        const float lr = ray_loss(r, acc.c, acc.d, C_t, D_t, mask, lambda_d, 1.f / (float)n_rays, S,
                                  gc, &gd);
        if (gl == 0) l += lr;            // counted once per ray
        if (gl == 0) {
            if (C_out) {
                C_out[3 * r] = acc.c[0];
                C_out[3 * r + 1] = acc.c[1];
                C_out[3 * r + 2] = acc.c[2];
            }
            if (D_out) D_out[r] = acc.d;
        }
        if (dsa) group_ray_backward(a, b, has_b, r, gl, acc.c, acc.d, gc, gd, dsa, dra, dsb, drb);
    }
    if (partials) block_sum_store(l, partials);
    else block_sum_atomic(l, loss);
}

nvr_status launch_fill_zero(float *p, int64_t n, hipStream_t st) {
    if (n <= 0) return NVR_OK;
    fill_zero<<<grid_for(n, 256, 2048), 256, 0, st>>>(p, n);
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status launch_composite_loss(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                 const float *C_t, const float *D_t, const float *mask,
                                 float lambda_d, const nvr_train_state *state, float *loss,
                                 float *C_out, float *D_out, float *dsa, float *dra, float *dsb,
                                 float *drb, hipStream_t st, int blocks, float *partials) {
    if (n_rays <= 0 || partials == nullptr) NVR_TRY(launch_fill_zero(loss, 1, st));
    if (n_rays <= 0) return NVR_OK;
    nvr_samples bb = b ? *b : nvr_samples{};
    const unsigned gr = grid_for(n_rays * kGroup, 256, blocks > 0 ? blocks : kMaxLossBlocks);
    composite_loss_fused<<<gr, 256, 0, st>>>(
        n_rays, a, bb, b != nullptr, C_t, D_t, mask, lambda_d, state, loss, C_out, D_out, dsa, dra,
        dsb, drb, partials);
    NVR_LAUNCHED();
    if (partials) {
        sum_in_order<<<1, 256, 0, st>>>((int)gr, partials, loss);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}

nvr_status launch_composite_fwd(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                float t_stop, float *C, float *D, float *TN, hipStream_t st) {
    if (n_rays <= 0) return NVR_OK;
    nvr_samples bb = b ? *b : nvr_samples{};
    composite_fwd_kernel<<<grid_for(n_rays * kGroup, 256, 65536), 256, 0, st>>>(
        n_rays, a, bb, b != nullptr, t_stop, C, D, TN);
    NVR_LAUNCHED();
    return NVR_OK;
}

static nvr_status check_samples(const nvr_samples *s, const char *name) {
    NVR_REQUIRE(s->off && s->sigma && s->rgb && s->t && s->dt, NVR_EINVAL,
                "sample list %s has a NULL array", name);
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_composite_fwd(int64_t n_rays, const nvr_samples *a, const nvr_samples *b,
                                        float t_stop, float *C, float *D, float *TN,
                                        nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n_rays >= 0, NVR_EINVAL, "n_rays < 0");
    NVR_REQUIRE(a != nullptr, NVR_EINVAL, "sample list a is NULL");
    NVR_REQUIRE(t_stop >= 0.f && t_stop < 1.f, NVR_EINVAL, "t_stop out of [0,1)");
    if (n_rays == 0) return NVR_OK;
    NVR_TRY(check_samples(a, "a"));
    if (b) NVR_TRY(check_samples(b, "b"));
    return launch_composite_fwd(n_rays, *a, b, t_stop, C, D, TN, hs(stream));
}

extern "C" nvr_status nvr_composite_bwd(int64_t n_rays, const nvr_samples *a, const nvr_samples *b,
                                        const float *C, const float *D, const float *dC,
                                        const float *dD, float *dsigma_a, float *drgb_a,
                                        float *dsigma_b, float *drgb_b, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n_rays >= 0, NVR_EINVAL, "n_rays < 0");
    NVR_REQUIRE(a != nullptr, NVR_EINVAL, "sample list a is NULL");
    if (n_rays == 0) return NVR_OK;
    NVR_TRY(check_samples(a, "a"));
    if (b) {
        NVR_TRY(check_samples(b, "b"));
        NVR_REQUIRE(dsigma_b && drgb_b, NVR_EINVAL, "b outputs are NULL");
    }
    NVR_REQUIRE(C && D && dC && dsigma_a && drgb_a, NVR_EINVAL, "NULL array");
    nvr_samples bb = b ? *b : nvr_samples{};
    composite_bwd_kernel<<<grid_for(n_rays * kGroup, 256, 65536), 256, 0, hs(stream)>>>(
        n_rays, *a, bb, b != nullptr, C, D, dC, dD, dsigma_a, drgb_a, dsigma_b, drgb_b);
    NVR_LAUNCHED();
    return NVR_OK;
}

extern "C" nvr_status nvr_loss(int64_t n_rays, const float *C, const float *D, const float *C_t,
                               const float *D_t, const float *mask, float lambda_d,
                               const float *loss_scale_dev, float *loss_dev, float *dC, float *dD,
                               nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n_rays >= 0, NVR_EINVAL, "n_rays < 0");
    NVR_REQUIRE(loss_dev, NVR_EINVAL, "loss_dev is NULL");
    hipStream_t st = hs(stream);
    NVR_TRY(launch_fill_zero(loss_dev, 1, st));
    if (n_rays == 0) return NVR_OK;
    NVR_REQUIRE(C && D && C_t && dC && dD, NVR_EINVAL, "NULL array");
    loss_kernel<<<(unsigned)((n_rays + 255) / 256), 256, 0, st>>>(n_rays, C, D, C_t, D_t, mask,
                                                                 lambda_d, loss_scale_dev,
                                                                 loss_dev, dC, dD);
    NVR_LAUNCHED();
    return NVR_OK;
}
