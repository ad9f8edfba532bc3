// Adam with loss scaling and the device-resident step state (no host sync):
// nvr_state_begin marks the step finite, nvr_check_finite clears the flag on
// any non-finite gradient, nvr_adam updates (or only zeroes the gradient when
// the step is skipped), nvr_state_end advances the step count or halves the
// loss scale.
#include "common.hpp"

#include <cmath>
#include "optim_dev.hpp"

namespace nvr {

__global__ void state_begin_kernel(nvr_train_state *s) { s->finite = 1; }

__global__ void state_end_kernel(nvr_train_state *s) {
    if (s->finite) s->step += 1;
    else s->loss_scale *= 0.5f;
}

__global__ void __launch_bounds__(256)
check_finite_kernel(int64_t n, const float *__restrict__ g, nvr_train_state *s) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(g[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) s->finite = 0;
}

template <int COPY>  // 0 none, 1 float16, 2 bfloat16
__global__ void __launch_bounds__(256)
adam_kernel(AdamParams a, int64_t n, float *__restrict__ p, float *__restrict__ m,
            float *__restrict__ v, float *__restrict__ grad, int skip_zero,
            const nvr_train_state *__restrict__ st, uint16_t *__restrict__ copy) {
    const int finite = st->finite;
    const float inv_s = 1.f / st->loss_scale;
    const int k = st->step + 1;
    const float bc1 = 1.f - powf(a.b1, (float)k);
    const float bc2 = 1.f - powf(a.b2, (float)k);
    const float lr = a.lr * exp2f(a.log2_decay * (float)(k - 1));   // lr decay^(k-1)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[i] * inv_s;
        grad[i] = 0.f;
        if (!finite) continue;
        if (skip_zero && g == 0.f) continue;
        const float mi = a.b1 * m[i] + (1.f - a.b1) * g;
        const float vi = a.b2 * v[i] + (1.f - a.b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + a.eps);
        p[i] = pi;
        if (COPY == 1) copy[i] = f32_to_f16_bits(pi);
        if (COPY == 2) copy[i] = f32_to_bf16_bits(pi);
    }
}

__global__ void __launch_bounds__(256)
convert_kernel(int64_t n, const float *__restrict__ p, uint16_t *__restrict__ out, int to_bf16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = to_bf16 ? f32_to_bf16_bits(p[i]) : f32_to_f16_bits(p[i]);
}

nvr_status launch_state_begin(nvr_train_state *s, hipStream_t st) {
    state_begin_kernel<<<1, 1, 0, st>>>(s);
    NVR_LAUNCHED();
    return NVR_OK;
}
nvr_status launch_state_end(nvr_train_state *s, hipStream_t st) {
    state_end_kernel<<<1, 1, 0, st>>>(s);
    NVR_LAUNCHED();
    return NVR_OK;
}
nvr_status launch_check_finite(int64_t n, const float *g, nvr_train_state *s, hipStream_t st) {
    if (n <= 0) return NVR_OK;
    check_finite_kernel<<<grid_for(n, 256, 2048), 256, 0, st>>>(n, g, s);
    NVR_LAUNCHED();
    return NVR_OK;
}
AdamParams adam_params(const nvr_adam_desc &a) {
    const bool decays = a.lr_decay > 0.f && a.lr_decay < 1.f;
    return AdamParams{a.lr, a.beta1, a.beta2, a.eps,
                      decays ? (float)std::log2((double)a.lr_decay) : 0.f};
}

nvr_status launch_adam(const AdamParams &a, int64_t n, float *p, float *m, float *v, float *grad,
                       int skip_zero, const nvr_train_state *s, void *copy, nvr_dtype copy_dtype,
                       hipStream_t st) {
    if (n <= 0) return NVR_OK;
    const unsigned gr = grid_for(n, 256, 4096);
    if (copy == nullptr)
        adam_kernel<0><<<gr, 256, 0, st>>>(a, n, p, m, v, grad, skip_zero, s, nullptr);
    else if (copy_dtype == NVR_F16)
        adam_kernel<1><<<gr, 256, 0, st>>>(a, n, p, m, v, grad, skip_zero, s, (uint16_t *)copy);
    else
        adam_kernel<2><<<gr, 256, 0, st>>>(a, n, p, m, v, grad, skip_zero, s, (uint16_t *)copy);
    NVR_LAUNCHED();
    return NVR_OK;
}
nvr_status launch_convert(int64_t n, const float *p, void *out, nvr_dtype dt, hipStream_t st) {
    if (n <= 0) return NVR_OK;
    convert_kernel<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, p, (uint16_t *)out, dt == NVR_BF16);
    NVR_LAUNCHED();
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_state_begin(nvr_train_state *state_dev, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(state_dev, NVR_EINVAL, "state is NULL");
    return launch_state_begin(state_dev, hs(stream));
}

extern "C" nvr_status nvr_check_finite(int64_t n, const float *g, nvr_train_state *state_dev,
                                       nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n >= 0 && state_dev && (n == 0 || g), NVR_EINVAL, "bad arguments");
    return launch_check_finite(n, g, state_dev, hs(stream));
}

extern "C" nvr_status nvr_adam(const nvr_adam_desc *a, int64_t n, float *param, float *m, float *v,
                               float *grad, int32_t skip_zero, const nvr_train_state *state_dev,
                               void *copy, nvr_dtype copy_dtype, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(a && state_dev, NVR_EINVAL, "NULL descriptor or state");
    NVR_REQUIRE(n >= 0, NVR_EINVAL, "n < 0");
    NVR_REQUIRE(a->lr > 0.f && a->beta1 >= 0.f && a->beta1 < 1.f && a->beta2 >= 0.f &&
                    a->beta2 < 1.f && a->eps >= 0.f && a->lr_decay >= 0.f && a->lr_decay <= 1.f,
                NVR_EINVAL, "bad Adam hyper-parameters");
    NVR_REQUIRE(copy == nullptr || copy_dtype == NVR_F16 || copy_dtype == NVR_BF16, NVR_EINVAL,
                "copy dtype must be F16 or BF16");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(param && m && v && grad, NVR_EINVAL, "NULL array");
    const AdamParams ap = adam_params(*a);
    return launch_adam(ap, n, param, m, v, grad, skip_zero, state_dev, copy, copy_dtype, hs(stream));
}

extern "C" nvr_status nvr_state_end(nvr_train_state *state_dev, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(state_dev, NVR_EINVAL, "state is NULL");
    return launch_state_end(state_dev, hs(stream));
}
