// Plain float32 density + colour networks: one launch per layer, every
// layer's activations stored unit-major ([unit][capacity]) in HBM, backward
// as per-layer data-gradient launches plus a tiled weight-gradient reduction.
// This is the unfused baseline the fused bf16 MFMA path is measured against.
#include "common.hpp"
#include "mlp_dev.hpp"
#include "sh_dev.hpp"

namespace nvr {

constexpr int kPlainBlock = 256;
constexpr int kMaxW = 64;

// A strided 2-D view: element (unit u, sample s) at p[u * su + s * ss].
struct View {
    float *p;
    int64_t su, ss;
    __device__ __forceinline__ float &at(int u, int64_t s) const { return p[u * su + s * ss]; }
};

enum { ACT_NONE = 0, ACT_RELU = 1, ACT_SIGMOID = 2 };

// Y = act(W X) per sample; weights are wave-uniform (scalar loads).
template <int ACT>
__global__ void __launch_bounds__(kPlainBlock)
linear_fwd(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, int IN, int OUT,
           View X, const float *__restrict__ W, View Y) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
        float x[kMaxW];
#pragma unroll
        for (int i = 0; i < kMaxW; ++i)
            if (i < IN) x[i] = X.at(i, s);
#pragma unroll
        for (int o = 0; o < kMaxW; ++o) {
            if (o < OUT) {
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i < kMaxW; ++i)
                    if (i < IN) acc += W[o * IN + i] * x[i];
                if (ACT == ACT_RELU) acc = fmaxf(acc, 0.f);
                if (ACT == ACT_SIGMOID) acc = 1.f / (1.f + expf(-acc));
                Y.at(o, s) = acc;
            }
        }
    }
}

// dX = (W^T dY) [* (X > 0) when X came out of a ReLU]
__global__ void __launch_bounds__(kPlainBlock)
linear_dgrad(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, int IN, int OUT,
             View dY, const float *__restrict__ W, View X, int mask_relu, View dX) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
        float g[kMaxW];
#pragma unroll
        for (int o = 0; o < kMaxW; ++o)
            if (o < OUT) g[o] = dY.at(o, s);
#pragma unroll
        for (int i = 0; i < kMaxW; ++i) {
            if (i < IN) {
                float acc = 0.f;
#pragma unroll
                for (int o = 0; o < kMaxW; ++o)
                    if (o < OUT) acc += W[o * IN + i] * g[o];
                if (mask_relu && !(X.at(i, s) > 0.f)) acc = 0.f;
                dX.at(i, s) = acc;
            }
        }
    }
}

// dW[o][i] += sum_s dY[o][s] X[i][s]: thread = 4x4 tile of (o, i), workgroup =
// a chunk of samples, one atomic per weight per workgroup.
constexpr int kWgradChunk = 8192;
__global__ void __launch_bounds__(256)
linear_wgrad(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, int IN, int OUT,
             View dY, View X, float *__restrict__ dW) {
    const int64_t count = count_of(n, n_dev, cap);
    const int o0 = (threadIdx.x / 16) * 4, i0 = (threadIdx.x % 16) * 4;
    if (o0 >= OUT || i0 >= IN) return;
    float acc[4][4] = {};
    for (int64_t c = blockIdx.x * (int64_t)kWgradChunk; c < count; c += (int64_t)gridDim.x * kWgradChunk) {
        const int64_t e = c + kWgradChunk < count ? c + kWgradChunk : count;
        for (int64_t s = c; s < e; ++s) {
            float a[4], b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                a[k] = (o0 + k < OUT) ? dY.at(o0 + k, s) : 0.f;
                b[k] = (i0 + k < IN) ? X.at(i0 + k, s) : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (o0 + u < OUT && i0 + v < IN && acc[u][v] != 0.f)
                unsafeAtomicAdd(dW + (o0 + u) * IN + (i0 + v), acc[u][v]);
}

// sigma = exp(clamp(o_0)), and the SH rows of the colour input.
__global__ void __launch_bounds__(kPlainBlock)
sigma_sh_fwd(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, View CIN, int dout,
             int sh_degree, const float *__restrict__ dirs, const int32_t *__restrict__ ray_id,
             float *__restrict__ sigma) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
        const float o0 = CIN.at(0, s);
        sigma[s] = expf(fminf(fmaxf(o0, -kSigmaClamp), kSigmaClamp));
        const int64_t r = ray_id ? ray_id[s] : s;
        float sh[16];
        sh_eval(dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2], sh_degree, sh);
        for (int k = 0; k < sh_degree * sh_degree; ++k) CIN.at(dout + k, s) = sh[k];
    }
}

// dZ = drgb * rgb * (1 - rgb), with rgb the stored sigmoid output.
__global__ void __launch_bounds__(kPlainBlock)
sigmoid_bwd(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, const float *__restrict__ rgb,
            const float *__restrict__ drgb, View dZ) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = rgb[3 * s + c];
            dZ.at(c, s) = drgb[3 * s + c] * v * (1.f - v);
        }
    }
}

// dO_0 += dsigma * sigma where o_0 was inside the clamp.
__global__ void __launch_bounds__(kPlainBlock)
sigma_bwd(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, View CIN,
          const float *__restrict__ sigma, const float *__restrict__ dsigma, View dCIN) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
        const float o0 = CIN.at(0, s);
        if (fabsf(o0) < kSigmaClamp) dCIN.at(0, s) += dsigma[s] * sigma[s];
    }
}

// ---------------------------------------------------------------- host
// Workspace (floats, unit-major [unit][cap]): every layer input except the
// encoding, then one gradient buffer per layer output and one per input.
struct PlainWs {
    float *act[2 * kMaxLayers];   // input of layer k (k >= 1); act[0] unused
    float *grad[2 * kMaxLayers];  // gradient w.r.t. the output of layer k
    float *gin;                   // gradient w.r.t. the colour input
};

static int64_t plain_units(const Net &net) {
    int64_t u = 0;
    for (int k = 1; k < net.n_layers; ++k) u += net.in[k];   // stored inputs
    for (int k = 0; k < net.n_layers; ++k) u += net.out[k];  // output gradients
    u += net.in[net.n_density];                              // colour-input gradient
    return u;
}

size_t plain_workspace(const Net &net, int64_t cap) {
    return sizeof(float) * (size_t)plain_units(net) * (size_t)cap;
}

static PlainWs carve(const Net &net, float *ws, int64_t cap) {
    PlainWs w{};
    float *p = ws;
    for (int k = 1; k < net.n_layers; ++k) {
        w.act[k] = p;
        p += (size_t)net.in[k] * cap;
    }
    for (int k = 0; k < net.n_layers; ++k) {
        w.grad[k] = p;
        p += (size_t)net.out[k] * cap;
    }
    w.gin = p;
    // the density outputs' gradient is the first dout rows of the colour-input gradient
    w.grad[net.n_density - 1] = w.gin;
    return w;
}

static View um(float *p, int64_t cap) { return View{p, cap, 1}; }

// Forward: feat viewed by `F` (unit i of sample s).  Stores activations.
nvr_status plain_forward(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, View F,
                         const float *dirs, const int32_t *ray_id, const float *params,
                         float *sigma, float *rgb, float *ws, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    PlainWs w = carve(net, ws, cap);
    const unsigned gr = grid_for(cap, kPlainBlock, 4096);
    const int nd = net.n_density;
    View in = F;
    for (int k = 0; k < net.n_layers; ++k) {
        const float *W = params + net.woff[k];
        const bool last_density = (k == nd - 1);
        const bool last = (k == net.n_layers - 1);
        View out = last ? View{rgb, 1, 3} : um(w.act[k + 1], cap);
        if (last)
            linear_fwd<ACT_SIGMOID><<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, net.in[k], net.out[k], in, W, out);
        else if (last_density)
            linear_fwd<ACT_NONE><<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, net.in[k], net.out[k], in, W, out);
        else
            linear_fwd<ACT_RELU><<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, net.in[k], net.out[k], in, W, out);
        NVR_LAUNCHED();
        if (last_density) {
            sigma_sh_fwd<<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, out, net.dout, net.sh_degree, dirs,
                                                    ray_id, sigma);
            NVR_LAUNCHED();
        }
        in = out;
    }
    return NVR_OK;
}

// Backward from dsigma, drgb; needs the activations plain_forward stored.
nvr_status plain_backward(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, View F,
                          const float *params, const float *sigma, const float *rgb,
                          const float *dsigma, const float *drgb, float *dparams, View dF,
                          bool want_dfeat, float *ws, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    PlainWs w = carve(net, ws, cap);
    const unsigned gr = grid_for(cap, kPlainBlock, 4096);
    const unsigned grw = grid_for(cap, kWgradChunk, 1024);
    const int nd = net.n_density;
    const int L = net.n_layers;
    sigmoid_bwd<<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, rgb, drgb, um(w.grad[L - 1], cap));
    NVR_LAUNCHED();
    for (int k = L - 1; k >= 0; --k) {
        const float *W = params + net.woff[k];
        View X = k == 0 ? F : um(w.act[k], cap);
        View dY = um(w.grad[k], cap);
        linear_wgrad<<<grw, 256, 0, st>>>(n, n_dev, cap, net.in[k], net.out[k], dY, X,
                                         dparams + net.woff[k]);
        NVR_LAUNCHED();
        if (k == 0 && !want_dfeat) break;
        View dX;
        int mask = 0;
        if (k == 0) dX = dF;
        else if (k == nd) dX = um(w.gin, cap);             // colour input: o and SH
        else {
            dX = um(w.grad[k - 1], cap);
            mask = 1;                                       // input came out of a ReLU
        }
        linear_dgrad<<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, net.in[k], net.out[k], dY, W, X,
                                                mask, dX);
        NVR_LAUNCHED();
        if (k == nd) {
            // density outputs: gradient rows 0..dout-1 of the colour input, plus sigma
            sigma_bwd<<<gr, kPlainBlock, 0, st>>>(n, n_dev, cap, um(w.act[nd], cap), sigma, dsigma,
                                                 um(w.gin, cap));
            NVR_LAUNCHED();
        }
    }
    return NVR_OK;
}

}  // namespace nvr

#include "launch.hpp"

namespace nvr {

static View as_view(PlainView v) { return View{v.p, v.su, v.ss}; }

nvr_status plain_fwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, PlainView F,
                     const float *dirs, const int32_t *ray_id, const float *params, float *sigma,
                     float *rgb, float *ws, hipStream_t st) {
    return plain_forward(net, n, n_dev, cap, as_view(F), dirs, ray_id, params, sigma, rgb, ws, st);
}

nvr_status plain_bwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap, PlainView F,
                     const float *params, const float *sigma, const float *rgb,
                     const float *dsigma, const float *drgb, float *dparams, PlainView dF,
                     bool want_dfeat, float *ws, hipStream_t st) {
    return plain_backward(net, n, n_dev, cap, as_view(F), params, sigma, rgb, dsigma, drgb, dparams,
                          as_view(dF), want_dfeat, ws, st);
}

}  // namespace nvr
