// Pose-conditioned deformation network (Sec. 4.2, hybrid deformation; widths
// in Sec. 4.3): v_c = v_t + MLP([hash(v_t), theta]), 104 -> 4 x 128 -> 3,
// bias-free, ReLU on the hidden layers, float32.
//
// The encoding runs on the hash-grid kernels of this library (fp32 table);
// each layer is one rocBLAS sgemm over all points (row-major [n][width]
// activations, weights W[out][in] row-major as the flat parameter vector
// holds them); the small kernels here assemble the input, apply the ReLU and
// its mask, add the residual and split the input gradient.  The backward
// recomputes the forward into the workspace.
#include <algorithm>
#include <mutex>

#include <rocblas/rocblas.h>

#include "common.hpp"
#include "grid_dev.hpp"
#include "scatter_dev.hpp"

namespace nvr {
namespace {

constexpr int kFeat = 32, kPose = 72, kIn = kFeat + kPose, kWidth = 128, kHidden = 4;
constexpr int64_t kParams = (int64_t)kWidth * kIn + (int64_t)(kHidden - 1) * kWidth * kWidth +
                            3 * kWidth;

// The table gradient goes through the binned scatter (no float atomics; its
// records never read the table when no position gradient is asked of it), the
// position gradient through dn_encode_dx (one thread per point).
// The weight gradients reduce over all points; rocBLAS is given the points in
// kDwParts chunks of kDwChunk (a batched product into partials, summed by
// dn_reduce_partials), so that the reduction spreads over many workgroups.
constexpr int kDwChunk = 4096, kDwParts = 64;

struct DeformWs {
    float *feat, *a0, *h[kHidden], *dv, *dh0, *dh1, *da0, *dfeat, *partial;
    void *binned;
};

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

// Carves the workspace; returns its size (base may be null to only measure).
size_t carve(const nvr_grid_desc *g, int64_t n, char *base, DeformWs *w) {
    size_t off = 0;
    auto take = [&](size_t floats) {
        float *p = base ? reinterpret_cast<float *>(base + off) : nullptr;
        off += round_up(floats * sizeof(float));
        return p;
    };
    DeformWs t;
    t.feat = take((size_t)n * kFeat);
    t.a0 = take((size_t)n * kIn);
    for (int i = 0; i < kHidden; ++i) t.h[i] = take((size_t)n * kWidth);
    t.dv = take((size_t)n * 3);
    t.dh0 = take((size_t)n * kWidth);
    t.dh1 = take((size_t)n * kWidth);
    t.da0 = take((size_t)n * kIn);
    t.dfeat = take((size_t)n * kFeat);
    t.partial = take((size_t)kDwParts * kWidth * kWidth);   // largest layer: 128 x 128
    t.binned = take((nvr_encode_bwd_workspace(g, n) + sizeof(float) - 1) / sizeof(float));
    if (w) *w = t;
    return off;
}

__global__ void __launch_bounds__(256)
dn_concat(int64_t n, const float *__restrict__ feat, const float *__restrict__ theta,
          float *__restrict__ a0) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kIn;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / kIn;
        const int c = (int)(i - s * kIn);
        a0[i] = c < kFeat ? feat[s * kFeat + c] : theta[c - kFeat];
    }
}

__global__ void __launch_bounds__(256)
dn_relu(int64_t m, float *__restrict__ h) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        h[i] = h[i] > 0.f ? h[i] : 0.f;
}

__global__ void __launch_bounds__(256)
dn_relu_bwd(int64_t m, float *__restrict__ dh, const float *__restrict__ h) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        dh[i] = h[i] > 0.f ? dh[i] : 0.f;
}

__global__ void __launch_bounds__(256)
dn_residual(int64_t m, const float *__restrict__ x, const float *__restrict__ dv,
            float *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[i] + dv[i];
}

__global__ void __launch_bounds__(256)
dn_add(int64_t m, float *__restrict__ acc, const float *__restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        acc[i] += v[i];
}

__global__ void __launch_bounds__(256)
dn_split(int64_t n, const float *__restrict__ da0, float *__restrict__ dfeat) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kFeat;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / kFeat;
        dfeat[i] = da0[s * kIn + (i - s * kFeat)];
    }
}

// dtheta[c] += sum over points of da0[s][32 + c]: each workgroup sums a chunk
// of kThetaChunk points (lanes over the 72 components, so each row is read
// contiguously) and adds its partial with one atomic per component.
constexpr int kThetaChunk = 256;

__global__ void __launch_bounds__(128)
dn_theta_sum(int64_t n, const float *__restrict__ da0, float *__restrict__ dtheta) {
    const int c = threadIdx.x;
    if (c >= kPose) return;
    const int64_t s0 = (int64_t)blockIdx.x * kThetaChunk;
    const int64_t s1 = s0 + kThetaChunk < n ? s0 + kThetaChunk : n;
    float acc = 0.f;
    for (int64_t s = s0; s < s1; ++s) acc += da0[s * kIn + kFeat + c];
    atomicAdd(dtheta + c, acc);
}

// dW_partial[b] = (dY rows of chunk b)^T (X rows of chunk b), then summed.
__global__ void __launch_bounds__(256)
dn_reduce_partials(int64_t m, int32_t parts, const float *__restrict__ partial,
                   float *__restrict__ dW) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int b = 0; b < parts; ++b) acc += partial[(int64_t)b * m + i];
        dW[i] += acc;
    }
}

// Position gradient of the encoding alone (the table gradient is binned
// separately): one thread per point over all levels, so each point's gradient
// is summed in registers and added once, with no atomics.  dfeat is the
// row-major [n][2 L] feature gradient; fp32 table.
__global__ void __launch_bounds__(256)
dn_encode_dx(GridParams p, int64_t n, const float *__restrict__ x,
             const float2 *__restrict__ table, const float *__restrict__ dfeat,
             float *__restrict__ dx) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const float x0 = x[3 * s], x1 = x[3 * s + 1], x2 = x[3 * s + 2];
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
        for (int l = 0; l < p.L; ++l) {
            const LevelPos lp = level_pos(p, l, x0, x1, x2);
            const float g0 = dfeat[(s * p.L + l) * 2], g1 = dfeat[(s * p.L + l) * 2 + 1];
            float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float2 v = table[p.off[l] + corner_index(p, l, lp, k)];
                const float tg = v.x * g0 + v.y * g1;
                const float3 dw = corner_dweight(lp, k);
                d0 += dw.x * tg;
                d1 += dw.y * tg;
                d2 += dw.z * tg;
            }
            const float N = (float)p.res[l];
            if (lp.inside[0]) acc0 += d0 * N * (float)p.inv_side[0];
            if (lp.inside[1]) acc1 += d1 * N * (float)p.inv_side[1];
            if (lp.inside[2]) acc2 += d2 * N * (float)p.inv_side[2];
        }
        dx[3 * s] += acc0;
        dx[3 * s + 1] += acc1;
        dx[3 * s + 2] += acc2;
    }
}

// One rocBLAS handle per device, created on first use.
std::mutex g_blas_mu;
rocblas_handle g_blas[64] = {};

nvr_status blas_for(hipStream_t st, rocblas_handle *out) {
    int dev = 0;
    NVR_HIP(hipGetDevice(&dev));
    NVR_REQUIRE(dev >= 0 && dev < 64, NVR_EUNSUPPORTED, "device index %d out of range", dev);
    if (!g_blas[dev]) {
        NVR_REQUIRE(rocblas_create_handle(&g_blas[dev]) == rocblas_status_success, NVR_EHIP,
                    "rocblas_create_handle failed");
    }
    NVR_REQUIRE(rocblas_set_stream(g_blas[dev], st) == rocblas_status_success, NVR_EHIP,
                "rocblas_set_stream failed");
    *out = g_blas[dev];
    return NVR_OK;
}

// Row-major Y[n][out] (+)= X[n][in] W^T with W[out][in] row-major.
nvr_status gemm_fwd(rocblas_handle h, int64_t n, int out, int in, const float *W, const float *X,
                    float *Y) {
    const float one = 1.f, zero = 0.f;
    NVR_REQUIRE(rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, out, (int)n,
                              in, &one, W, in, X, in, &zero, Y, out) == rocblas_status_success,
                NVR_EHIP, "rocblas_sgemm failed");
    return NVR_OK;
}

// Row-major dX[n][in] = dY[n][out] W.
nvr_status gemm_dx(rocblas_handle h, int64_t n, int out, int in, const float *W, const float *dY,
                   float *dX) {
    const float one = 1.f, zero = 0.f;
    NVR_REQUIRE(rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, in, (int)n, out,
                              &one, W, in, dY, out, &zero, dX, in) == rocblas_status_success,
                NVR_EHIP, "rocblas_sgemm failed");
    return NVR_OK;
}

// Row-major dW[out][in] += dY^T X over the n points: whole chunks of kDwChunk
// points as one strided-batched product into `partial` (up to kDwParts chunks
// per pass) summed into dW, the remaining points as one product into dW.
nvr_status gemm_dw(rocblas_handle h, hipStream_t st, int64_t n, int out, int in, const float *dY,
                   const float *X, float *dW, float *partial) {
    const float one = 1.f, zero = 0.f;
    int64_t s = 0;
    while (n - s >= kDwChunk) {
        const int parts = (int)std::min<int64_t>(kDwParts, (n - s) / kDwChunk);
        NVR_REQUIRE(rocblas_sgemm_strided_batched(
                        h, rocblas_operation_none, rocblas_operation_transpose, in, out,
                        kDwChunk, &one, X + s * in, in, (rocblas_stride)kDwChunk * in,
                        dY + s * out, out, (rocblas_stride)kDwChunk * out, &zero, partial, in,
                        (rocblas_stride)in * out, parts) == rocblas_status_success,
                    NVR_EHIP, "rocblas_sgemm_strided_batched failed");
        const int64_t m = (int64_t)in * out;
        dn_reduce_partials<<<grid_for(m, 256, 1024), 256, 0, st>>>(m, parts, partial, dW);
        NVR_LAUNCHED();
        s += (int64_t)parts * kDwChunk;
    }
    if (s < n) {
        NVR_REQUIRE(rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, in, out,
                                  (int)(n - s), &one, X + s * in, in, dY + s * out, out, &one, dW,
                                  in) == rocblas_status_success,
                    NVR_EHIP, "rocblas_sgemm failed");
    }
    return NVR_OK;
}

const float *layer_w(const float *params, int i) {
    if (i == 0) return params;
    return params + (int64_t)kWidth * kIn + (int64_t)(i - 1) * kWidth * kWidth;
}

// Every check of both entry points, including those of the encoding and the
// binned scatter they call, so that nothing is launched before an error.
nvr_status check(const nvr_grid_desc *g, int64_t n, const void *ws) {
    NVR_REQUIRE(g != nullptr, NVR_EINVAL, "grid descriptor is NULL");
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(g->n_levels * g->n_features == kFeat, NVR_EUNSUPPORTED,
                "the deformation encoding must be 32 wide (levels x features)");
    NVR_REQUIRE(n >= 0 && n <= (1ll << 31) / kWidth, NVR_EINVAL, "n out of 0..2^24");
    NVR_REQUIRE(n == 0 || (ws && aligned(ws, 256)), NVR_EINVAL,
                "workspace NULL or not 256-byte aligned");
    const GridParams p = make_grid_params(g);
    NVR_TRY(scatter_check(p));
    NVR_REQUIRE((size_t)n * p.L * 8 < (1ull << 32), NVR_EINVAL, "too many contributions");
    return NVR_OK;
}

nvr_status forward(const nvr_grid_desc *g, int64_t n, const float *x, const float *theta,
                   const float *table, const float *params, const DeformWs &w, hipStream_t st,
                   rocblas_handle h) {
    NVR_TRY(nvr_encode_fwd(g, n, x, table, NVR_F32, w.feat, NVR_F32,
                           reinterpret_cast<nvr_stream>(st)));
    dn_concat<<<grid_for(n * kIn, 256, 16384), 256, 0, st>>>(n, w.feat, theta, w.a0);
    NVR_LAUNCHED();
    const float *in = w.a0;
    int width_in = kIn;
    for (int i = 0; i < kHidden; ++i) {
        NVR_TRY(gemm_fwd(h, n, kWidth, width_in, layer_w(params, i), in, w.h[i]));
        dn_relu<<<grid_for(n * kWidth, 256, 16384), 256, 0, st>>>(n * kWidth, w.h[i]);
        NVR_LAUNCHED();
        in = w.h[i];
        width_in = kWidth;
    }
    NVR_TRY(gemm_fwd(h, n, 3, kWidth, layer_w(params, kHidden), in, w.dv));
    return NVR_OK;
}

}  // namespace
}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_deform_workspace(const nvr_grid_desc *g, int64_t n) {
    if (g == nullptr || n < 0) return 0;
    return carve(g, n, nullptr, nullptr);
}

extern "C" int64_t nvr_deform_param_count(void) { return kParams; }

extern "C" nvr_status nvr_deform_fwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const float *theta, const float *table, const float *params,
                                     float *x_can, void *workspace, nvr_stream stream) {
    clear_error();
    NVR_TRY(check(g, n, workspace));
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && theta && table && params && x_can, NVR_EINVAL, "NULL array");
    const hipStream_t st = hs(stream);
    rocblas_handle h;
    std::lock_guard<std::mutex> lock(g_blas_mu);
    NVR_TRY(blas_for(st, &h));
    DeformWs w;
    carve(g, n, static_cast<char *>(workspace), &w);
    NVR_TRY(forward(g, n, x, theta, table, params, w, st, h));
    dn_residual<<<grid_for(n * 3, 256, 16384), 256, 0, st>>>(n * 3, x, w.dv, x_can);
    NVR_LAUNCHED();
    return NVR_OK;
}

extern "C" nvr_status nvr_deform_bwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const float *theta, const float *table, const float *params,
                                     const float *dx_can, float *dparams, float *dtable,
                                     float *dx, float *dtheta, void *workspace,
                                     nvr_stream stream) {
    clear_error();
    NVR_TRY(check(g, n, workspace));
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && theta && table && params && dx_can && dparams && dtable, NVR_EINVAL,
                "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(theta, 4) && aligned(table, 8) && aligned(params, 4) &&
                    aligned(dx_can, 4) && aligned(dparams, 4) && aligned(dtable, 8) &&
                    aligned(dx, 4) && aligned(dtheta, 4),
                NVR_EINVAL, "misaligned array");
    const hipStream_t st = hs(stream);
    rocblas_handle h;
    std::lock_guard<std::mutex> lock(g_blas_mu);
    NVR_TRY(blas_for(st, &h));
    DeformWs w;
    carve(g, n, static_cast<char *>(workspace), &w);
    NVR_TRY(forward(g, n, x, theta, table, params, w, st, h));
    // output layer: dW_out += dx_can^T h4; dh = dx_can W_out
    float *dW = dparams + (kParams - 3 * kWidth);
    NVR_TRY(gemm_dw(h, st, n, 3, kWidth, dx_can, w.h[kHidden - 1], dW, w.partial));
    NVR_TRY(gemm_dx(h, n, 3, kWidth, layer_w(params, kHidden), dx_can, w.dh0));
    float *dh = w.dh0, *dh_next = w.dh1;
    for (int i = kHidden - 1; i >= 0; --i) {
        dn_relu_bwd<<<grid_for(n * kWidth, 256, 16384), 256, 0, st>>>(n * kWidth, dh, w.h[i]);
        NVR_LAUNCHED();
        const int width_in = i == 0 ? kIn : kWidth;
        const float *in = i == 0 ? w.a0 : w.h[i - 1];
        float *dWi = dparams + (layer_w(params, i) - params);
        NVR_TRY(gemm_dw(h, st, n, kWidth, width_in, dh, in, dWi, w.partial));
        float *dst = i == 0 ? w.da0 : dh_next;
        NVR_TRY(gemm_dx(h, n, kWidth, width_in, layer_w(params, i), dh, dst));
        if (i > 0) {
            dh_next = dh;
            dh = dst;
        }
    }
    dn_split<<<grid_for(n * kFeat, 256, 16384), 256, 0, st>>>(n, w.da0, w.dfeat);
    NVR_LAUNCHED();
    if (dtheta) {
        dn_theta_sum<<<(unsigned)((n + kThetaChunk - 1) / kThetaChunk), 128, 0, st>>>(n, w.da0,
                                                                                  dtheta);
        NVR_LAUNCHED();
    }
    NVR_TRY(nvr_encode_bwd_binned(g, n, x, table, w.dfeat, dtable, nullptr, w.binned, stream));
    if (dx) {
        dn_encode_dx<<<grid_for(n, 256, 16384), 256, 0, st>>>(
            make_grid_params(g), n, x, reinterpret_cast<const float2 *>(table), w.dfeat, dx);
        NVR_LAUNCHED();
    }
    if (dx) {
        // the residual's identity: dx += dx_can
        dn_add<<<grid_for(n * 3, 256, 16384), 256, 0, st>>>(n * 3, dx, dx_can);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}
