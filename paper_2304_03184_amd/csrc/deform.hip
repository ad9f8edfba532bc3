// Pose-conditioned deformation network (Sec. 4.2, hybrid deformation; widths
// in Sec. 4.3): v_c = v_t + MLP([hash(v_t), theta]), 104 -> 4 x 128 -> 3,
// bias-free, ReLU on the hidden layers.
//
// The encoding runs on the hash-grid kernels of this library (fp32 table).
// Two paths share the entry points: a float32 one (each layer one tiled
// product over the points, row-major [n][width] activations, weights W[out][in]
// row-major as the flat parameter vector holds them; weight gradients formed
// as per-chunk partials summed in chunk order) and the matrix-core one below.
// Every kernel takes the point count from the host or from a device word (at
// most a capacity), so the training step can call both without reading the
// sample count back; the backward recomputes the forward into the workspace.
#include <algorithm>
#include <atomic>

#include "common.hpp"
#include "deform_dev.hpp"
#include "grid_dev.hpp"
#include "scatter_dev.hpp"

namespace nvr {
namespace {

constexpr int kFeat = 32, kPose = 72, kIn = kFeat + kPose, kWidth = 128, kHidden = 4;
constexpr int64_t kParams = (int64_t)kWidth * kIn + (int64_t)(kHidden - 1) * kWidth * kWidth +
                            3 * kWidth;

// The table gradient goes through the binned scatter (its records never read
// the table when no position gradient is asked of it), the position gradient
// through dn_encode_dx (one thread per point).
constexpr int kMmT = 64, kMmK = 16;     // product tiles: 64 x 64 outputs, 16-deep slices
constexpr int kMmParts = 256;           // most point chunks of a weight gradient
constexpr int kThetaChunk = 256;        // points per pose-gradient partial

struct DeformWs {
    float *feat, *a0, *h[kHidden], *dv, *dh0, *dh1, *da0, *dfeat, *partial, *theta_part;
    void *binned;
};

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of the matrix-core path (carved like the float32 one).
struct DeformMfmaWs {
    uint16_t *feat;      // [8][n][4] fp16 encoding, level-group layout of the split gather
    float *bias;         // [128] pose term
    uint4 *fwd, *bwd;    // weight fragments
    uint16_t *hbuf, *zbuf;
    uint32_t *mwords;    // [block][4][64] ReLU mask words of the training forward
    float *dfeat;        // [8][n][4] encoding gradient, same layout
    float *dx_parts;     // [8][n][3] position-gradient partials of the level groups
    uint32_t *jac;       // [8][n][6] the training gather's spatial derivatives (fp16 pairs)
    float *partial;      // [kDwGrid][128][144] weight-gradient partials
    uint32_t *half;      // fp16 copy of the table (public entry points)
    void *binned;        // binned table-gradient scatter
};
constexpr int kDwGrid = 512;

size_t carve_mfma(const nvr_grid_desc *g, int64_t n, bool det, char *base, DeformMfmaWs *w);

// Matrix-core path: the encoding slot j of lane group g reads level-group
// planes 2g and 2g+1 (levels 2g, 2g+8, then 2g+1, 2g+9, two features each),
// which is feature dfp(g, j) of the standard [level][feature] order.
__host__ __device__ __forceinline__ int dfp(int g, int j) {
    return 4 * g + (j & 1) + ((j >> 1) & 1) * 16 + (j >> 2) * 2;
}

// point chunks of the float32 weight gradients at capacity cap
int mm_parts(int64_t cap) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMmParts, cap / 1024));
}

// Carves the workspace of capacity n; returns its size (base may be null to
// only measure).
size_t carve(const nvr_grid_desc *g, int64_t n, bool det, char *base, DeformWs *w) {
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
    t.partial = take((size_t)mm_parts(n) * kWidth * kWidth);  // largest layer: 128 x 128
    t.theta_part = take((size_t)((n + kThetaChunk - 1) / kThetaChunk + 1) * kPose);
    t.binned = take((scatter_rows_ws_bytes(make_grid_params(g), n, det) + sizeof(float) - 1) /
                    sizeof(float));
    if (w) *w = t;
    return off;
}

__global__ void __launch_bounds__(256)
dn_concat(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
          const float *__restrict__ feat, const float *__restrict__ theta, float *__restrict__ a0) {
    n = count_of(n, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kIn;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / kIn;
        const int c = (int)(i - s * kIn);
        a0[i] = c < kFeat ? feat[s * kFeat + c] : theta[c - kFeat];
    }
}

// dh = h > 0 ? dh : 0 over the first count rows of width w
__global__ void __launch_bounds__(256)
dn_relu_bwd(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, int w,
            float *__restrict__ dh, const float *__restrict__ h) {
    const int64_t m = count_of(n, n_dev, cap) * w;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        dh[i] = h[i] > 0.f ? dh[i] : 0.f;
}

__global__ void __launch_bounds__(256)
dn_residual(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
            const float *__restrict__ x, const float *__restrict__ dv, float *__restrict__ out) {
    const int64_t m = 3 * count_of(n, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[i] + dv[i];
}

// acc += v over the first m values, or over 3 * (device count) when n_dev is given
__global__ void __launch_bounds__(256)
dn_add(int64_t m, float *__restrict__ acc, const float *__restrict__ v,
       const int32_t *__restrict__ n_dev = nullptr, int64_t cap = 0) {
    if (n_dev != nullptr) m = 3 * count_of(0, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        acc[i] += v[i];
}

__global__ void __launch_bounds__(256)
dn_split(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
         const float *__restrict__ da0, float *__restrict__ dfeat) {
    n = count_of(n, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kFeat;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / kFeat;
        dfeat[i] = da0[s * kIn + (i - s * kFeat)];
    }
}

// Pose gradient, summed over the points in a fixed order: workgroup b sums
// points [b kThetaChunk, (b + 1) kThetaChunk) into part[b] (lanes over the 72
// components, each row read contiguously); dn_theta_reduce then adds the
// partials in order.
__global__ void __launch_bounds__(128)
dn_theta_sum(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const float *__restrict__ da0, float *__restrict__ part) {
    n = count_of(n, n_dev, cap);
    const int c = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kThetaChunk;
    if (c >= kPose || s0 >= n) return;
    const int64_t s1 = s0 + kThetaChunk < n ? s0 + kThetaChunk : n;
    float acc = 0.f;
    for (int64_t s = s0; s < s1; ++s) acc += da0[s * kIn + kFeat + c];
    part[blockIdx.x * kPose + c] = acc;
}

// one workgroup per pose component: thread t sums partials t, t + 256, ...,
// then the 256 sums are added in a fixed tree order
__global__ void __launch_bounds__(256)
dn_theta_reduce(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
                const float *__restrict__ part, float *__restrict__ dtheta) {
    __shared__ float red[256];
    n = count_of(n, n_dev, cap);
    const int c = blockIdx.x, t = threadIdx.x;
    const int64_t nb = (n + kThetaChunk - 1) / kThetaChunk;
    float acc = 0.f;
    for (int64_t b = t; b < nb; b += 256) acc += part[b * kPose + c];
    red[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) dtheta[c] += red[0];
}

// Y[s][j] = act(sum_k X[s][k] B(j, k)) for the first count points s and j < J,
// with B(j, k) = W[j bj + k bk] (bj = K, bk = 1: Y = X W^T for W[J][K]; bj = 1,
// bk = J: Y = X W for W[K][J]).  A workgroup forms 64 points x 64 outputs
// (thread: 4 points x 4 outputs, outputs 16 apart so each row's stores are
// contiguous) over 16-deep slices of X and B staged in LDS; workgroups stride
// over the point tiles.
template <bool RELU>
__global__ void __launch_bounds__(256)
dn_mm(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, const float *__restrict__ X,
      int ldx, int K, const float *__restrict__ W, int bj, int bk, int J, float *__restrict__ Y,
      int ldy) {
    n = count_of(n, n_dev, cap);
    __shared__ __align__(16) float xs[kMmK][kMmT + 4];
    __shared__ __align__(16) float bs[kMmK][kMmT + 4];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int j0 = blockIdx.y * kMmT;
    for (int64_t s0 = (int64_t)blockIdx.x * kMmT; s0 < n; s0 += (int64_t)gridDim.x * kMmT) {
        float acc[4][4] = {};
        for (int k0 = 0; k0 < K; k0 += kMmK) {
#pragma unroll
            for (int e = t; e < kMmT * kMmK; e += 256) {
                const int r = e / kMmK, c = e % kMmK;
                const int64_t s = s0 + r;
                const int k = k0 + c, j = j0 + r;
                xs[c][r] = (s < n && k < K) ? X[s * ldx + k] : 0.f;
                bs[c][r] = (j < J && k < K) ? W[(int64_t)j * bj + (int64_t)k * bk] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kMmK; ++c) {
                const float4 a = *reinterpret_cast<const float4 *>(&xs[c][4 * ty]);
                const float av[4] = {a.x, a.y, a.z, a.w};
                float bv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) bv[q] = bs[c][tx + 16 * q];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[i][q] = fmaf(av[i], bv[q], acc[i][q]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t s = s0 + 4 * ty + i;
            if (s >= n) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + tx + 16 * q;
                if (j < J) Y[s * ldy + j] = RELU ? fmaxf(acc[i][q], 0.f) : acc[i][q];
            }
        }
    }
}

// part[p][o][i] = sum over the points s of chunk p of dY[s][o] X[s][i]: the
// count points split into `parts` chunks of a multiple of 16 points (p =
// blockIdx.z); a workgroup forms 64 o x 64 i over 16-point slices in LDS.
// Empty chunks write zeros, so dn_reduce_partials can add every part in order.
__global__ void __launch_bounds__(256)
dn_mm_dw(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap, const float *__restrict__ dY,
         int O, const float *__restrict__ X, int ldx, int I, int parts,
         float *__restrict__ part) {
    n = count_of(n, n_dev, cap);
    __shared__ __align__(16) float ys[16][kMmT + 4];
    __shared__ __align__(16) float xs[16][kMmT + 4];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int o0 = blockIdx.y * kMmT, i0 = blockIdx.x * kMmT;
    const int64_t chunk = ((n + parts - 1) / parts + 15) / 16 * 16;
    const int64_t sb = (int64_t)blockIdx.z * chunk;
    const int64_t se = sb + chunk < n ? sb + chunk : n;
    float acc[4][4] = {};
    for (int64_t s0 = sb; s0 < se; s0 += 16) {
#pragma unroll
        for (int e = t; e < 16 * kMmT; e += 256) {
            const int r = e / kMmT, c = e % kMmT;
            const int64_t s = s0 + r;
            ys[r][c] = (s < se && o0 + c < O) ? dY[s * O + o0 + c] : 0.f;
            xs[r][c] = (s < se && i0 + c < I) ? X[s * ldx + i0 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float4 a = *reinterpret_cast<const float4 *>(&ys[r][4 * ty]);
            const float av[4] = {a.x, a.y, a.z, a.w};
            float bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) bv[q] = xs[r][tx + 16 * q];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] = fmaf(av[i], bv[q], acc[i][q]);
        }
        __syncthreads();
    }
    float *dst = part + (int64_t)blockIdx.z * O * I;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = o0 + 4 * ty + i;
        if (o >= O) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = i0 + tx + 16 * q;
            if (c < I) dst[(int64_t)o * I + c] = acc[i][q];
        }
    }
}

// dW[i] += sum over the parts of partial[b][i]: a workgroup takes 64 entries,
// its four waves sum the parts b = wave, wave + 4, ... in order, and the four
// sums are added in wave order (a fixed order for given parts)
__global__ void __launch_bounds__(256)
dn_reduce_partials(int64_t m, int32_t parts, const float *__restrict__ partial,
                   float *__restrict__ dW) {
    __shared__ float part4[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < m; i0 += (int64_t)gridDim.x * 64) {
        const int64_t i = i0 + lane;
        float acc = 0.f;
        if (i < m)
            for (int b = wave; b < parts; b += 4) acc += partial[(int64_t)b * m + i];
        part4[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && i < m)
            dW[i] += ((part4[0][lane] + part4[1][lane]) + part4[2][lane]) + part4[3][lane];
        __syncthreads();
    }
}

// Position gradient of the encoding alone (the table gradient is binned
// separately): one thread per point over all levels, so each point's gradient
// is summed in registers and added once, with no atomics.  dfeat is the
// row-major [n][2 L] feature gradient; fp32 table.
__global__ void __launch_bounds__(256)
dn_encode_dx(GridParams p, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const float *__restrict__ x,
             const float2 *__restrict__ table, const float *__restrict__ dfeat,
             float *__restrict__ dx) {
    n = count_of(n, n_dev, cap);
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
            if (lp.inside[0]) acc0 += d0 * p.s_hi[l][0];
            if (lp.inside[1]) acc1 += d1 * p.s_hi[l][1];
            if (lp.inside[2]) acc2 += d2 * p.s_hi[l][2];
        }
        dx[3 * s] += acc0;
        dx[3 * s + 1] += acc1;
        dx[3 * s + 2] += acc2;
    }
}

unsigned mm_grid_x(int64_t cap) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + kMmT - 1) / kMmT, 4096));
}

// Y = act(X B) as dn_mm describes, over the first count of cap points
template <bool RELU>
nvr_status mm(int64_t n, const int32_t *n_dev, int64_t cap, const float *X, int ldx, int K,
              const float *W, int bj, int bk, int J, float *Y, int ldy, hipStream_t st) {
    const dim3 grid(mm_grid_x(cap), (unsigned)((J + kMmT - 1) / kMmT));
    dn_mm<RELU><<<grid, 256, 0, st>>>(n, n_dev, cap, X, ldx, K, W, bj, bk, J, Y, ldy);
    NVR_LAUNCHED();
    return NVR_OK;
}

// dW[O][I] += dY^T X over the first count of cap points, chunk partials summed in order
nvr_status mm_dw(int64_t n, const int32_t *n_dev, int64_t cap, const float *dY, int O,
                 const float *X, int ldx, int I, float *dW, float *partial, hipStream_t st) {
    const int parts = mm_parts(cap);
    const dim3 grid((unsigned)((I + kMmT - 1) / kMmT), (unsigned)((O + kMmT - 1) / kMmT),
                    (unsigned)parts);
    dn_mm_dw<<<grid, 256, 0, st>>>(n, n_dev, cap, dY, O, X, ldx, I, parts, partial);
    NVR_LAUNCHED();
    const int64_t m = (int64_t)O * I;
    dn_reduce_partials<<<grid_for(m, 64, 1024), 256, 0, st>>>(m, parts, partial, dW);
    NVR_LAUNCHED();
    return NVR_OK;
}

__host__ __device__ const float *layer_w(const float *params, int i) {
    if (i == 0) return params;
    return params + (int64_t)kWidth * kIn + (int64_t)(i - 1) * kWidth * kWidth;
}

// Every check of both entry points and of the step's calls, including those of
// the encoding and the binned scatter they call, so that nothing is launched
// before an error.
nvr_status check_desc(const nvr_grid_desc *g, int64_t n) {
    NVR_REQUIRE(g != nullptr, NVR_EINVAL, "grid descriptor is NULL");
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(g->n_levels == 16 && g->n_features == 2, NVR_EUNSUPPORTED,
                "the deformation encoding must be 16 levels x 2 features");
    NVR_REQUIRE(n >= 0 && n <= (1ll << 31) / kWidth, NVR_EINVAL, "n out of 0..2^24");
    const GridParams p = make_grid_params(g);
    NVR_TRY(scatter_check(p));
    NVR_REQUIRE((size_t)n * p.L * 8 < (1ull << 32), NVR_EINVAL, "too many contributions");
    return NVR_OK;
}

nvr_status check(const nvr_grid_desc *g, int64_t n, const void *ws) {
    NVR_TRY(check_desc(g, n));
    NVR_REQUIRE(n == 0 || (ws && aligned(ws, 256)), NVR_EINVAL,
                "workspace NULL or not 256-byte aligned");
    return NVR_OK;
}

// ---------------------------------------------------------------- matrix-core path
// fp16 forward (features, weights, activations), bf16 backward products, fp32
// accumulation, as the field networks.  A wave works on blocks of 16 points in
// the orientation of the field networks: a layer computes D = W X (rows =
// units, columns = points); lane l holds units 16m + 4g..4g+3 (g = l / 16) of
// point l % 16, and pairing row tiles 2q and 2q+1 gives the operand of the
// next layer's K-step q once its contraction index is permuted to match (the
// weight fragments carry the same permutation), so activations stay in
// registers.  The pose enters the first layer as a bias shared by every point,
// W0[:, 32:] theta, formed once per call.
//
// Fragments (16 bytes per lane and tile) are built once per call into the
// workspace: the forward kernel copies its set into LDS, the backward kernel
// copies the transposed set and reads the forward set (L2-resident) to
// recompute each block.  The backward writes, per block of 16 points, the
// bf16 activations and output gradients of every layer unit-major ([units][16]);
// the weight gradients are then contracted over the points on the matrix
// cores by workgroups over point chunks (partials summed in a fixed order).
typedef __attribute__((ext_vector_type(8))) __bf16 dbf8;
typedef __attribute__((ext_vector_type(8))) _Float16 dh8;
typedef __attribute__((ext_vector_type(4))) short ds4;
typedef __attribute__((ext_vector_type(4))) float df4;

__device__ __forceinline__ df4 dmfma(dh8 a, dh8 b, df4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ df4 dmfma(dbf8 a, dbf8 b, df4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ df4 dmfma16(ds4 a, ds4 b, df4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ df4 dzero() { return df4{0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ df4 drelu(df4 a) {
    // max(x, 0) as an integer max on the bits (-0 becomes +0)
    auto r = [](float x) { return __int_as_float(max(__float_as_int(x), 0)); };
    return df4{r(a[0]), r(a[1]), r(a[2]), r(a[3])};
}
__device__ __forceinline__ dh8 dpackh(df4 a, df4 b) {
    dh8 r;
    r[0] = (_Float16)a[0]; r[1] = (_Float16)a[1]; r[2] = (_Float16)a[2]; r[3] = (_Float16)a[3];
    r[4] = (_Float16)b[0]; r[5] = (_Float16)b[1]; r[6] = (_Float16)b[2]; r[7] = (_Float16)b[3];
    return r;
}
__device__ __forceinline__ dbf8 dpackb(df4 a, df4 b) {
    dbf8 r;
    r[0] = (__bf16)a[0]; r[1] = (__bf16)a[1]; r[2] = (__bf16)a[2]; r[3] = (__bf16)a[3];
    r[4] = (__bf16)b[0]; r[5] = (__bf16)b[1]; r[6] = (__bf16)b[2]; r[7] = (__bf16)b[3];
    return r;
}
// contraction index of a 128-wide layer input: K-step q, lane group g, slot j
__host__ __device__ __forceinline__ int dkh(int q, int g, int j) {
    return j < 4 ? 32 * q + 4 * g + j : 32 * q + 16 + 4 * g + (j - 4);
}

// fragment offsets, in 16-byte units (one per lane and tile)
constexpr int kFw0 = 0;                       // W0 (feature part): 8 row tiles
constexpr int kFw1 = kFw0 + 8 * 64;           // W1..W3: 8 row tiles x 4 K-steps each
constexpr int kFw4 = kFw1 + 3 * 32 * 64;      // W4 (3 rows of 16): 4 K-steps
constexpr int kFwd = kFw4 + 4 * 64;           // forward set: 6912 (108 KiB)
constexpr int kBw1 = 0;                       // W1^T..W3^T: 8 row tiles x 4 K-steps each
constexpr int kBw0 = kBw1 + 3 * 32 * 64;      // W0f^T: 2 row tiles (features) x 4 K-steps
constexpr int kBw4 = kBw0 + 8 * 64;           // W4^T: 8 row tiles, 8-byte operands (half units)
constexpr int kBwd = kBw4 + 8 * 64 / 2;       // backward set: 6912 (108 KiB)
constexpr int kDnBlock = 512;                 // 8 waves: two per SIMD around one fragment copy
constexpr int kDnBwdBlock = 1024;             // backward: 16 waves (<= 128 registers each)
// dynamic LDS: the fragment set plus a 1 KiB tile-staging area per wave
constexpr int kFwdStoreLds = (int)(sizeof(uint4) * kFwd) + (kDnBlock / 64) * 1024;      // 116 KiB
constexpr int kBwdLds = (int)(sizeof(uint4) * kBwd) + (kDnBwdBlock / 64) * 1024;        // 124 KiB

// One lane-tile fragment per thread of the grid: forward (fp16, W rows) and
// backward (bf16, W^T rows) sets, both with the chained contraction order.
__global__ void __launch_bounds__(256)
dn_frags(const float *__restrict__ params, uint4 *__restrict__ fwd, uint4 *__restrict__ bwd) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    auto W = [&](int layer, int row, int col) -> float {
        const int in = layer == 0 ? kIn : kWidth;
        return layer_w(params, layer)[(int64_t)row * in + col];
    };
    if (e < kFwd) {
        const int l = e % 64, r = l % 16, g = l / 16, t = e / 64;
        dh8 v;
        if (e < kFw1) {                                     // W0 feature part
            const int m = t;
            for (int j = 0; j < 8; ++j) v[j] = (_Float16)W(0, 16 * m + r, dfp(g, j));
        } else if (e < kFw4) {
            const int u = t - kFw1 / 64, layer = 1 + u / 32, m = (u % 32) / 4, q = u % 4;
            for (int j = 0; j < 8; ++j) v[j] = (_Float16)W(layer, 16 * m + r, dkh(q, g, j));
        } else {
            const int q = t - kFw4 / 64;
            for (int j = 0; j < 8; ++j) v[j] = (_Float16)(r < 3 ? W(4, r, dkh(q, g, j)) : 0.f);
        }
        fwd[e] = __builtin_bit_cast(uint4, v);
        return;
    }
    const int b = e - kFwd;
    if (b < kBw4) {
        const int l = b % 64, r = l % 16, g = l / 16, t = b / 64;
        dbf8 v;
        if (b < kBw0) {                                     // W_L^T, L = 1..3
            const int layer = 1 + t / 32, m = (t % 32) / 4, q = t % 4;
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)W(layer, dkh(q, g, j), 16 * m + r);
        } else {                                            // W0f^T: rows = features
            const int u = t - kBw0 / 64, m = u / 4, q = u % 4;
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)W(0, dkh(q, g, j), 16 * m + r);
        }
        bwd[b] = __builtin_bit_cast(uint4, v);
    } else if (b < kBw4 + 8 * 64) {                         // W4^T, 16x16x16 operands
        const int i = b - kBw4, l = i % 64, r = l % 16, g = l / 16, m = i / 64;
        ds4 v;
        for (int j = 0; j < 4; ++j)
            v[j] = __builtin_bit_cast(short, (__bf16)(4 * g + j < 3 ? W(4, 4 * g + j, 16 * m + r)
                                                                   : 0.f));
        reinterpret_cast<uint2 *>(bwd + kBw4)[i] = __builtin_bit_cast(uint2, v);
    }
}

// bias[u] = sum_c W0[u][32 + c] theta[c]: the pose term of the first layer
__global__ void __launch_bounds__(kWidth)
dn_pose_bias(const float *__restrict__ params, const float *__restrict__ theta,
             float *__restrict__ bias) {
    const int u = threadIdx.x;
    const float *w = params + (int64_t)u * kIn + kFeat;
    float a = 0.f;
    for (int c = 0; c < kPose; ++c) a += w[c] * theta[c];
    bias[u] = a;
}

// Per-block activation / gradient tiles of the backward, bf16, unit-major
// [block][units][16 points]: H holds the encoding (32 units) then the four
// hidden layers' outputs (4 x 128); Z the output gradients of W0..W3 (4 x 128)
// then of W4 (16 units, 3 used).  The ReLU masks of the hidden layers are kept
// as one word per lane and layer: bit 8q + j is slot j of K-step q, the
// register layout of both the forward and the backward chain.
constexpr int kHUnits = kFeat + 4 * kWidth;   // 544
constexpr int kZUnits = 4 * kWidth + 16;      // 528
__device__ __forceinline__ uint16_t bfbits(float v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

// Hidden layer l's activations of one block into its H tile and mask word
// (lane g, c; zero for points past n).
// One 32-unit slice of a block's unit-major tile ([unit][16 points], bf16)
// stored through the wave's 1 KiB LDS staging area: every lane puts its
// point's 8 values (slice units u[j]) there, then stores one 16-byte chunk,
// so the slice leaves as 64 contiguous 16-byte stores instead of 512 2-byte
// ones.  A wave's LDS operations complete in order; the empty asm statements
// keep the compiler from moving the accesses across each other.
__device__ __forceinline__ void dn_put_slice(uint16_t *stage, uint16_t *dst, const int (&u)[8],
                                             const uint16_t (&v)[8], int lane, int c) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < 8; ++j) stage[u[j] * 16 + c] = v[j];
    asm volatile("" ::: "memory");
    reinterpret_cast<uint4 *>(dst)[lane] = reinterpret_cast<const uint4 *>(stage)[lane];
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ void dn_store_hidden(const dh8 *hid, int l, uint16_t *H, uint32_t *mw,
                                                uint16_t *stage, int lane, int g, int c,
                                                bool valid) {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int u[8];
        uint16_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float f = (float)hid[q][j];
            u[j] = dkh(q, g, j) - 32 * q;
            v[j] = valid ? bfbits(f) : (uint16_t)0;
            m |= (f > 0.f ? 1u : 0u) << (8 * q + j);
        }
        dn_put_slice(stage, H + (kFeat + l * kWidth + 32 * q) * 16, u, v, lane, c);
    }
    mw[l * 64 + lane] = m;
}

// Forward of one block of 16 points: acc[m] are the output row tiles of the
// last hidden layer; hid[l][q] the packed (fp16) activations of hidden layer l.
// STORE: each hidden layer's tile and mask word are written as soon as the
// layer is formed (H: the block's tile, mw: its 4 x 64 mask words).
struct DnFwd {
    df4 acc[8];
    dh8 hid[4][4];
    df4 out;
};

// bias4: the pose bias at rows 16m + 4g.. of this lane (read per block)
template <bool STORE = false>
__device__ __forceinline__ void dn_block_fwd(const uint4 *__restrict__ F,
                                             const float *__restrict__ bias4, dh8 x0, DnFwd &s,
                                             uint16_t *H = nullptr, uint32_t *mw = nullptr,
                                             uint16_t *stage = nullptr, int lane = 0,
                                             bool valid = false) {
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int m = 0; m < 8; ++m)
        s.acc[m] = dmfma(__builtin_bit_cast(dh8, F[kFw0 + m * 64]), x0,
                         *reinterpret_cast<const df4 *>(bias4 + 16 * m));
#pragma unroll
    for (int layer = 1; layer <= 3; ++layer) {
        asm volatile("" ::: "memory");   // load each layer's fragments when it runs
#pragma unroll
        for (int q = 0; q < 4; ++q)
            s.hid[layer - 1][q] = dpackh(drelu(s.acc[2 * q]), drelu(s.acc[2 * q + 1]));
        if (STORE) dn_store_hidden(s.hid[layer - 1], layer - 1, H, mw, stage, lane, g, c, valid);
        const int base = kFw1 + (layer - 1) * 32 * 64;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            if (m == 4) asm volatile("" ::: "memory");   // half a layer of fragments at a time
            df4 a = dzero();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a = dmfma(__builtin_bit_cast(dh8, F[base + (m * 4 + q) * 64]), s.hid[layer - 1][q],
                          a);
            s.acc[m] = a;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s.hid[3][q] = dpackh(drelu(s.acc[2 * q]), drelu(s.acc[2 * q + 1]));
    if (STORE) dn_store_hidden(s.hid[3], 3, H, mw, stage, lane, g, c, valid);
    df4 o = dzero();
#pragma unroll
    for (int q = 0; q < 4; ++q) o = dmfma(__builtin_bit_cast(dh8, F[kFw4 + q * 64]), s.hid[3][q], o);
    s.out = o;
}

// The 8 fp16 encoding values of lane group g for point p (zero past n), from
// the level-group planes of stride cap.
__device__ __forceinline__ dh8 dn_load_feat(const uint16_t *__restrict__ feat, int64_t cap,
                                            int64_t p, int g, bool valid) {
    if (!valid) return dh8{};
    const uint2 a = *reinterpret_cast<const uint2 *>(feat + ((int64_t)(2 * g) * cap + p) * 4);
    const uint2 b = *reinterpret_cast<const uint2 *>(feat + ((int64_t)(2 * g + 1) * cap + p) * 4);
    return __builtin_bit_cast(dh8, uint4{a.x, a.y, b.x, b.y});
}

// Forward: x_can = x + W4 relu(W3 relu(W2 relu(W1 relu(W0f feat + bias)))).
// feat: fp16 encoding, level-group planes [8][cap][4]; bias: the pose term
// [128]; x_can nullable.  STORE (training): each block's encoding and hidden
// activations go to its H tile (bf16) and the ReLU masks to mwords
// [block][4][64], for the backward, which then does not recompute the forward.
template <bool STORE>
__global__ void __launch_bounds__(kDnBlock)
dn_fwd_mfma(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
            const uint16_t *__restrict__ feat, const float *__restrict__ bias,
            const uint4 *__restrict__ gfwd, const float *__restrict__ x,
            float *__restrict__ x_can, uint16_t *__restrict__ hbuf,
            uint32_t *__restrict__ mwords) {
    extern __shared__ uint4 F[];   // [kFwd] fragments, then (STORE) 1 KiB staging per wave
    for (int i = threadIdx.x; i < kFwd; i += kDnBlock) F[i] = gfwd[i];
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    uint16_t *stage = reinterpret_cast<uint16_t *>(F + kFwd) + (threadIdx.x >> 6) * 512;
    const float *bias4 = bias + 4 * g;
    __syncthreads();
    n = count_of(n, n_dev, cap);
    const int64_t waves = (int64_t)gridDim.x * (kDnBlock / 64);
    for (int64_t blk = blockIdx.x * (int64_t)(kDnBlock / 64) + (threadIdx.x >> 6); blk * 16 < n;
         blk += waves) {
        // the fragments are re-read from LDS each block: keeps the compiler
        // from hoisting all 108 of them into registers across the loop
        asm volatile("" ::: "memory");
        const int64_t p = blk * 16 + c;
        const bool valid = p < n;
        const dh8 x0 = dn_load_feat(feat, cap, p, g, valid);
        uint16_t *H = STORE ? hbuf + blk * (int64_t)kHUnits * 16 : nullptr;
        if (STORE) {
            // encoding: slot j = feature dfp(g, j); the hidden layers follow
            // in dn_block_fwd (slot j of K-step q = unit dkh(q, g, j))
            int u[8];
            uint16_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                u[j] = dfp(g, j);
                v[j] = bfbits((float)x0[j]);
            }
            dn_put_slice(stage, H, u, v, lane, c);
        }
        DnFwd s;
        dn_block_fwd<STORE>(F + lane, bias4, x0, s, H, STORE ? mwords + blk * 4 * 64 : nullptr,
                            stage, lane, valid);
        if (g == 0 && valid && x_can != nullptr) {
            x_can[3 * p] = x[3 * p] + s.out[0];
            x_can[3 * p + 1] = x[3 * p + 1] + s.out[1];
            x_can[3 * p + 2] = x[3 * p + 2] + s.out[2];
        }
    }
}

// Backward chain of each block from the stored masks: dZ4 = dx_can, then
// dH3 = W4^T dZ4 (16x16x16) and dH_{l-1} = W_l^T dZ_l (bf16, masked by
// layer l-1's ReLU), dfeat = W0f^T dZ0; each block's output gradients are
// stored as bf16 tiles for the weight-gradient contraction.
__global__ void __launch_bounds__(kDnBwdBlock)
dn_bwd_mfma(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
            const uint4 *__restrict__ gbwd, const uint32_t *__restrict__ mwords,
            const float *__restrict__ dxc, float *__restrict__ dfeat,
            uint16_t *__restrict__ zbuf) {
    extern __shared__ uint4 Bt[];   // [kBwd] fragments, then 1 KiB staging per wave
    for (int i = threadIdx.x; i < kBwd; i += kDnBwdBlock) Bt[i] = gbwd[i];
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    uint16_t *stage = reinterpret_cast<uint16_t *>(Bt + kBwd) + (threadIdx.x >> 6) * 512;
    __syncthreads();
    const uint4 *Bl = Bt + lane;
    const uint2 *B4 = reinterpret_cast<const uint2 *>(Bt + kBw4) + lane;
    n = count_of(n, n_dev, cap);
    const int64_t waves = (int64_t)gridDim.x * (kDnBwdBlock / 64);
    for (int64_t blk = blockIdx.x * (int64_t)(kDnBwdBlock / 64) + (threadIdx.x >> 6); blk * 16 < n;
         blk += waves) {
        asm volatile("" ::: "memory");   // fragments are re-read each block (see the forward)
        const int64_t p = blk * 16 + c;
        const bool valid = p < n;
        uint32_t mask[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) mask[l] = mwords[(blk * 4 + l) * 64 + lane];
        uint16_t *Z = zbuf + blk * (int64_t)kZUnits * 16;
        // output layer: dZ4 = dx_can (rows 0..2 of a 16-row operand)
        ds4 z4 = {};
        if (g == 0 && valid) {
            z4[0] = __builtin_bit_cast(short, (__bf16)dxc[3 * p]);
            z4[1] = __builtin_bit_cast(short, (__bf16)dxc[3 * p + 1]);
            z4[2] = __builtin_bit_cast(short, (__bf16)dxc[3 * p + 2]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) Z[(4 * kWidth + 4 * g + j) * 16 + c] = (uint16_t)z4[j];
        df4 d[8];
#pragma unroll
        for (int m = 0; m < 8; ++m)
            d[m] = dmfma16(__builtin_bit_cast(ds4, B4[m * 64]), z4, dzero());
        dbf8 zb[4];
#pragma unroll
        for (int layer = 3; layer >= 0; --layer) {
            asm volatile("" ::: "memory");   // load each layer's fragments when it runs
            // dZ = dH through the ReLU of hidden layer `layer`, staged, then
            // paired into the next operands
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (!((mask[layer] >> (8 * q + i)) & 1u)) d[2 * q][i] = 0.f;
                    if (!((mask[layer] >> (8 * q + 4 + i)) & 1u)) d[2 * q + 1][i] = 0.f;
                }
                zb[q] = dpackb(d[2 * q], d[2 * q + 1]);
                int u[8];
                uint16_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    u[j] = dkh(q, g, j) - 32 * q;
                    v[j] = valid ? bfbits(j < 4 ? d[2 * q][j] : d[2 * q + 1][j - 4]) : (uint16_t)0;
                }
                dn_put_slice(stage, Z + (layer * kWidth + 32 * q) * 16, u, v, lane, c);
            }
            if (layer > 0) {
                const int base = kBw1 + (layer - 1) * 32 * 64;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    if (m == 4) asm volatile("" ::: "memory");
                    df4 a = dzero();
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        a = dmfma(__builtin_bit_cast(dbf8, Bl[base + (m * 4 + q) * 64]), zb[q], a);
                    d[m] = a;
                }
            }
        }
        // encoding gradient: dfeat = W0f^T dZ0, rows = features 16m + 4g + i,
        // that is levels 8m + 2g (i = 0, 1) and 8m + 2g + 1 (i = 2, 3): planes
        // 2g and 2g+1, slots 2m and 2m+1
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            df4 a = dzero();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a = dmfma(__builtin_bit_cast(dbf8, Bl[kBw0 + (m * 4 + q) * 64]), zb[q], a);
            if (valid) {
                *reinterpret_cast<float2 *>(dfeat + ((int64_t)(2 * g) * cap + p) * 4 + 2 * m) =
                    float2{a[0], a[1]};
                *reinterpret_cast<float2 *>(dfeat + ((int64_t)(2 * g + 1) * cap + p) * 4 + 2 * m) =
                    float2{a[2], a[3]};
            }
        }
    }
}

// Weight gradients dW = dZ H^T over the points: workgroup b contracts K-steps
// of 32 points (two blocks) b, b + grid, ... for out tiles w and w + 4 of its
// wave w and every in tile; `ones` adds an in tile of ones (the sums over the
// points of dZ, for the pose gradient).  The next K-step's operands are loaded
// while the current one is contracted.  Writes its [16 TO][16 (TI + ones)]
// partial.
template <int TO, int TI, bool ONES>
__global__ void __launch_bounds__(256)
dn_dw(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
      const uint16_t *__restrict__ zbuf, int z_off,
      const uint16_t *__restrict__ hbuf, int h_off, float *__restrict__ partial) {
    constexpr int TIN = TI + (ONES ? 1 : 0);
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15, w = threadIdx.x >> 6;
    df4 acc[2][TIN];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < TIN; ++t) acc[a][t] = dzero();
    const int64_t nblk = (count_of(n, n_dev, cap) + 15) / 16;
    const int64_t nstep = (nblk + 1) / 2;
    dbf8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = (__bf16)1.f;
    const int pt = 8 * (g & 1);
    auto load = [&](int64_t st, dbf8 *A, dbf8 *B) {
        const int64_t blk = 2 * st + (g >> 1);
        const bool in_range = st < nstep && blk < nblk;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int mo = w + 4 * a;
            A[a] = {};
            if (mo < TO && in_range)
                A[a] = __builtin_bit_cast(dbf8, *reinterpret_cast<const uint4 *>(
                    zbuf + (blk * kZUnits + z_off + 16 * mo + r) * 16 + pt));
        }
#pragma unroll
        for (int t = 0; t < TI; ++t) {
            B[t] = {};
            if (in_range)
                B[t] = __builtin_bit_cast(dbf8, *reinterpret_cast<const uint4 *>(
                    hbuf + (blk * kHUnits + h_off + 16 * t + r) * 16 + pt));
        }
    };
    dbf8 An[2], Bn[TI];
    load(blockIdx.x, An, Bn);
    for (int64_t st = blockIdx.x; st < nstep; st += gridDim.x) {
        dbf8 A[2], B[TI];
#pragma unroll
        for (int a = 0; a < 2; ++a) A[a] = An[a];
#pragma unroll
        for (int t = 0; t < TI; ++t) B[t] = Bn[t];
        load(st + gridDim.x, An, Bn);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (w + 4 * a >= TO) continue;
#pragma unroll
            for (int t = 0; t < TI; ++t) acc[a][t] = dmfma(A[a], B[t], acc[a][t]);
            if (ONES) acc[a][TI] = dmfma(A[a], ones, acc[a][TI]);
        }
    }
    // partial[b][row 16 mo + 4g + i][col 16 t + r]
    const int ncol = 16 * TIN;
    float *out = partial + (int64_t)blockIdx.x * (16 * TO) * ncol;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int mo = w + 4 * a;
        if (mo >= TO) continue;
#pragma unroll
        for (int t = 0; t < TIN; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[(16 * mo + 4 * g + i) * ncol + 16 * t + r] = acc[a][t][i];
    }
}

// dW[row][col] (acc, rows < out_rows, cols < in_cols of the weight, stride
// w_ld) += sum over the workgroups' partials: a workgroup takes 64 outputs,
// its four waves sum the parts b = wave, wave + 4, ... in order, and the four
// sums are added in wave order (a fixed order for given parts).
__global__ void __launch_bounds__(256)
dn_dw_reduce(int parts, int rows, int ncol, int out_rows, int in_cols,
             const float *__restrict__ partial, float *__restrict__ dW, int w_ld) {
    __shared__ float part4[4][64];
    const int64_t total = (int64_t)out_rows * in_cols;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < total; i0 += (int64_t)gridDim.x * 64) {
        const int64_t i = i0 + lane;
        float a = 0.f;
        if (i < total) {
            const int row = (int)(i / in_cols), col = (int)(i % in_cols);
            for (int b = wave; b < parts; b += 4)
                a += partial[((int64_t)b * rows + row) * ncol + col];
        }
        part4[wave][lane] = a;
        __syncthreads();
        if (wave == 0 && i < total) {
            const int row = (int)(i / in_cols), col = (int)(i % in_cols);
            dW[(int64_t)row * w_ld + col] +=
                ((part4[0][lane] + part4[1][lane]) + part4[2][lane]) + part4[3][lane];
        }
        __syncthreads();
    }
}

// The pose part of the first layer, from s[u] = sum over the points of dZ0[u]
// (the ones column, column `col` of the layer-0 partials, summed in order):
// dW0[u][32 + c] += s[u] theta[c] and (nullable) dtheta[c] += sum_u W0[u][32 + c] s[u].
// One workgroup of kPoseSplit x kWidth threads: thread (k, u) sums the parts
// k, k + kPoseSplit, ... of unit u (independent loads, several in flight), and
// the kPoseSplit sums of a unit are added in k order: a fixed order.
constexpr int kPoseSplit = 8;
__global__ void __launch_bounds__(kPoseSplit * kWidth)
dn_pose_grad(int parts, int ncol, int col, const float *__restrict__ partial,
             const float *__restrict__ params, const float *__restrict__ theta,
             float *__restrict__ dparams, float *__restrict__ dtheta) {
    __shared__ float sk[kPoseSplit][kWidth];
    __shared__ float su[kWidth];
    const int u = threadIdx.x % kWidth, k = threadIdx.x / kWidth;
    float a = 0.f;
#pragma unroll 8
    for (int b = k; b < parts; b += kPoseSplit) a += partial[((int64_t)b * kWidth + u) * ncol + col];
    sk[k][u] = a;
    __syncthreads();
    if (k == 0) {
        a = 0.f;
        for (int j = 0; j < kPoseSplit; ++j) a += sk[j][u];
        su[u] = a;
        for (int c = 0; c < kPose; ++c) dparams[(int64_t)u * kIn + kFeat + c] += a * theta[c];
    }
    __syncthreads();
    if (dtheta != nullptr && k == 0 && u < kPose) {
        float t = 0.f;
        for (int v = 0; v < kWidth; ++v) t += params[(int64_t)v * kIn + kFeat + u] * su[v];
        dtheta[u] += t;
    }
}

size_t carve_mfma(const nvr_grid_desc *g, int64_t n, bool det, char *base, DeformMfmaWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += round_up(bytes);
        return p;
    };
    const int64_t nblk = (n + 15) / 16 + 1;   // one spare block: K-steps pair blocks
    DeformMfmaWs t;
    const GridParams gp = make_grid_params(g);
    t.feat = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * (size_t)n * kFeat));
    t.bias = reinterpret_cast<float *>(take(sizeof(float) * kWidth));
    t.fwd = reinterpret_cast<uint4 *>(take(sizeof(uint4) * kFwd));
    t.bwd = reinterpret_cast<uint4 *>(take(sizeof(uint4) * kBwd));
    t.hbuf = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * (size_t)nblk * kHUnits * 16));
    t.zbuf = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * (size_t)nblk * kZUnits * 16));
    t.mwords = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * (size_t)nblk * 4 * 64));
    t.dfeat = reinterpret_cast<float *>(take(sizeof(float) * (size_t)n * kFeat));
    t.dx_parts = reinterpret_cast<float *>(take(sizeof(float) * (size_t)kXcds * n * 3));
    t.jac = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * (size_t)3 * (kFeat / 2) * n));
    t.partial = reinterpret_cast<float *>(take(sizeof(float) * (size_t)kDwGrid * kWidth * 144));
    t.half = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * (size_t)gp.off[gp.L]));
    t.binned = take(det ? scatter_det_ws_bytes(gp, n) : scatter_ws_bytes(gp, n));
    if (w) *w = t;
    return off;
}

// opt in to the fragment copies' LDS, once per device
nvr_status dn_lds_opt_in() {
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    NVR_HIP(hipGetDevice(&dev));
    const uint64_t bit = 1ull << (dev & 63);
    if (done.load() & bit) return NVR_OK;
    NVR_HIP(hipFuncSetAttribute((const void *)dn_fwd_mfma<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(uint4) * kFwd)));
    NVR_HIP(hipFuncSetAttribute((const void *)dn_fwd_mfma<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kFwdStoreLds));
    NVR_HIP(hipFuncSetAttribute((const void *)dn_bwd_mfma,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kBwdLds));
    done.fetch_or(bit);
    return NVR_OK;
}

// fp16 copy of an fp32 table (the public entry points' matrix-core path)
__global__ void __launch_bounds__(256)
dn_to_half(int64_t m, const float2 *__restrict__ t, uint32_t *__restrict__ h) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = t[i];
        h[i] = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v.x) |
               ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v.y) << 16);
    }
}

// dx[i] += dx_can[i] + the eight level groups' partials, i < 3 count: the
// position gradient through the encoding plus the residual's identity
__global__ void __launch_bounds__(256)
dn_dx_total(int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
            const float *__restrict__ parts, const float *__restrict__ dx_can,
            float *__restrict__ dx) {
    const int64_t m = 3 * count_of(n, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        float a = dx_can[i];
#pragma unroll
        for (int g = 0; g < kXcds; ++g) a += parts[(int64_t)g * 3 * cap + i];
        dx[i] += a;
    }
}

// Encoding (split gather of the fp16 table into level-group planes, with the
// scatter's tile counts when `counter` is given; skipped when the features
// are already in the workspace), fragments and pose bias.  The point count is
// n, or *n_dev (at most cap) when n_dev is given.
nvr_status mfma_prologue(const GridParams &gp, int64_t n, const int32_t *n_dev, int64_t cap,
                         const float *x, const float *theta, const void *table_half,
                         const float *params, const DeformMfmaWs &w, bool encode,
                         const TileCounter *counter, bool jac, hipStream_t st) {
    NVR_TRY(dn_lds_opt_in());
    if (encode)
        NVR_TRY(launch_encode_fwd(gp, n, n_dev, cap, x, table_half, NVR_F16, w.feat, NVR_F16,
                                  true, st, counter, 0, jac ? w.jac : nullptr));
    dn_frags<<<(kFwd + kBw4 + 8 * 64 + 255) / 256, 256, 0, st>>>(params, w.fwd, w.bwd);
    NVR_LAUNCHED();
    dn_pose_bias<<<1, kWidth, 0, st>>>(params, theta, w.bias);
    NVR_LAUNCHED();
    return NVR_OK;
}

unsigned dn_grid(int64_t cap, int block = kDnBlock) {
    const int64_t nblk = (cap + 15) / 16;
    const int64_t wg = (nblk + block / 64 - 1) / (block / 64);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(wg, kCus));
}

// count: form the binned scatter's tile counts during the encoding; store:
// keep the activation tiles and ReLU masks for a backward (a training
// forward); x_can nullable.
nvr_status mfma_forward(const GridParams &gp, int64_t n, const int32_t *n_dev, int64_t cap,
                        const float *x, const float *theta, const void *table_half,
                        const float *params, float *x_can, const DeformMfmaWs &w, bool count,
                        bool store, hipStream_t st) {
    TileCounter counter{};
    if (count) {
        counter = scatter_counter(gp, w.binned);
        NVR_TRY(launch_counter_reset(gp, w.binned, st));
    }
    // a training forward also keeps the encoding's spatial derivatives for the
    // backward's position gradient
    NVR_TRY(mfma_prologue(gp, n, n_dev, cap, x, theta, table_half, params, w, true,
                          count ? &counter : nullptr, store, st));
    if (store)
        dn_fwd_mfma<true><<<dn_grid(cap), kDnBlock, kFwdStoreLds, st>>>(
            n, n_dev, cap, w.feat, w.bias, w.fwd, x, x_can, w.hbuf, w.mwords);
    else
        dn_fwd_mfma<false><<<dn_grid(cap), kDnBlock, sizeof(uint4) * kFwd, st>>>(
            n, n_dev, cap, w.feat, w.bias, w.fwd, x, x_can, nullptr, nullptr);
    NVR_LAUNCHED();
    return NVR_OK;
}

int dw_parts(int64_t cap) {
    const int64_t nstep = ((cap + 15) / 16 + 1) / 2;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nstep, kDwGrid));
}

// dW (acc) of one layer: dZ rows at z_off (TO tiles) against H rows at h_off (TI tiles)
template <int TO, int TI, bool ONES>
nvr_status mfma_dw(int64_t n, const int32_t *n_dev, int64_t cap, const DeformMfmaWs &w,
                   int z_off, int h_off, float *dW, int out_rows, int in_cols, int w_ld,
                   hipStream_t st) {
    const int parts = dw_parts(cap);
    dn_dw<TO, TI, ONES><<<parts, 256, 0, st>>>(n, n_dev, cap, w.zbuf, z_off, w.hbuf, h_off,
                                               w.partial);
    NVR_LAUNCHED();
    const int ncol = 16 * (TI + (ONES ? 1 : 0));
    dn_dw_reduce<<<grid_for((int64_t)out_rows * in_cols, 64, 1024), 256, 0, st>>>(
        parts, 16 * TO, ncol, out_rows, in_cols, w.partial, dW, w_ld);
    NVR_LAUNCHED();
    return NVR_OK;
}

// Matrix-core backward: the chain per block from the training forward's
// masks, weight gradients over the points from its activation tiles, pose
// terms, then the encoding's table gradient (binned scatter of the fp16-table
// encoding; deterministic variant when det) and, when dx is given, its
// position gradient plus the residual's identity.  features_ready: a training
// forward over the same points left its encoding, tiles and masks in the
// workspace (and, with counted, its tile counts); otherwise one runs first.
nvr_status mfma_backward(const GridParams &gp, int64_t n, const int32_t *n_dev, int64_t cap,
                         const float *x, const float *theta, const void *table_half,
                         const float *params, const float *dx_can, float *dparams, float *dtable,
                         float *dx, float *dtheta, bool features_ready, bool counted, bool det,
                         const DeformMfmaWs &w, hipStream_t st, const ScatterTail *tail) {
    if (!features_ready)
        NVR_TRY(mfma_forward(gp, n, n_dev, cap, x, theta, table_half, params, nullptr, w, false,
                             true, st));
    dn_bwd_mfma<<<dn_grid(cap, kDnBwdBlock), kDnBwdBlock, kBwdLds, st>>>(
        n, n_dev, cap, w.bwd, w.mwords, dx_can, w.dfeat, w.zbuf);
    NVR_LAUNCHED();
    // W4 [3][128]: dZ4 rows at 512 (one tile) x H3 at 416
    NVR_TRY((mfma_dw<1, 8, false>(n, n_dev, cap, w, 4 * kWidth, kFeat + 3 * kWidth,
                                  dparams + (layer_w(params, 4) - params), 3, kWidth, kWidth,
                                  st)));
    for (int layer = 3; layer >= 1; --layer)   // W_L [128][128]: dZ_L x H_{L-1}
        NVR_TRY((mfma_dw<8, 8, false>(n, n_dev, cap, w, layer * kWidth,
                                      kFeat + (layer - 1) * kWidth,
                                      dparams + (layer_w(params, layer) - params), kWidth,
                                      kWidth, kWidth, st)));
    // W0's feature columns: dZ0 x encoding, plus the sums of dZ0 for the pose
    NVR_TRY((mfma_dw<8, 2, true>(n, n_dev, cap, w, 0, 0, dparams, kWidth, kFeat, kIn, st)));
    dn_pose_grad<<<1, kPoseSplit * kWidth, 0, st>>>(dw_parts(cap), 16 * 3, 16 * 2, w.partial,
                                                    params, theta, dparams, dtheta);
    NVR_LAUNCHED();
    float *parts = dx ? w.dx_parts : nullptr;
    if (det)
        NVR_TRY(launch_scatter_det(gp, n, n_dev, cap, x, table_half, w.dfeat, dtable, parts,
                                   w.binned, st, parts ? w.jac : nullptr));
    else
        NVR_TRY(launch_scatter(gp, n, n_dev, cap, x, table_half, w.dfeat, dtable, parts, w.binned,
                               st, counted && features_ready, 1024, 512, parts ? w.jac : nullptr,
                               tail));
    if (dx) {
        dn_dx_total<<<grid_for(cap * 3, 256, 16384), 256, 0, st>>>(n, n_dev, cap, w.dx_parts,
                                                                   dx_can, dx);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}

// float32 forward into the workspace: encoding, input [enc | theta], hidden
// layers, output dv (the residual is added by the caller)
nvr_status f32_forward(const GridParams &gp, int64_t n, const int32_t *n_dev, int64_t cap,
                       const float *x, const float *theta, const float *table,
                       const float *params, const DeformWs &w, hipStream_t st) {
    NVR_TRY(launch_encode_fwd(gp, n, n_dev, cap, x, table, NVR_F32, w.feat, NVR_F32, false, st));
    dn_concat<<<grid_for(cap * kIn, 256, 16384), 256, 0, st>>>(n, n_dev, cap, w.feat, theta, w.a0);
    NVR_LAUNCHED();
    const float *in = w.a0;
    int width_in = kIn;
    for (int i = 0; i < kHidden; ++i) {
        NVR_TRY(mm<true>(n, n_dev, cap, in, width_in, width_in, layer_w(params, i), width_in, 1,
                         kWidth, w.h[i], kWidth, st));
        in = w.h[i];
        width_in = kWidth;
    }
    return mm<false>(n, n_dev, cap, in, kWidth, kWidth, layer_w(params, kHidden), kWidth, 1, 3,
                     w.dv, 3, st);
}

nvr_status f32_backward(const GridParams &gp, int64_t n, const int32_t *n_dev, int64_t cap,
                        const float *x, const float *theta, const float *table,
                        const float *params, const float *dx_can, float *dparams, float *dtable,
                        float *dx, float *dtheta, bool det, const DeformWs &w, hipStream_t st) {
    NVR_TRY(f32_forward(gp, n, n_dev, cap, x, theta, table, params, w, st));
    // output layer: dW_out += dx_can^T h4; dh = dx_can W_out
    float *dW = dparams + (kParams - 3 * kWidth);
    NVR_TRY(mm_dw(n, n_dev, cap, dx_can, 3, w.h[kHidden - 1], kWidth, kWidth, dW, w.partial, st));
    NVR_TRY(mm<false>(n, n_dev, cap, dx_can, 3, 3, layer_w(params, kHidden), 1, kWidth, kWidth,
                      w.dh0, kWidth, st));
    float *dh = w.dh0, *dh_next = w.dh1;
    for (int i = kHidden - 1; i >= 0; --i) {
        dn_relu_bwd<<<grid_for(cap * kWidth, 256, 16384), 256, 0, st>>>(n, n_dev, cap, kWidth, dh,
                                                                        w.h[i]);
        NVR_LAUNCHED();
        const int width_in = i == 0 ? kIn : kWidth;
        const float *in = i == 0 ? w.a0 : w.h[i - 1];
        float *dWi = dparams + (layer_w(params, i) - params);
        NVR_TRY(mm_dw(n, n_dev, cap, dh, kWidth, in, width_in, width_in, dWi, w.partial, st));
        float *dst = i == 0 ? w.da0 : dh_next;
        NVR_TRY(mm<false>(n, n_dev, cap, dh, kWidth, kWidth, layer_w(params, i), 1, width_in,
                          width_in, dst, width_in, st));
        if (i > 0) {
            dh_next = dh;
            dh = dst;
        }
    }
    dn_split<<<grid_for(cap * kFeat, 256, 16384), 256, 0, st>>>(n, n_dev, cap, w.da0, w.dfeat);
    NVR_LAUNCHED();
    if (dtheta) {
        const unsigned nb = (unsigned)std::max<int64_t>(1, (cap + kThetaChunk - 1) / kThetaChunk);
        dn_theta_sum<<<nb, 128, 0, st>>>(n, n_dev, cap, w.da0, w.theta_part);
        NVR_LAUNCHED();
        dn_theta_reduce<<<kPose, 256, 0, st>>>(n, n_dev, cap, w.theta_part, dtheta);
        NVR_LAUNCHED();
    }
    NVR_TRY(launch_scatter_rows(gp, n, n_dev, cap, x, w.dfeat, dtable, w.binned, st, det));
    if (dx) {
        dn_encode_dx<<<grid_for(cap, 256, 16384), 256, 0, st>>>(
            gp, n, n_dev, cap, x, reinterpret_cast<const float2 *>(table), w.dfeat, dx);
        NVR_LAUNCHED();
        // the residual's identity: dx += dx_can
        dn_add<<<grid_for(cap * 3, 256, 16384), 256, 0, st>>>(n * 3, dx, dx_can, n_dev, cap);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}

size_t ws_bytes(const nvr_grid_desc *g, int64_t cap, bool matrix_cores, bool det) {
    return matrix_cores ? carve_mfma(g, cap, det, nullptr, nullptr)
                        : carve(g, cap, det, nullptr, nullptr);
}

// table_half: the fp16 copy of the table, or null to form it in the workspace
// (matrix-core path only).  count, store: a training forward whose tile counts
// and activation tiles the backward will use (matrix-core path only).
nvr_status run_fwd(const nvr_grid_desc *g, bool matrix_cores, int64_t n, const int32_t *n_dev,
                   int64_t cap, const float *x, const float *theta, const float *table,
                   const void *table_half, const float *params, float *x_can, bool count,
                   bool store, bool det, void *ws, hipStream_t st) {
    const GridParams gp = make_grid_params(g);
    if (matrix_cores) {
        DeformMfmaWs w;
        carve_mfma(g, cap, det, static_cast<char *>(ws), &w);
        if (!table_half) {
            dn_to_half<<<grid_for(gp.off[gp.L], 256, 16384), 256, 0, st>>>(
                gp.off[gp.L], reinterpret_cast<const float2 *>(table), w.half);
            NVR_LAUNCHED();
            table_half = w.half;
        }
        return mfma_forward(gp, n, n_dev, cap, x, theta, table_half, params, x_can, w, count,
                            store, st);
    }
    DeformWs w;
    carve(g, cap, det, static_cast<char *>(ws), &w);
    NVR_TRY(f32_forward(gp, n, n_dev, cap, x, theta, table, params, w, st));
    dn_residual<<<grid_for(cap * 3, 256, 16384), 256, 0, st>>>(n, n_dev, cap, x, w.dv, x_can);
    NVR_LAUNCHED();
    return NVR_OK;
}

// after_fwd: a training forward over the same points ran on this workspace
// (matrix-core path: its encoding, and unless det its tile counts, are reused)
nvr_status run_bwd(const nvr_grid_desc *g, bool matrix_cores, int64_t n, const int32_t *n_dev,
                   int64_t cap, const float *x, const float *theta, const float *table,
                   const void *table_half, const float *params, const float *dx_can,
                   float *dparams, float *dtable, float *dx, float *dtheta, bool after_fwd,
                   bool det, void *ws, hipStream_t st, const ScatterTail *tail = nullptr) {
    const GridParams gp = make_grid_params(g);
    if (matrix_cores) {
        DeformMfmaWs w;
        carve_mfma(g, cap, det, static_cast<char *>(ws), &w);
        if (!table_half) {
            dn_to_half<<<grid_for(gp.off[gp.L], 256, 16384), 256, 0, st>>>(
                gp.off[gp.L], reinterpret_cast<const float2 *>(table), w.half);
            NVR_LAUNCHED();
            table_half = w.half;
        }
        return mfma_backward(gp, n, n_dev, cap, x, theta, table_half, params, dx_can, dparams,
                             dtable, dx, dtheta, after_fwd, after_fwd && !det, det, w, st, tail);
    }
    DeformWs w;
    carve(g, cap, det, static_cast<char *>(ws), &w);
    return f32_backward(gp, n, n_dev, cap, x, theta, table, params, dx_can, dparams, dtable, dx,
                        dtheta, det, w, st);
}

}  // namespace

// ------------------------------------------------------- training-step calls
nvr_status deform_check(const nvr_grid_desc *g, int64_t cap) { return check_desc(g, cap); }

nvr_status deform_setup() { return dn_lds_opt_in(); }

size_t deform_ws_bytes(const nvr_grid_desc *g, int64_t cap, bool matrix_cores, bool det) {
    return ws_bytes(g, cap, matrix_cores, det);
}

nvr_status deform_fwd_dev(const nvr_grid_desc *g, bool matrix_cores, const int32_t *n_dev,
                          int64_t cap, const float *x, const float *theta, const float *table,
                          const void *table_half, const float *params, float *x_can, bool train,
                          bool det, void *ws, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    return run_fwd(g, matrix_cores, 0, n_dev, cap, x, theta, table, table_half, params, x_can,
                   train && !det, train, det, ws, st);
}

nvr_status deform_bwd_dev(const nvr_grid_desc *g, bool matrix_cores, const int32_t *n_dev,
                          int64_t cap, const float *x, const float *theta, const float *table,
                          const void *table_half, const float *params, const float *dx_can,
                          float *dparams, float *dtable, float *dx, float *dtheta, bool det,
                          void *ws, hipStream_t st, const ScatterTail *tail) {
    if (cap <= 0) return NVR_OK;
    return run_bwd(g, matrix_cores, 0, n_dev, cap, x, theta, table, table_half, params, dx_can,
                   dparams, dtable, dx, dtheta, true, det, ws, st, tail);
}

int64_t deform_param_count() { return kParams; }

// dst[i] = sum over p < parts (in order) of src[p stride + i], i < 3 count
__global__ void __launch_bounds__(256)
dn_sum_parts(const int32_t *__restrict__ n_dev, int64_t cap, int parts, int64_t stride,
             const float *__restrict__ src, float *__restrict__ dst) {
    const int64_t m = 3 * count_of(0, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int p = 0; p < parts; ++p) acc += src[p * stride + i];
        dst[i] = acc;
    }
}

nvr_status launch_sum_parts(const int32_t *n_dev, int64_t cap, int parts, int64_t stride,
                            const float *src, float *dst, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    dn_sum_parts<<<grid_for(3 * cap, 256, 16384), 256, 0, st>>>(n_dev, cap, parts, stride, src,
                                                                dst);
    NVR_LAUNCHED();
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_deform_workspace(const nvr_grid_desc *g, int64_t n) {
    if (g == nullptr || n < 0 || check_grid(g) != NVR_OK) return 0;
    return std::max(ws_bytes(g, n, false, false), ws_bytes(g, n, true, false));
}

extern "C" int64_t nvr_deform_param_count(void) { return kParams; }

extern "C" nvr_status nvr_deform_fwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const float *theta, const float *table, const float *params,
                                     nvr_dtype math, float *x_can, void *workspace,
                                     nvr_stream stream) {
    clear_error();
    NVR_TRY(check(g, n, workspace));
    NVR_REQUIRE(math == NVR_F32 || math == NVR_F16, NVR_EINVAL, "math must be F32 or F16");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && theta && table && params && x_can, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(theta, 4) && aligned(table, 8) && aligned(params, 4) &&
                    aligned(x_can, 4),
                NVR_EINVAL, "misaligned array");
    return run_fwd(g, math == NVR_F16, n, nullptr, n, x, theta, table, nullptr, params, x_can,
                   false, false, false, workspace, hs(stream));
}

extern "C" nvr_status nvr_deform_bwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const float *theta, const float *table, const float *params,
                                     nvr_dtype math, const float *dx_can, float *dparams,
                                     float *dtable, float *dx, float *dtheta, void *workspace,
                                     nvr_stream stream) {
    clear_error();
    NVR_TRY(check(g, n, workspace));
    NVR_REQUIRE(math == NVR_F32 || math == NVR_F16, NVR_EINVAL, "math must be F32 or F16");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && theta && table && params && dx_can && dparams && dtable, NVR_EINVAL,
                "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(theta, 4) && aligned(table, 8) && aligned(params, 4) &&
                    aligned(dx_can, 4) && aligned(dparams, 4) && aligned(dtable, 8) &&
                    aligned(dx, 4) && aligned(dtheta, 4),
                NVR_EINVAL, "misaligned array");
    return run_bwd(g, math == NVR_F16, n, nullptr, n, x, theta, table, nullptr, params, dx_can,
                   dparams, dtable, dx, dtheta, false, false, workspace, hs(stream));
}
