// Density + colour networks on the matrix cores, fp32 accumulation.  The
// forward (features, weights, activations) runs in FT: fp16
// (v_mfma_f32_16x16x32_f16, 10-bit mantissa; weights converted from the fp32
// masters) or bf16 (v_mfma_f32_16x16x32_bf16, weights from a bf16 copy).  All
// backward products (gradients times transposed weights, weight gradients)
// run in bf16 (v_mfma_f32_16x16x32_bf16 / 16x16x16_bf16), whose fp32 exponent
// range needs no loss scaling.  An encoding rounded to bf16 (8-bit mantissa)
// measurably slows training of a hash-grid field; rounded to fp16 it does not.
//
// Layout.  A wave works on column blocks of 16 samples.  In "orientation A"
// a layer computes D = W X (rows = units, columns = samples): lane l holds
// units 4g..4g+3 (g = l/16) of sample l%16, which is exactly the B-operand
// layout the next layer needs once two 16-unit tiles are paired per lane (the
// contraction index of the next layer is permuted to match, and the weight
// fragments are built with the same permutation), so activations never leave
// registers.  Swapping the two operands of the same MFMA gives "orientation
// B", D = X W^T (rows = samples): lane l then holds samples 4g..4g+3 of unit
// l%16, which is the operand layout of the weight-gradient contraction over
// samples.  The backward computes every layer once in orientation A; each
// wave stages its activation and gradient tiles (bf16, unit-major 16 x 16) in
// its own LDS and reads them back as "4 samples of one unit" operands for
// dW = dY X^T (one 8-byte read per tile and lane).  Each layer's dW is formed
// as soon as its output gradient is staged, which then takes the place of the
// activations just consumed: 17 tiles (8.5 KiB) per wave, so that with the
// ReLU masks kept as the packed bf16 activations two waves share a SIMD.
//
// The colour network's SH inputs come from a per-ray table in the step and
// the renderer (rays share their direction), else they are evaluated per
// sample.
//
// Weight fragments (forward W and backward W^T, 38 KiB) are built in LDS once
// per workgroup from the flat parameters; the per-wave weight gradients
// stay in accumulation registers for the whole persistent loop, are summed
// over the workgroup in LDS and written as one partial per workgroup, which a
// final launch adds into dparams (no global atomics, deterministic order).
//
// Supported shape: n_in <= 32, one density hidden layer of 64, 16 density
// outputs, 16 + SH <= 32 colour inputs, one or two colour hidden layers of 64.
#include <type_traits>

#include "common.hpp"
#include "mlp_dev.hpp"
#include "sh_dev.hpp"

namespace nvr {

typedef __attribute__((ext_vector_type(8))) __bf16 bf8;
typedef __attribute__((ext_vector_type(8))) _Float16 h8;
typedef __attribute__((ext_vector_type(4))) short s4;
typedef __attribute__((ext_vector_type(4))) float f4;

// forward operand vector of element type FT
template <typename FT> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf8 type; };
template <> struct Vec8<_Float16> { typedef h8 type; };

constexpr int kMfmaBlock = 256;   // 4 waves

__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma32(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ short bfs(float v) {
    return __builtin_bit_cast(short, (__bf16)v);
}
__device__ __forceinline__ float bf_of_bits(uint16_t b) { return bf16_bits_to_f32(b); }
__device__ __forceinline__ bf8 pair8(f4 a, f4 b) {
    bf8 r;
    r[0] = (__bf16)a[0]; r[1] = (__bf16)a[1]; r[2] = (__bf16)a[2]; r[3] = (__bf16)a[3];
    r[4] = (__bf16)b[0]; r[5] = (__bf16)b[1]; r[6] = (__bf16)b[2]; r[7] = (__bf16)b[3];
    return r;
}
// the same in the forward type
template <typename FT>
__device__ __forceinline__ typename Vec8<FT>::type packf(f4 a, f4 b) {
    typename Vec8<FT>::type r;
    r[0] = (FT)a[0]; r[1] = (FT)a[1]; r[2] = (FT)a[2]; r[3] = (FT)a[3];
    r[4] = (FT)b[0]; r[5] = (FT)b[1]; r[6] = (FT)b[2]; r[7] = (FT)b[3];
    return r;
}
// a stored feature (16-bit pattern of FT) as float
template <typename FT> __device__ __forceinline__ float feat_bits_to_f32(uint16_t b);
template <> __device__ __forceinline__ float feat_bits_to_f32<__bf16>(uint16_t b) {
    return bf16_bits_to_f32(b);
}
template <> __device__ __forceinline__ float feat_bits_to_f32<_Float16>(uint16_t b) {
    return f16_bits_to_f32(b);
}
__device__ __forceinline__ s4 quad(f4 a) {
    s4 r;
    r[0] = bfs(a[0]); r[1] = bfs(a[1]); r[2] = bfs(a[2]); r[3] = bfs(a[3]);
    return r;
}
// max(x, 0) as one integer max on the bits (a negative float is a negative
// int; -0 becomes +0), without the quieting that fmaxf's NaN rules add
__device__ __forceinline__ float relu1(float x) {
    return __int_as_float(max(__float_as_int(x), 0));
}
__device__ __forceinline__ f4 relu4(f4 a) {
    f4 r;
    for (int i = 0; i < 4; ++i) r[i] = relu1(a[i]);
    return r;
}
__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

// Per-wave staging tiles of the backward: 16 units x 16 samples, bf16 bits,
// unit-major.  A lane of orientation A (sample c, rows 4g..4g+3) writes its
// four values; a lane reading operand rows (unit u, samples 4g..4g+3) gets
// 8 contiguous bytes.  The forward's activations take 16 tiles; each layer's
// weight gradient is formed as soon as its output gradient is staged, after
// which the gradient of the layer below takes the place of the activations
// just consumed, so 17 tiles per wave suffice.
constexpr int kTiles = 17;
constexpr int TX = 0, THD = 2, TCI = 6, TH1 = 8, TH2 = 12, TDZ = 16;
__device__ __forceinline__ void stage4(uint16_t *tile, int g, int c, f4 v) {
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[(4 * g + j) * 16 + c] = (uint16_t)bfs(v[j]);
}
// four activations as bf16 bits, two per word (element 2i in the low half)
struct P4 {
    uint32_t lo, hi;
};
typedef __attribute__((ext_vector_type(2))) __bf16 bf2;
__device__ __forceinline__ P4 pk4(f4 v) {
    return P4{__builtin_bit_cast(uint32_t, bf2{(__bf16)v[0], (__bf16)v[1]}),
              __builtin_bit_cast(uint32_t, bf2{(__bf16)v[2], (__bf16)v[3]})};
}
__device__ __forceinline__ void stagep(uint16_t *tile, int g, int c, P4 p) {
    tile[(4 * g + 0) * 16 + c] = (uint16_t)(p.lo & 0xffffu);
    tile[(4 * g + 1) * 16 + c] = (uint16_t)(p.lo >> 16);
    tile[(4 * g + 2) * 16 + c] = (uint16_t)(p.hi & 0xffffu);
    tile[(4 * g + 3) * 16 + c] = (uint16_t)(p.hi >> 16);
}
// gradient through a ReLU whose output was rounded to bf16: passes where the
// output is nonzero (a positive output below bf16's smallest subnormal counts
// as zero)
__device__ __forceinline__ f4 maskp(f4 gr, P4 p) {
    f4 r;
    r[0] = (p.lo & 0x7fffu) ? gr[0] : 0.f;
    r[1] = (p.lo & 0x7fff0000u) ? gr[1] : 0.f;
    r[2] = (p.hi & 0x7fffu) ? gr[2] : 0.f;
    r[3] = (p.hi & 0x7fff0000u) ? gr[3] : 0.f;
    return r;
}
__device__ __forceinline__ s4 unstage(const uint16_t *tile, int u, int g) {
    return *reinterpret_cast<const s4 *>(tile + u * 16 + 4 * g);
}

// contraction index of a 64-wide hidden layer, K-step q, lane group g, slot j
__device__ __forceinline__ int kh(int q, int g, int j) {
    return j < 4 ? 32 * q + 4 * g + j : 32 * q + 16 + 4 * g + (j - 4);
}
// colour input: o units 0..15 then SH coefficients
__device__ __forceinline__ int kc(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4); }
// feature index of slot (g, j) of the encoding operand
template <bool PLANAR>
__device__ __forceinline__ int kin(int g, int j) {
    if (!PLANAR) return 8 * g + j;
    const int p = 2 * g + (j >> 2), e = j & 3;
    return 2 * (p + 8 * (e >> 1)) + (e & 1);
}
// feature index held by row r (0..15) of dfeat output tile m
template <bool PLANAR>
__device__ __forceinline__ int fo(int m, int r) {
    if (!PLANAR) return 16 * m + r;
    const int p = 2 * (r >> 2) + m, e = r & 3;
    return 2 * (p + 8 * (e >> 1)) + (e & 1);
}

template <typename FT>
struct Frags {
    typedef typename Vec8<FT>::type V;
    V d1[4][64];          // forward fragments (FT)
    V d2[2][64];
    V c1[4][64];
    V c2[4][2][64];
    V c3[2][64];
    s4 c3t[4][64];        // backward (transposed) fragments (bf16)
    bf8 c2t[4][2][64];
    bf8 c1t[2][64];
    s4 d2t[4][64];
    bf8 d1t[2][2][64];
};

struct MfmaNet {
    int n_in, nsh, nch;
    int64_t off_d1, off_d2, off_c1, off_c2, off_c3;
    int64_t n_params;
    const float *sh;   // per-ray SH coefficients [rays][16] (zero past nsh), or nullptr
};

// Builds the LDS weight fragments from the flat parameters: fp32 masters for
// an fp16 forward, the bf16 copy for a bf16 forward.
template <int NCH, bool PLANAR, typename FT>
__device__ void build_frags(Frags<FT> &F, const MfmaNet &net, const void *__restrict__ wp) {
    const int cin = 16 + net.nsh;
    auto W = [&](int64_t off, int row, int col, int ncol) -> float {
        const int64_t i = off + (int64_t)row * ncol + col;
        if (std::is_same<FT, _Float16>::value) return reinterpret_cast<const float *>(wp)[i];
        return bf_of_bits(reinterpret_cast<const uint16_t *>(wp)[i]);
    };
    typedef typename Vec8<FT>::type V;
    for (int e = threadIdx.x; e < 64 * 4; e += blockDim.x) {
        const int m = e / 64, l = e % 64, r = l % 16, g = l / 16;
        bf8 v;
        V vf;
        for (int j = 0; j < 8; ++j) {
            const int k = kin<PLANAR>(g, j);
            vf[j] = (FT)(k < net.n_in ? W(net.off_d1, 16 * m + r, k, net.n_in) : 0.f);
        }
        F.d1[m][l] = vf;
        for (int j = 0; j < 8; ++j) {
            const int k = kc(g, j);
            vf[j] = (FT)(k < cin ? W(net.off_c1, 16 * m + r, k, cin) : 0.f);
        }
        F.c1[m][l] = vf;
        s4 t;
        for (int j = 0; j < 4; ++j)
            t[j] = bfs(4 * g + j < 3 ? W(net.off_c3, 4 * g + j, 16 * m + r, 64) : 0.f);
        F.c3t[m][l] = t;
        for (int j = 0; j < 4; ++j) t[j] = bfs(W(net.off_d2, 4 * g + j, 16 * m + r, 64));
        F.d2t[m][l] = t;
        if (NCH == 2) {
            for (int q = 0; q < 2; ++q) {
                for (int j = 0; j < 8; ++j) vf[j] = (FT)W(net.off_c2, 16 * m + r, kh(q, g, j), 64);
                F.c2[m][q][l] = vf;
                for (int j = 0; j < 8; ++j) v[j] = (__bf16)W(net.off_c2, kh(q, g, j), 16 * m + r, 64);
                F.c2t[m][q][l] = v;
            }
        }
    }
    for (int e = threadIdx.x; e < 64 * 2; e += blockDim.x) {
        const int q = e / 64, l = e % 64, r = l % 16, g = l / 16;
        bf8 v;
        V vf;
        for (int j = 0; j < 8; ++j) vf[j] = (FT)W(net.off_d2, r, kh(q, g, j), 64);
        F.d2[q][l] = vf;
        for (int j = 0; j < 8; ++j) vf[j] = (FT)(r < 3 ? W(net.off_c3, r, kh(q, g, j), 64) : 0.f);
        F.c3[q][l] = vf;
        for (int j = 0; j < 8; ++j) v[j] = (__bf16)W(net.off_c1, kh(q, g, j), r, cin);
        F.c1t[q][l] = v;
        for (int m = 0; m < 2; ++m) {
            const int f = fo<PLANAR>(m, r);
            for (int j = 0; j < 8; ++j)
                v[j] = (__bf16)(f < net.n_in ? W(net.off_d1, kh(q, g, j), f, net.n_in) : 0.f);
            F.d1t[m][q][l] = v;
        }
    }
}

// Feature access (16-bit patterns of FT).  Row-major: [cap][n_in]; planar:
// [8][cap][4].
template <bool PLANAR, typename FT>
__device__ __forceinline__ typename Vec8<FT>::type load_feat_a(const uint16_t *__restrict__ feat,
                                                               int64_t s, int64_t cap, int n_in,
                                                               int g, bool valid) {
    typename Vec8<FT>::type v;
    if (!valid) {
        for (int j = 0; j < 8; ++j) v[j] = (FT)0.f;
        return v;
    }
    if (PLANAR) {
        const uint2 a = *reinterpret_cast<const uint2 *>(feat + ((int64_t)(2 * g) * cap + s) * 4);
        const uint2 b = *reinterpret_cast<const uint2 *>(feat + ((int64_t)(2 * g + 1) * cap + s) * 4);
        const uint32_t u[4] = {a.x, a.y, b.x, b.y};
        for (int j = 0; j < 8; ++j)
            v[j] = __builtin_bit_cast(FT, (uint16_t)((u[j >> 1] >> (16 * (j & 1))) & 0xffffu));
        return v;
    }
    if (n_in == 32) {
        const uint4 a = *reinterpret_cast<const uint4 *>(feat + s * 32 + 8 * g);
        const uint32_t u[4] = {a.x, a.y, a.z, a.w};
        for (int j = 0; j < 8; ++j)
            v[j] = __builtin_bit_cast(FT, (uint16_t)((u[j >> 1] >> (16 * (j & 1))) & 0xffffu));
        return v;
    }
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * g + j;
        v[j] = __builtin_bit_cast(FT, k < n_in ? feat[s * n_in + k] : (uint16_t)0);
    }
    return v;
}

template <bool PLANAR, typename FT>
__device__ __forceinline__ float load_feat_one(const uint16_t *__restrict__ feat, int64_t s,
                                               int64_t cap, int n_in, int f) {
    if (f >= n_in) return 0.f;
    if (PLANAR) {
        const int level = f >> 1, plane = level & 7, e = 2 * (level >> 3) + (f & 1);
        return feat_bits_to_f32<FT>(feat[((int64_t)plane * cap + s) * 4 + e]);
    }
    return feat_bits_to_f32<FT>(feat[s * n_in + f]);
}

__device__ __forceinline__ float pick16(const float *sh, int k) {
    float v = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) v = (k == i) ? sh[i] : v;
    return v;
}

// Orientation-A forward of one column block.
template <int NCH, typename FT>
struct FwdA {
    typedef typename Vec8<FT>::type V;
    f4 hd[4];
    V hdb[2];
    f4 o;
    V cin;
    f4 h1[4];
    V h1b[2];
    f4 h2[4];
    V h2b[2];
    f4 z;
    f4 sh4;    // SH coefficients 4g..4g+3 of this lane's sample
};

// SH coefficients 4g..4g+3 of a sample's ray: from the per-ray table when
// there is one, else evaluated from the direction
template <bool SHT>
__device__ __forceinline__ f4 sh4_lane(const MfmaNet &net, int64_t r, const float *dirs, int g) {
    if (SHT) return *reinterpret_cast<const f4 *>(net.sh + 16 * r + 4 * g);
    const int nsh = net.nsh;
    float sh[16];
    for (int k = 0; k < 16; ++k) sh[k] = 0.f;
    sh_eval(dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2],
            nsh == 1 ? 1 : (nsh == 4 ? 2 : (nsh == 9 ? 3 : 4)), sh);
    f4 v;
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        v[j] = k < nsh ? pick16(sh, k) : 0.f;
    }
    return v;
}

template <int NCH, typename FT>
__device__ __forceinline__ void forward_a(const Frags<FT> &F, int l, int g,
                                         typename Vec8<FT>::type xf, f4 s4v,
                                         FwdA<NCH, FT> &a) {
    for (int m = 0; m < 4; ++m) a.hd[m] = relu4(mfma32(F.d1[m][l], xf, zero4()));
    a.hdb[0] = packf<FT>(a.hd[0], a.hd[1]);
    a.hdb[1] = packf<FT>(a.hd[2], a.hd[3]);
    a.o = mfma32(F.d2[0][l], a.hdb[0], zero4());
    a.o = mfma32(F.d2[1][l], a.hdb[1], a.o);
    a.sh4 = s4v;
    a.cin = packf<FT>(a.o, s4v);
    for (int m = 0; m < 4; ++m) a.h1[m] = relu4(mfma32(F.c1[m][l], a.cin, zero4()));
    a.h1b[0] = packf<FT>(a.h1[0], a.h1[1]);
    a.h1b[1] = packf<FT>(a.h1[2], a.h1[3]);
    if (NCH == 2) {
        for (int m = 0; m < 4; ++m) {
            f4 acc = mfma32(F.c2[m][0][l], a.h1b[0], zero4());
            a.h2[m] = relu4(mfma32(F.c2[m][1][l], a.h1b[1], acc));
        }
        a.h2b[0] = packf<FT>(a.h2[0], a.h2[1]);
        a.h2b[1] = packf<FT>(a.h2[2], a.h2[3]);
        a.z = mfma32(F.c3[0][l], a.h2b[0], zero4());
        a.z = mfma32(F.c3[1][l], a.h2b[1], a.z);
    } else {
        a.z = mfma32(F.c3[0][l], a.h1b[0], zero4());
        a.z = mfma32(F.c3[1][l], a.h1b[1], a.z);
    }
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + expf(-x)); }
__device__ __forceinline__ float clamp_sigma(float o) {
    return fminf(fmaxf(o, -kSigmaClamp), kSigmaClamp);
}

// SHT: the colour network's SH inputs come from the per-ray table net.sh
template <int NCH, bool PLANAR, typename FT, bool SHT>
__global__ void __launch_bounds__(kMfmaBlock)
mlp_fwd_mfma(MfmaNet net, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const uint16_t *__restrict__ feat, const float *__restrict__ dirs,
             const int32_t *__restrict__ ray_id, const void *__restrict__ params,
             float *__restrict__ sigma, float *__restrict__ rgb) {
    __shared__ Frags<FT> F;
    build_frags<NCH, PLANAR, FT>(F, net, params);
    __syncthreads();
    const int64_t count = count_of(n, n_dev, cap);
    const int l = threadIdx.x % 64, g = l / 16, c = l % 16;
    const int64_t wave = blockIdx.x * (int64_t)(kMfmaBlock / 64) + threadIdx.x / 64;
    const int64_t nwaves = (int64_t)gridDim.x * (kMfmaBlock / 64);
    for (int64_t cb = wave; cb * 16 < count; cb += nwaves) {
        const int64_t s = cb * 16 + c;
        const bool valid = s < count;
        const typename Vec8<FT>::type xf = load_feat_a<PLANAR, FT>(feat, s, cap, net.n_in, g, valid);
        f4 s4v = zero4();
        if (valid) s4v = sh4_lane<SHT>(net, ray_id ? ray_id[s] : s, dirs, g);
        FwdA<NCH, FT> a;
        forward_a<NCH, FT>(F, l, g, xf, s4v, a);
        if (valid && g == 0) {
            sigma[s] = expf(clamp_sigma(a.o[0]));
            rgb[3 * s] = sigmoidf_(a.z[0]);
            rgb[3 * s + 1] = sigmoidf_(a.z[1]);
            rgb[3 * s + 2] = sigmoidf_(a.z[2]);
        }
    }
}

// Weight-gradient accumulators (orientation D[o][i]: lane holds i = l%16,
// o = 4g..4g+3 of each 16 x 16 tile).
template <int NCH>
struct DW {
    f4 d1[4][2];
    f4 d2[4];
    f4 c1[4][2];
    f4 c2[4][4];
    f4 c3[4];
};

// two waves per SIMD: at most 256 registers per lane (weight-gradient
// accumulators take 160 of them) and 72 KiB of LDS per workgroup
template <int NCH, bool PLANAR, typename FT, bool SHT>
__global__ void __launch_bounds__(kMfmaBlock) __attribute__((amdgpu_waves_per_eu(2)))
mlp_bwd_mfma(MfmaNet net, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const uint16_t *__restrict__ feat, const float *__restrict__ dirs,
             const int32_t *__restrict__ ray_id, const void *__restrict__ params,
             const float *__restrict__ dsigma, const float *__restrict__ drgb,
             float *__restrict__ dfeat, float *__restrict__ partial) {
    __shared__ Frags<FT> F;
    __shared__ uint16_t stage[kMfmaBlock / 64][kTiles][256];
    build_frags<NCH, PLANAR, FT>(F, net, params);
    const int l = threadIdx.x % 64, g = l / 16, c = l % 16;
    uint16_t (*tw)[256] = stage[threadIdx.x / 64];
    for (int i = l; i < kTiles * 256; i += 64) tw[i / 256][i % 256] = 0;   // unused rows stay 0
    __syncthreads();
    const int64_t count = count_of(n, n_dev, cap);
    const int64_t wave = blockIdx.x * (int64_t)(kMfmaBlock / 64) + threadIdx.x / 64;
    const int64_t nwaves = (int64_t)gridDim.x * (kMfmaBlock / 64);
    DW<NCH> acc;
    for (int a = 0; a < 4; ++a) {
        acc.d2[a] = zero4();
        acc.c3[a] = zero4();
        for (int b = 0; b < 2; ++b) {
            acc.d1[a][b] = zero4();
            acc.c1[a][b] = zero4();
        }
        for (int b = 0; b < 4; ++b) acc.c2[a][b] = zero4();
    }
    const int nsh = net.nsh;
    for (int64_t cb = wave; cb * 16 < count; cb += nwaves) {
        const int64_t base = cb * 16;
        const int64_t s = base + c;
        const bool valid = s < count;
        // ------------------------------------------------ orientation A forward
        const typename Vec8<FT>::type xf = load_feat_a<PLANAR, FT>(feat, s, cap, net.n_in, g, valid);
        f4 s4v = zero4();
        float ds = 0.f, dr[3] = {0.f, 0.f, 0.f};
        if (valid) {
            s4v = sh4_lane<SHT>(net, ray_id ? ray_id[s] : s, dirs, g);
            ds = dsigma[s];
            dr[0] = drgb[3 * s];
            dr[1] = drgb[3 * s + 1];
            dr[2] = drgb[3 * s + 2];
        }
        FwdA<NCH, FT> a;
        forward_a<NCH, FT>(F, l, g, xf, s4v, a);
        // activations of this block -> staging tiles (features at their index);
        // from here on the hidden activations are only needed as ReLU masks,
        // which their bf16 bits serve
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kin<PLANAR>(g, j);
            if (k < net.n_in) tw[TX + (k >> 4)][(k & 15) * 16 + c] = (uint16_t)bfs((float)xf[j]);
        }
        P4 phd[4], ph1[4], ph2[4];
        for (int m = 0; m < 4; ++m) {
            phd[m] = pk4(a.hd[m]);
            ph1[m] = pk4(a.h1[m]);
            stagep(tw[THD + m], g, c, phd[m]);
            stagep(tw[TH1 + m], g, c, ph1[m]);
            if (NCH == 2) {
                ph2[m] = pk4(a.h2[m]);
                stagep(tw[TH2 + m], g, c, ph2[m]);
            }
        }
        stage4(tw[TCI], g, c, a.o);
        stage4(tw[TCI + 1], g, c, a.sh4);
        // ------------------------------------------------ orientation A backward,
        // each layer's weight gradient (K = 16 samples) as soon as its operands
        // are staged; a wave's LDS operations complete in order, so its reads
        // see its writes and a tile is rewritten only after it was read
        f4 dz = zero4();
        if (g == 0) {
            for (int i = 0; i < 3; ++i) {
                const float v = sigmoidf_(a.z[i]);
                dz[i] = dr[i] * v * (1.f - v);
            }
        }
        const s4 dzq = quad(dz);
        stage4(tw[TDZ], g, c, dz);
        {   // last colour layer: dz x (h2 or h1)
            const s4 gq = unstage(tw[TDZ], c, g);
            const int th = NCH == 2 ? TH2 : TH1;
            for (int ti = 0; ti < 4; ++ti) acc.c3[ti] = mfma16(gq, unstage(tw[th + ti], c, g), acc.c3[ti]);
        }
        f4 dh1[4];
        if (NCH == 2) {
            f4 dh2[4];
            for (int m = 0; m < 4; ++m) dh2[m] = maskp(mfma16(F.c3t[m][l], dzq, zero4()), ph2[m]);
            const bf8 dh2b0 = pair8(dh2[0], dh2[1]), dh2b1 = pair8(dh2[2], dh2[3]);
            for (int m = 0; m < 4; ++m) stage4(tw[TH2 + m], g, c, dh2[m]);   // over h2
            {   // second colour layer: dh2 x h1
                s4 hq[4];
                for (int ti = 0; ti < 4; ++ti) hq[ti] = unstage(tw[TH1 + ti], c, g);
                for (int mo = 0; mo < 4; ++mo) {
                    const s4 gq = unstage(tw[TH2 + mo], c, g);
                    for (int ti = 0; ti < 4; ++ti) acc.c2[mo][ti] = mfma16(gq, hq[ti], acc.c2[mo][ti]);
                }
            }
            for (int m = 0; m < 4; ++m) {
                f4 t = mfma32(F.c2t[m][0][l], dh2b0, zero4());
                dh1[m] = maskp(mfma32(F.c2t[m][1][l], dh2b1, t), ph1[m]);
            }
        } else {
            for (int m = 0; m < 4; ++m) dh1[m] = maskp(mfma16(F.c3t[m][l], dzq, zero4()), ph1[m]);
        }
        const bf8 dh1b0 = pair8(dh1[0], dh1[1]), dh1b1 = pair8(dh1[2], dh1[3]);
        for (int m = 0; m < 4; ++m) stage4(tw[TH1 + m], g, c, dh1[m]);   // over h1
        {   // first colour layer: dh1 x [o, sh]
            const s4 c0 = unstage(tw[TCI], c, g), c1v = unstage(tw[TCI + 1], c, g);
            for (int mo = 0; mo < 4; ++mo) {
                const s4 gq = unstage(tw[TH1 + mo], c, g);
                acc.c1[mo][0] = mfma16(gq, c0, acc.c1[mo][0]);
                acc.c1[mo][1] = mfma16(gq, c1v, acc.c1[mo][1]);
            }
        }
        f4 dO = mfma32(F.c1t[0][l], dh1b0, zero4());
        dO = mfma32(F.c1t[1][l], dh1b1, dO);
        if (g == 0 && fabsf(a.o[0]) < kSigmaClamp) dO[0] += ds * expf(a.o[0]);
        const s4 dOq = quad(dO);
        stage4(tw[TCI], g, c, dO);   // over [o, sh]
        {   // density output layer: dO x hd
            const s4 gq = unstage(tw[TCI], c, g);
            for (int ti = 0; ti < 4; ++ti) acc.d2[ti] = mfma16(gq, unstage(tw[THD + ti], c, g), acc.d2[ti]);
        }
        f4 dhd[4];
        for (int m = 0; m < 4; ++m) dhd[m] = maskp(mfma16(F.d2t[m][l], dOq, zero4()), phd[m]);
        const bf8 dhdb0 = pair8(dhd[0], dhd[1]), dhdb1 = pair8(dhd[2], dhd[3]);
        for (int m = 0; m < 4; ++m) stage4(tw[THD + m], g, c, dhd[m]);   // over hd
        {   // density hidden layer: dhd x features
            const s4 x0 = unstage(tw[TX], c, g), x1 = unstage(tw[TX + 1], c, g);
            for (int mo = 0; mo < 4; ++mo) {
                const s4 gq = unstage(tw[THD + mo], c, g);
                acc.d1[mo][0] = mfma16(gq, x0, acc.d1[mo][0]);
                acc.d1[mo][1] = mfma16(gq, x1, acc.d1[mo][1]);
            }
        }
        if (dfeat != nullptr) {
            for (int m = 0; m < 2; ++m) {
                f4 df = mfma32(F.d1t[m][0][l], dhdb0, zero4());
                df = mfma32(F.d1t[m][1][l], dhdb1, df);
                if (valid) {
                    if (PLANAR) {
                        *reinterpret_cast<f4 *>(dfeat + ((int64_t)(2 * g + m) * cap + s) * 4) = df;
                    } else if (net.n_in == 32) {
                        *reinterpret_cast<f4 *>(dfeat + s * 32 + 16 * m + 4 * g) = df;
                    } else {
                        for (int i = 0; i < 4; ++i) {
                            const int f = 16 * m + 4 * g + i;
                            if (f < net.n_in) dfeat[s * net.n_in + f] = df[i];
                        }
                    }
                }
            }
        }
    }
    // ---------------------------------------------------- workgroup reduction
    __syncthreads();                       // fragments no longer needed
    float *red = reinterpret_cast<float *>(&F);
    const int np = (int)net.n_params;
    for (int i = threadIdx.x; i < np; i += blockDim.x) red[i] = 0.f;
    __syncthreads();
    const int cin = 16 + nsh;
    // the wavefronts add their sums one after the other (a fixed order, so the
    // partials do not depend on timing); inside one wavefront every lane owns
    // distinct (row, column) entries
    auto put = [&](int64_t off, int ncol, int nrow, int mo, int ti, f4 v) {
        const int col = 16 * ti + c;
        if (col >= ncol) return;
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mo + 4 * g + r;
            if (row < nrow) red[(off - net.off_d1) + row * ncol + col] += v[r];
        }
    };
    const int my_wave = threadIdx.x >> 6;
    for (int wv = 0; wv < kMfmaBlock / 64; ++wv) {
        if (my_wave == wv) {
            for (int mo = 0; mo < 4; ++mo)
                for (int ti = 0; ti < 2; ++ti) {
                    put(net.off_d1, net.n_in, 64, mo, ti, acc.d1[mo][ti]);
                    put(net.off_c1, cin, 64, mo, ti, acc.c1[mo][ti]);
                }
            for (int ti = 0; ti < 4; ++ti) {
                put(net.off_d2, 64, 16, 0, ti, acc.d2[ti]);
                put(net.off_c3, 64, 3, 0, ti, acc.c3[ti]);
            }
            if (NCH == 2)
                for (int mo = 0; mo < 4; ++mo)
                    for (int ti = 0; ti < 4; ++ti) put(net.off_c2, 64, 64, mo, ti, acc.c2[mo][ti]);
        }
        __syncthreads();
    }
    float *dst = partial + (int64_t)blockIdx.x * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = red[i];
}

// Per-ray SH coefficients of the colour network's direction input: [n][16],
// coefficients past nsh are 0.  The samples of a ray share its direction, so
// the networks read these instead of evaluating the basis per sample.
__global__ void __launch_bounds__(256)
sh_rays_kernel(int64_t n, const float *__restrict__ dirs, int nsh, float *__restrict__ out) {
    const int deg = nsh == 1 ? 1 : (nsh == 4 ? 2 : (nsh == 9 ? 3 : 4));
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        float sh[16];
        for (int k = 0; k < 16; ++k) sh[k] = 0.f;
        sh_eval(dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2], deg, sh);
        f4 *o = reinterpret_cast<f4 *>(out + 16 * r);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            o[q] = f4{4 * q < nsh ? sh[4 * q] : 0.f, 4 * q + 1 < nsh ? sh[4 * q + 1] : 0.f,
                      4 * q + 2 < nsh ? sh[4 * q + 2] : 0.f, 4 * q + 3 < nsh ? sh[4 * q + 3] : 0.f};
    }
}

// dparams[i] += sum over workgroups b of partial[b][i]: 64 parameters per
// workgroup, the 16 rows of threads each summing every 16th partial
// (coalesced along i), then the rows are added in LDS.
constexpr int kRedCols = 64, kRedRows = 16;
__global__ void __launch_bounds__(kRedCols * kRedRows)
reduce_partials(int nblocks, int np, const float *__restrict__ partial,
                float *__restrict__ dparams) {
    __shared__ float part[kRedRows][kRedCols];
    const int col = threadIdx.x % kRedCols, row = threadIdx.x / kRedCols;
    const int i = blockIdx.x * kRedCols + col;
    float acc = 0.f;
    if (i < np)
        for (int b = row; b < nblocks; b += kRedRows) acc += partial[(int64_t)b * np + i];
    part[row][col] = acc;
    __syncthreads();
    if (row == 0 && i < np) {
        float t = 0.f;
#pragma unroll
        for (int r = 0; r < kRedRows; ++r) t += part[r][col];
        dparams[i] += t;
    }
}

nvr_status make_mfma_net(const Net &net, MfmaNet *m) {
    NVR_REQUIRE(net.n_density == 2 && net.out[0] == 64, NVR_EUNSUPPORTED,
                "bf16 MFMA networks need one density hidden layer of width 64");
    NVR_REQUIRE(net.n_in <= 32, NVR_EUNSUPPORTED, "bf16 MFMA networks need n_in <= 32");
    NVR_REQUIRE(net.dout == 16, NVR_EUNSUPPORTED, "bf16 MFMA networks need 16 density outputs");
    NVR_REQUIRE(16 + net.n_sh <= 32, NVR_EUNSUPPORTED, "bf16 MFMA networks need 16 + SH <= 32");
    const int nch = net.n_layers - net.n_density - 1;
    NVR_REQUIRE(nch == 1 || nch == 2, NVR_EUNSUPPORTED, "bf16 MFMA networks need 1 or 2 colour hidden layers");
    for (int k = net.n_density; k < net.n_layers - 1; ++k)
        NVR_REQUIRE(net.out[k] == 64, NVR_EUNSUPPORTED, "bf16 MFMA colour hidden width must be 64");
    m->n_in = net.n_in;
    m->nsh = net.n_sh;
    m->nch = nch;
    m->off_d1 = net.woff[0];
    m->off_d2 = net.woff[1];
    m->off_c1 = net.woff[2];
    m->off_c2 = nch == 2 ? net.woff[3] : 0;
    m->off_c3 = net.woff[2 + nch];
    m->n_params = net.woff[net.n_layers];
    m->sh = nullptr;
    NVR_REQUIRE(m->n_params * 4 <= (int64_t)sizeof(Frags<__bf16>), NVR_EUNSUPPORTED, "too many parameters");
    return NVR_OK;
}

unsigned mfma_blocks(int64_t cap) {
    const int64_t cbs = (cap + 15) / 16;
    int64_t b = (cbs + 3) / 4;
    if (b > 512) b = 512;
    if (b < 1) b = 1;
    return (unsigned)b;
}

size_t mfma_workspace(const MfmaNet &m, int64_t cap) {
    return sizeof(float) * (size_t)mfma_blocks(cap) * (size_t)m.n_params;
}

nvr_status mfma_forward(const MfmaNet &m, int64_t n, const int32_t *n_dev, int64_t cap,
                        const uint16_t *feat, bool planar, const float *dirs,
                        const int32_t *ray_id, const void *params, bool f16, float *sigma,
                        float *rgb, hipStream_t st, int blocks = 0) {
    if (cap <= 0) return NVR_OK;
    // the forward keeps no per-workgroup partials: by default one 16-sample block
    // per wave, at most 2048 workgroups (the tuned shape at millions of samples)
    const unsigned gr = blocks > 0 ? (unsigned)blocks : grid_for((cap + 15) / 16, 4, 2048);
#define NVR_FWD(NCH, PL, FT)                                                                   \
    do {                                                                                       \
        if (m.sh)                                                                              \
            mlp_fwd_mfma<NCH, PL, FT, true><<<gr, kMfmaBlock, 0, st>>>(m, n, n_dev, cap, feat, \
                dirs, ray_id, params, sigma, rgb);                                             \
        else                                                                                   \
            mlp_fwd_mfma<NCH, PL, FT, false><<<gr, kMfmaBlock, 0, st>>>(m, n, n_dev, cap, feat,\
                dirs, ray_id, params, sigma, rgb);                                             \
    } while (0)
#define NVR_FWD_T(FT)                                                                          \
    if (m.nch == 2) {                                                                          \
        if (planar) NVR_FWD(2, true, FT); else NVR_FWD(2, false, FT);                          \
    } else {                                                                                   \
        if (planar) NVR_FWD(1, true, FT); else NVR_FWD(1, false, FT);                          \
    }
    if (f16) {
        NVR_FWD_T(_Float16)
    } else {
        NVR_FWD_T(__bf16)
    }
#undef NVR_FWD_T
#undef NVR_FWD
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status mfma_backward(const MfmaNet &m, int64_t n, const int32_t *n_dev, int64_t cap,
                         const uint16_t *feat, bool planar, const float *dirs,
                         const int32_t *ray_id, const void *params, bool f16, const float *dsigma,
                         const float *drgb, float *dparams, float *dfeat, float *partial,
                         hipStream_t st, int blocks = 0) {
    if (cap <= 0) return NVR_OK;
    // the partials workspace holds mfma_blocks(cap) workgroups
    const unsigned gr = blocks > 0 && (unsigned)blocks < mfma_blocks(cap) ? (unsigned)blocks
                                                                          : mfma_blocks(cap);
#define NVR_BWD(NCH, PL, FT)                                                                   \
    do {                                                                                       \
        if (m.sh)                                                                              \
            mlp_bwd_mfma<NCH, PL, FT, true><<<gr, kMfmaBlock, 0, st>>>(m, n, n_dev, cap, feat, \
                dirs, ray_id, params, dsigma, drgb, dfeat, partial);                           \
        else                                                                                   \
            mlp_bwd_mfma<NCH, PL, FT, false><<<gr, kMfmaBlock, 0, st>>>(m, n, n_dev, cap, feat,\
                dirs, ray_id, params, dsigma, drgb, dfeat, partial);                           \
    } while (0)
#define NVR_BWD_T(FT)                                                                          \
    if (m.nch == 2) {                                                                          \
        if (planar) NVR_BWD(2, true, FT); else NVR_BWD(2, false, FT);                          \
    } else {                                                                                   \
        if (planar) NVR_BWD(1, true, FT); else NVR_BWD(1, false, FT);                          \
    }
    if (f16) {
        NVR_BWD_T(_Float16)
    } else {
        NVR_BWD_T(__bf16)
    }
#undef NVR_BWD_T
#undef NVR_BWD
    NVR_LAUNCHED();
    if (dparams == nullptr) return NVR_OK;
    reduce_partials<<<(unsigned)((m.n_params + kRedCols - 1) / kRedCols), kRedCols * kRedRows, 0, st>>>(
        (int)gr, (int)m.n_params, partial,
                                                                   dparams);
    NVR_LAUNCHED();
    return NVR_OK;
}

}  // namespace nvr

#include "launch.hpp"

namespace nvr {

nvr_status mfma_check(const Net &net) {
    MfmaNet m;
    return make_mfma_net(net, &m);
}

size_t mfma_ws_bytes(const Net &net, int64_t cap) {
    MfmaNet m;
    if (make_mfma_net(net, &m) != NVR_OK) return 0;
    return mfma_workspace(m, cap);
}

nvr_status launch_sh_rays(const Net &net, int64_t n_rays, const float *dirs, float *out,
                          hipStream_t st) {
    if (n_rays <= 0) return NVR_OK;
    sh_rays_kernel<<<grid_for(n_rays, 256, 4096), 256, 0, st>>>(n_rays, dirs, net.n_sh, out);
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status mfma_fwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap,
                    const uint16_t *feat, bool planar, const float *dirs, const int32_t *ray_id,
                    const void *params, bool f16, float *sigma, float *rgb, hipStream_t st,
                    int blocks, const float *sh_rays) {
    MfmaNet m;
    NVR_TRY(make_mfma_net(net, &m));
    m.sh = sh_rays;
    return mfma_forward(m, n, n_dev, cap, feat, planar, dirs, ray_id, params, f16, sigma, rgb, st,
                        blocks);
}

nvr_status mfma_bwd(const Net &net, int64_t n, const int32_t *n_dev, int64_t cap,
                    const uint16_t *feat, bool planar, const float *dirs, const int32_t *ray_id,
                    const void *params, bool f16, const float *dsigma, const float *drgb,
                    float *dparams, float *dfeat, void *ws, hipStream_t st, int blocks,
                    const float *sh_rays) {
    MfmaNet m;
    NVR_TRY(make_mfma_net(net, &m));
    m.sh = sh_rays;
    return mfma_backward(m, n, n_dev, cap, feat, planar, dirs, ray_id, params, f16, dsigma, drgb,
                         dparams, dfeat, (float *)ws, st, blocks);
}

}  // namespace nvr
