// Device-side pieces of the hash encoding shared by the encoder kernels.
#pragma once
#include "common.hpp"

namespace nvr {

struct bf16_t { uint16_t v; };
struct f16_t { uint16_t v; };

struct GridParams {
    int L;
    uint32_t mask;                 // T - 1
    int res[NVR_MAX_LEVELS];
    int dense[NVR_MAX_LEVELS];
    uint32_t off[NVR_MAX_LEVELS + 1];
    float lo[3];
    // N_l / side per level and axis as an unevaluated float pair (hi + lo),
    // formed in float64 on the host
    float s_hi[NVR_MAX_LEVELS][3];
    float s_lo[NVR_MAX_LEVELS][3];
    float side[3];                 // aabb_max - aabb_min, float32
};

GridParams make_grid_params(const nvr_grid_desc *g);
nvr_status check_grid(const nvr_grid_desc *g);

struct LevelPos {
    int c[3];        // cell (lower corner)
    float f[3];      // fraction in the cell
    bool inside[3];  // x_hat was inside [0,1] (gradient flows)
};

// Sign of (d_hi + d_lo) * N - m * side, exactly: every product is split into
// two floats with a fused multiply-add, and the six terms are summed into a
// non-overlapping expansion (error-free two-sums), whose most significant
// non-zero component carries the sign.  Only used near a cell face.
inline __host__ __device__ __noinline__ int exact_face_sign(float d_hi, float d_lo, float N, float m, float side) {
#pragma clang fp contract(off)
    float t[6];
    t[0] = d_hi * N;
    t[1] = __builtin_fmaf(d_hi, N, -t[0]);
    t[2] = d_lo * N;
    t[3] = __builtin_fmaf(d_lo, N, -t[2]);
    const float b = m * side;
    t[4] = -b;
    t[5] = -__builtin_fmaf(m, side, -b);
    float h[6];
    int n = 0;
    for (int i = 0; i < 6; ++i) {
        float q = t[i];
        for (int j = 0; j < n; ++j) {
            const float sm = q + h[j];
            const float bv = sm - q;
            const float err = (q - (sm - bv)) + (h[j] - bv);
            q = sm;
            h[j] = err;
        }
        h[n++] = q;
    }
    for (int j = n - 1; j >= 0; --j)
        if (h[j] != 0.f) return h[j] > 0.f ? 1 : -1;
    return 0;
}

// x_l = clamp((x - lo) N_l / side, 0, N_l), cell = min(floor(x_l), N_l - 1), in
// float32 only: x - lo is formed exactly as a pair (two-sum) and multiplied by
// the pair N_l / side (exact head product by fused multiply-add, plus the cross
// terms), which carries x_l to about 2^-47 relative.  Near a cell face the side
// is decided exactly (exact_face_sign), so the cell is the floor of the exact
// x_l; the float32 fraction is that of the pair.
__host__ __device__ __forceinline__ LevelPos level_pos(const GridParams &p, int l, float x, float y,
                                              float z) {
#pragma clang fp contract(off)
    LevelPos r;
    const int N = p.res[l];
    const float fN = (float)N;
    const float xs[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float nlo = -p.lo[a];
        const float d_hi = xs[a] + nlo;
        const float t = d_hi - xs[a];
        const float d_lo = (xs[a] - (d_hi - t)) + (nlo - t);
        const float sh = p.s_hi[l][a], sl = p.s_lo[l][a];
        const float pr = d_hi * sh;
        float e = __builtin_fmaf(d_hi, sh, -pr);
        e = __builtin_fmaf(d_hi, sl, e);
        e = __builtin_fmaf(d_lo, sh, e);
        const float v_hi = pr + e;
        const float v_lo = e - (v_hi - pr);
        // floor of the exact x_l: robust from v_hi away from integers, decided
        // exactly near one
        const float mr = rintf(v_hi);
        int sgn;
        if (fabsf(v_hi - mr) <= 1e-6f * fmaxf(fabsf(mr), 1.f))
            sgn = exact_face_sign(d_hi, d_lo, fN, mr, p.side[a]);
        else
            sgn = v_hi > mr ? 1 : -1;
        const float fl = sgn >= 0 ? mr : mr - 1.f;
        const bool below = d_hi < 0.f;                       // x - lo < 0 (exact sign)
        const bool above = fl > fN || (fl == fN && sgn > 0);  // x_l > N
        r.inside[a] = !below && !above;
        int c;
        float f;
        if (below) {
            c = 0;
            f = 0.f;
        } else if (above || fl >= fN) {   // beyond the box, or x_l == N: the last cell's far face
            c = N - 1;
            f = 1.f;
        } else {
            c = (int)fl;
            f = (v_hi - fl) + v_lo;
            f = fminf(fmaxf(f, 0.f), 1.f);
            if (sgn == 0) f = 0.f;
        }
        r.c[a] = c;
        r.f[a] = f;
    }
    return r;
}

// corner k: bit 0 -> +x, bit 1 -> +y, bit 2 -> +z
__device__ __forceinline__ float corner_weight(const LevelPos &lp, int k) {
    const float wx = (k & 1) ? lp.f[0] : 1.f - lp.f[0];
    const float wy = (k & 2) ? lp.f[1] : 1.f - lp.f[1];
    const float wz = (k & 4) ? lp.f[2] : 1.f - lp.f[2];
    return wx * wy * wz;
}

__device__ __forceinline__ float3 corner_dweight(const LevelPos &lp, int k) {
    const float wx = (k & 1) ? lp.f[0] : 1.f - lp.f[0];
    const float wy = (k & 2) ? lp.f[1] : 1.f - lp.f[1];
    const float wz = (k & 4) ? lp.f[2] : 1.f - lp.f[2];
    const float sx = (k & 1) ? 1.f : -1.f;
    const float sy = (k & 2) ? 1.f : -1.f;
    const float sz = (k & 4) ? 1.f : -1.f;
    return make_float3(sx * wy * wz, sy * wx * wz, sz * wx * wy);
}

__device__ __forceinline__ uint32_t corner_index(const GridParams &p, int l, const LevelPos &lp,
                                                 int k) {
    const uint32_t cx = (uint32_t)(lp.c[0] + (k & 1));
    const uint32_t cy = (uint32_t)(lp.c[1] + ((k >> 1) & 1));
    const uint32_t cz = (uint32_t)(lp.c[2] + ((k >> 2) & 1));
    if (p.dense[l]) {
        const uint32_t s = (uint32_t)p.res[l] + 1u;
        return cx + s * (cy + s * cz);
    }
    return (cx ^ (cy * 2654435761u) ^ (cz * 805459861u)) & p.mask;
}

__device__ __forceinline__ void store2(float *o, float a, float b) {
    o[0] = a;
    o[1] = b;
}
__device__ __forceinline__ void store2(bf16_t *o, float a, float b) {
    const uint32_t v = (uint32_t)f32_to_bf16_bits(a) | ((uint32_t)f32_to_bf16_bits(b) << 16);
    *reinterpret_cast<uint32_t *>(o) = v;
}
__device__ __forceinline__ void store2(f16_t *o, float a, float b) {
    const uint32_t v = (uint32_t)f32_to_f16_bits(a) | ((uint32_t)f32_to_f16_bits(b) << 16);
    *reinterpret_cast<uint32_t *>(o) = v;
}

// Per-tile contribution counts of the binned table scatter, formed by the
// forward gather of a training step (it visits the same corners).
struct TileCounter {
    uint32_t *count;    // [n_tiles], zeroed before the forward
    int tb;             // log2 of the entries per tile
    int level_tiles;    // most tiles one level spans
};

// launchers (grid.hip).  jac (nullable; planar fp16 gather only) receives,
// per sample and level, the level's spatial derivatives in cell units: three
// fp16 pairs (d feature 0, d feature 1 along axis a), level-group-planar
// [8][cap][3 lpg] words (level g + 8 m at [g][s][3m, 3m + 3)), which the
// binned scatter's position gradient reads instead of the table's corners.
nvr_status launch_encode_fwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             void *feat, nvr_dtype feat_dtype, bool planar, hipStream_t st,
                             const TileCounter *counter = nullptr, int chunks = 0,
                             uint32_t *jac = nullptr);
nvr_status launch_encode_bwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             const float *dfeat, float *dtable, float *dx, bool planar,
                             hipStream_t st);

}  // namespace nvr
