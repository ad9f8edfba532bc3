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
    double inv_side[3];
};

GridParams make_grid_params(const nvr_grid_desc *g);
nvr_status check_grid(const nvr_grid_desc *g);

struct LevelPos {
    int c[3];        // cell (lower corner)
    float f[3];      // fraction in the cell
    bool inside[3];  // x_hat was inside [0,1] (gradient flows)
};

// x_l = clamp((x - lo) / side, 0, 1) * N_l in float64; cell = min(floor, N-1).
__device__ __forceinline__ LevelPos level_pos(const GridParams &p, int l, float x, float y,
                                              float z) {
    LevelPos r;
    const int N = p.res[l];
    const float xs[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double u = ((double)xs[a] - (double)p.lo[a]) * p.inv_side[a];
        r.inside[a] = (u >= 0.0) && (u <= 1.0);
        u = fmin(fmax(u, 0.0), 1.0);
        const double v = u * (double)N;
        int c = (int)floor(v);
        if (c > N - 1) c = N - 1;
        r.c[a] = c;
        r.f[a] = (float)(v - (double)c);
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

// launchers (grid.hip)
nvr_status launch_encode_fwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             void *feat, nvr_dtype feat_dtype, bool planar, hipStream_t st,
                             const TileCounter *counter = nullptr, int chunks = 0);
nvr_status launch_encode_bwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             const float *dfeat, float *dtable, float *dx, bool planar,
                             hipStream_t st);

}  // namespace nvr
