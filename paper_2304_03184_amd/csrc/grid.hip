// Multiresolution hash encoding: forward gather + trilinear blend, backward
// scatter-add of table gradients and position gradients.
//
// Two kernel families:
//   * plain   -- float32 table, one thread per (sample, level), global atomics;
//   * split   -- float16 table, level-split across the 8 XCDs: workgroup b
//                serves level group b % 8 (levels g, g+8, g+16, g+24), so each
//                XCD's L2 only ever holds the table slices of its own levels
//                (two 2 MiB fp16 slices at T = 2^19) and its gathers and
//                gradient atomics stay L2-resident.  Workgroups are dispatched
//                round-robin over the XCDs; the mapping only affects locality.
//
// Coordinate transform (both): x_l = clamp((x - lo) N_l / side, 0, N_l) carried
// as a float32 pair (level_pos), so the fractional position keeps float32
// accuracy at N_l = 2048 (one float32 product carries an error of ~1e-4 of a
// cell at the finest level) and the cell is the floor of the exact x_l.
#include "common.hpp"
#include "grid_dev.hpp"

#include <cmath>

namespace nvr {

GridParams make_grid_params(const nvr_grid_desc *g) {
    GridParams p{};
    p.L = g->n_levels;
    p.mask = (uint32_t)((1ull << g->log2_table) - 1);
    for (int l = 0; l < g->n_levels; ++l) {
        p.res[l] = g->res[l];
        p.dense[l] = g->dense[l];
        p.off[l] = (uint32_t)g->offset[l];
    }
    p.off[g->n_levels] = (uint32_t)g->offset[g->n_levels];
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = g->aabb_min[a];
        const double side = (double)g->aabb_max[a] - (double)g->aabb_min[a];
        p.side[a] = (float)side;
        for (int l = 0; l < g->n_levels; ++l) {
            const double s = (double)g->res[l] / side;
            p.s_hi[l][a] = (float)s;
            p.s_lo[l][a] = (float)(s - (double)p.s_hi[l][a]);
        }
    }
    return p;
}

nvr_status check_grid(const nvr_grid_desc *g) {
    NVR_REQUIRE(g != nullptr, NVR_EINVAL, "grid descriptor is NULL");
    NVR_REQUIRE(g->n_levels >= 1 && g->n_levels <= NVR_MAX_LEVELS, NVR_EINVAL,
                "n_levels %d out of 1..32", g->n_levels);
    NVR_REQUIRE(g->n_features == 2, NVR_EUNSUPPORTED, "only n_features == 2 is implemented");
    NVR_REQUIRE(g->log2_table >= 4 && g->log2_table <= 24, NVR_EINVAL,
                "log2_table %d out of 4..24", g->log2_table);
    int64_t T = 1ll << g->log2_table;
    for (int l = 0; l < g->n_levels; ++l) {
        NVR_REQUIRE(g->res[l] >= 1 && g->res[l] <= (1 << 20), NVR_EINVAL, "res[%d] invalid", l);
        int64_t v = (int64_t)(g->res[l] + 1) * (g->res[l] + 1) * (g->res[l] + 1);
        NVR_REQUIRE((g->dense[l] != 0) == (v <= T), NVR_EINVAL, "dense[%d] inconsistent", l);
        const int64_t slice = ((g->dense[l] ? v : T) + 7) / 8 * 8;
        NVR_REQUIRE(g->offset[l + 1] - g->offset[l] == slice, NVR_EINVAL,
                    "offset[%d] inconsistent with the level size", l + 1);
    }
    NVR_REQUIRE(g->offset[0] == 0, NVR_EINVAL, "offset[0] must be 0");
    NVR_REQUIRE(g->offset[g->n_levels] < (1ll << 31), NVR_EINVAL, "table too large");
    for (int a = 0; a < 3; ++a)
        NVR_REQUIRE(g->aabb_max[a] > g->aabb_min[a], NVR_EINVAL, "empty box on axis %d", a);
    return NVR_OK;
}

// ---------------------------------------------------------------- plain
template <typename OutT>
__global__ void __launch_bounds__(256)
encode_fwd_plain(GridParams p, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
                 const float *__restrict__ x, const float2 *__restrict__ table,
                 OutT *__restrict__ feat) {
    const int64_t count = count_of(n, n_dev, cap) * p.L;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / p.L;
        const int l = (int)(i - s * p.L);
        LevelPos lp = level_pos(p, l, x[3 * s], x[3 * s + 1], x[3 * s + 2]);
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float w = corner_weight(lp, k);
            float2 v = table[p.off[l] + corner_index(p, l, lp, k)];
            a0 += w * v.x;
            a1 += w * v.y;
        }
        store2(feat + 2 * i, a0, a1);
    }
}

__global__ void __launch_bounds__(256)
encode_bwd_plain(GridParams p, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
                 const float *__restrict__ x, const float2 *__restrict__ table,
                 const float *__restrict__ dfeat, float *__restrict__ dtable,
                 float *__restrict__ dx) {
    const int64_t count = count_of(n, n_dev, cap) * p.L;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / p.L;
        const int l = (int)(i - s * p.L);
        LevelPos lp = level_pos(p, l, x[3 * s], x[3 * s + 1], x[3 * s + 2]);
        const float g0 = dfeat[2 * i], g1 = dfeat[2 * i + 1];
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float w = corner_weight(lp, k);
            uint32_t e = p.off[l] + corner_index(p, l, lp, k);
            if (g0 != 0.f) unsafeAtomicAdd(dtable + 2 * (size_t)e, w * g0);
            if (g1 != 0.f) unsafeAtomicAdd(dtable + 2 * (size_t)e + 1, w * g1);
            if (dx != nullptr) {
                float2 v = table[e];
                float tg = v.x * g0 + v.y * g1;
                float3 dw = corner_dweight(lp, k);
                d0 += dw.x * tg;
                d1 += dw.y * tg;
                d2 += dw.z * tg;
            }
        }
        if (dx != nullptr) {
            if (lp.inside[0]) unsafeAtomicAdd(dx + 3 * s + 0, d0 * p.s_hi[l][0]);
            if (lp.inside[1]) unsafeAtomicAdd(dx + 3 * s + 1, d1 * p.s_hi[l][1]);
            if (lp.inside[2]) unsafeAtomicAdd(dx + 3 * s + 2, d2 * p.s_hi[l][2]);
        }
    }
}

// ---------------------------------------------------------------- split
// Block b serves level group g = b % 8 over sample chunks b/8, b/8 + nb/8, ...
// PLANAR output: plane g holds, per sample, the LPG levels of the group
// (level g + 8m at elements 2m, 2m+1); otherwise row-major [n][2L].
// COUNT: the corners are also counted per table tile of 2^tb entries (LDS
// histogram per level of the group, added into the global counts at the end).
// i-th 32-bit word of q (i in 0..3)
__device__ __forceinline__ uint32_t pick4(const uint4 &q, uint32_t i) {
    const uint32_t lo = (i & 1u) ? q.y : q.x;
    const uint32_t hi = (i & 1u) ? q.w : q.z;
    return (i & 2u) ? hi : lo;
}

// QUAD (16-byte aligned table, level slices at multiples of 8 entries): the two
// corners of a cell edge along x are fetched with one 16-byte load of the
// aligned group of 4 entries holding the first; the second is in the same group
// unless the group boundary falls between them (a quarter of the cases for both
// the dense and the hashed index), and only then is it loaded on its own.
template <bool PLANAR, typename OutT, bool COUNT, bool QUAD>
__global__ void __launch_bounds__(256)
encode_fwd_split(GridParams p, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
                 const float *__restrict__ x, const uint32_t *__restrict__ table,
                 OutT *__restrict__ feat, TileCounter cnt, uint32_t *__restrict__ jac) {
    extern __shared__ uint32_t hist[];    // COUNT: [lpg][cnt.level_tiles]
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int lpg = (p.L + kXcds - 1) / kXcds;
    if (COUNT) {
        for (int i = threadIdx.x; i < lpg * cnt.level_tiles; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
    }
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < count; c += chunks) {
        const int64_t s = c * blockDim.x + threadIdx.x;
        if (s >= count) break;
        const float px = x[3 * s], py = x[3 * s + 1], pz = x[3 * s + 2];
        for (int m = 0; m < lpg; ++m) {
            const int l = g + kXcds * m;
            float a0 = 0.f, a1 = 0.f;
            if (l < p.L) {
                LevelPos lp = level_pos(p, l, px, py, pz);
                uint32_t e[8], v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = p.off[l] + corner_index(p, l, lp, k);
                if (QUAD) {
                    uint4 q[4];
                    uint32_t far_v[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        q[j] = *reinterpret_cast<const uint4 *>(table + (e[2 * j] & ~3u));
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        far_v[j] = 0u;
                        if ((e[2 * j] ^ e[2 * j + 1]) > 3u) far_v[j] = table[e[2 * j + 1]];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[2 * j] = pick4(q[j], e[2 * j] & 3u);
                        v[2 * j + 1] = (e[2 * j] ^ e[2 * j + 1]) > 3u ? far_v[j]
                                                                      : pick4(q[j], e[2 * j + 1] & 3u);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = table[e[k]];
                }
                if (COUNT) {   // the two corners of an x edge share a tile but rarely
                    uint32_t *h = hist + m * cnt.level_tiles - (int)((uint32_t)p.off[l] >> cnt.tb);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t t0 = e[2 * j] >> cnt.tb, t1 = e[2 * j + 1] >> cnt.tb;
                        atomicAdd(&h[t0], t0 == t1 ? 2u : 1u);
                        if (t0 != t1) atomicAdd(&h[t1], 1u);
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    float w = corner_weight(lp, k);
                    a0 += w * f16_bits_to_f32((uint16_t)(v[k] & 0xffffu));
                    a1 += w * f16_bits_to_f32((uint16_t)(v[k] >> 16));
                }
                if (PLANAR && jac != nullptr) {
                    // the level's spatial derivatives in cell units, d feature f / d axis a
                    // (the trilinear weights' derivatives against the corner values), one
                    // fp16 pair (f = 0, 1) per axis, for the backward's position gradient
                    float j0[3] = {0.f, 0.f, 0.f}, j1[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const float3 dw = corner_dweight(lp, k);
                        const float f0 = f16_bits_to_f32((uint16_t)(v[k] & 0xffffu));
                        const float f1 = f16_bits_to_f32((uint16_t)(v[k] >> 16));
                        j0[0] += dw.x * f0;
                        j0[1] += dw.y * f0;
                        j0[2] += dw.z * f0;
                        j1[0] += dw.x * f1;
                        j1[1] += dw.y * f1;
                        j1[2] += dw.z * f1;
                    }
                    uint32_t *o = jac + ((size_t)g * cap + s) * (3 * lpg) + 3 * m;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        o[a] = (uint32_t)f32_to_f16_bits(j0[a]) | ((uint32_t)f32_to_f16_bits(j1[a]) << 16);
                }
            }
            if (PLANAR) {
                store2(feat + ((size_t)g * cap + s) * (2 * lpg) + 2 * m, a0, a1);
            } else if (l < p.L) {
                store2(feat + (size_t)s * (2 * p.L) + 2 * l, a0, a1);
            }
        }
    }
    if (COUNT) {
        __syncthreads();
        for (int m = 0; m < lpg; ++m) {
            const int l = g + kXcds * m;
            if (l >= p.L) break;
            const int t_lo = (int)((uint32_t)p.off[l] >> cnt.tb);
            const int n_lt = (int)((uint32_t)(p.off[l + 1] - 1) >> cnt.tb) - t_lo + 1;
            for (int t = threadIdx.x; t < n_lt; t += blockDim.x) {
                const uint32_t h = hist[m * cnt.level_tiles + t];
                if (h) atomicAdd(&cnt.count[t_lo + t], h);
            }
        }
    }
}

template <bool PLANAR>
__global__ void __launch_bounds__(256)
encode_bwd_split(GridParams p, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
                 const float *__restrict__ x, const uint32_t *__restrict__ table,
                 const float *__restrict__ dfeat, float *__restrict__ dtable,
                 float *__restrict__ dx_parts) {
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int lpg = (p.L + kXcds - 1) / kXcds;
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < count; c += chunks) {
        const int64_t s = c * blockDim.x + threadIdx.x;
        if (s >= count) break;
        const float px = x[3 * s], py = x[3 * s + 1], pz = x[3 * s + 2];
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
        for (int m = 0; m < lpg; ++m) {
            const int l = g + kXcds * m;
            if (l >= p.L) break;
            float g0, g1;
            if (PLANAR) {
                const float *src = dfeat + ((size_t)g * cap + s) * (2 * lpg) + 2 * m;
                g0 = src[0];
                g1 = src[1];
            } else {
                g0 = dfeat[(size_t)s * (2 * p.L) + 2 * l];
                g1 = dfeat[(size_t)s * (2 * p.L) + 2 * l + 1];
            }
            LevelPos lp = level_pos(p, l, px, py, pz);
            float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float w = corner_weight(lp, k);
                uint32_t e = p.off[l] + corner_index(p, l, lp, k);
                if (g0 != 0.f) unsafeAtomicAdd(dtable + 2 * (size_t)e, w * g0);
                if (g1 != 0.f) unsafeAtomicAdd(dtable + 2 * (size_t)e + 1, w * g1);
                if (dx_parts != nullptr) {
                    uint32_t v = table[e];
                    float tg = f16_bits_to_f32((uint16_t)(v & 0xffffu)) * g0 +
                               f16_bits_to_f32((uint16_t)(v >> 16)) * g1;
                    float3 dw = corner_dweight(lp, k);
                    e0 += dw.x * tg;
                    e1 += dw.y * tg;
                    e2 += dw.z * tg;
                }
            }
            if (lp.inside[0]) d0 += e0 * p.s_hi[l][0];
            if (lp.inside[1]) d1 += e1 * p.s_hi[l][1];
            if (lp.inside[2]) d2 += e2 * p.s_hi[l][2];
        }
        if (dx_parts != nullptr) {
            if (PLANAR) {  // per-group partials, summed by the consumer
                float *o = dx_parts + ((size_t)g * cap + s) * 3;
                o[0] = d0;
                o[1] = d1;
                o[2] = d2;
            } else {       // accumulate into dx[n][3]
                unsafeAtomicAdd(dx_parts + 3 * s + 0, d0);
                unsafeAtomicAdd(dx_parts + 3 * s + 1, d1);
                unsafeAtomicAdd(dx_parts + 3 * s + 2, d2);
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
nvr_status launch_encode_fwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             void *feat, nvr_dtype feat_dtype, bool planar, hipStream_t st,
                             const TileCounter *counter, int chunks_cap, uint32_t *jac) {
    if (cap <= 0) return NVR_OK;
    NVR_REQUIRE(counter == nullptr || (table_dtype != NVR_F32 && planar && feat_dtype == NVR_F16),
                NVR_EUNSUPPORTED, "tile counting needs the planar fp16 gather");
    NVR_REQUIRE(jac == nullptr || (table_dtype != NVR_F32 && planar && feat_dtype == NVR_F16),
                NVR_EUNSUPPORTED, "the stored derivatives need the planar fp16 gather");
    if (table_dtype == NVR_F32) {
        unsigned gr = grid_for(cap * p.L, 256);
        if (feat_dtype == NVR_F32)
            encode_fwd_plain<float><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, (const float2 *)table,
                                                        (float *)feat);
        else if (feat_dtype == NVR_BF16)
            encode_fwd_plain<bf16_t><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, (const float2 *)table,
                                                         (bf16_t *)feat);
        else
            encode_fwd_plain<f16_t><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, (const float2 *)table,
                                                        (f16_t *)feat);
    } else {
        unsigned chunks = grid_for(cap, 256, chunks_cap > 0 ? chunks_cap : 2048);
        unsigned gr = chunks * kXcds;
        const uint32_t *tb = (const uint32_t *)table;
        const TileCounter none{nullptr, 0, 0};
        const bool quad = ((uintptr_t)table & 15u) == 0;   // level slices are 8-entry aligned
#define NVR_SPLIT_FWD(PL, T)                                                                  \
    do {                                                                                      \
        if (quad)                                                                             \
            encode_fwd_split<PL, T, false, true><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, tb, \
                                                                     (T *)feat, none, jac);   \
        else                                                                                  \
            encode_fwd_split<PL, T, false, false><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x,    \
                                                                      tb, (T *)feat, none,    \
                                                                      PL ? jac : nullptr);    \
    } while (0)
        if (counter != nullptr) {
            const int lpg = (p.L + kXcds - 1) / kXcds;
            const size_t lds = sizeof(uint32_t) * lpg * counter->level_tiles;
            if (quad)
                encode_fwd_split<true, f16_t, true, true><<<gr, 256, lds, st>>>(
                    p, n, n_dev, cap, x, tb, (f16_t *)feat, *counter, jac);
            else
                encode_fwd_split<true, f16_t, true, false><<<gr, 256, lds, st>>>(
                    p, n, n_dev, cap, x, tb, (f16_t *)feat, *counter, jac);
        } else if (planar) {
            if (feat_dtype == NVR_F32) NVR_SPLIT_FWD(true, float);
            else if (feat_dtype == NVR_BF16) NVR_SPLIT_FWD(true, bf16_t);
            else NVR_SPLIT_FWD(true, f16_t);
        } else {
            if (feat_dtype == NVR_F32) NVR_SPLIT_FWD(false, float);
            else if (feat_dtype == NVR_BF16) NVR_SPLIT_FWD(false, bf16_t);
            else NVR_SPLIT_FWD(false, f16_t);
        }
#undef NVR_SPLIT_FWD
    }
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status launch_encode_bwd(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                             const float *x, const void *table, nvr_dtype table_dtype,
                             const float *dfeat, float *dtable, float *dx, bool planar,
                             hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    if (table_dtype == NVR_F32) {
        unsigned gr = grid_for(cap * p.L, 256);
        encode_bwd_plain<<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, (const float2 *)table, dfeat,
                                            dtable, dx);
    } else {
        unsigned chunks = grid_for(cap, 256, 1024);
        unsigned gr = chunks * kXcds;
        if (planar)
            encode_bwd_split<true><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x, (const uint32_t *)table,
                                                      dfeat, dtable, dx);
        else
            encode_bwd_split<false><<<gr, 256, 0, st>>>(p, n, n_dev, cap, x,
                                                       (const uint32_t *)table, dfeat, dtable, dx);
    }
    NVR_LAUNCHED();
    return NVR_OK;
}

__global__ void sum_dx_parts(int64_t n, const float *__restrict__ parts, int64_t cap,
                             float *__restrict__ dx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int g = 0; g < kXcds; ++g) acc += parts[(size_t)g * cap * 3 + i];
        dx[i] += acc;
    }
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_grid_init(nvr_grid_desc *g, int32_t n_levels, int32_t n_features,
                                    int32_t log2_table, int32_t res_min, int32_t res_max,
                                    const float *aabb_min, const float *aabb_max) {
    clear_error();
    NVR_REQUIRE(g && aabb_min && aabb_max, NVR_EINVAL, "NULL argument");
    NVR_REQUIRE(n_levels >= 1 && n_levels <= NVR_MAX_LEVELS, NVR_EINVAL, "n_levels out of 1..32");
    NVR_REQUIRE(n_features == 2, NVR_EUNSUPPORTED, "only n_features == 2 is implemented");
    NVR_REQUIRE(log2_table >= 4 && log2_table <= 24, NVR_EINVAL, "log2_table out of 4..24");
    NVR_REQUIRE(res_min >= 1 && res_max >= res_min && res_max <= (1 << 20), NVR_EINVAL,
                "bad resolution range");
    *g = nvr_grid_desc{};
    g->n_levels = n_levels;
    g->n_features = n_features;
    g->log2_table = log2_table;
    const int64_t T = 1ll << log2_table;
    // N_l = floor(N_min * b^l), b = exp((ln N_max - ln N_min) / (L - 1)), float64
    const double b = n_levels > 1 ? std::exp((std::log((double)res_max) - std::log((double)res_min)) /
                                             (double)(n_levels - 1))
                                  : 1.0;
    int64_t off = 0;
    for (int l = 0; l < n_levels; ++l) {
        const int32_t N = (int32_t)std::floor((double)res_min * std::pow(b, (double)l));
        g->res[l] = N;
        const int64_t v = (int64_t)(N + 1) * (N + 1) * (N + 1);
        g->dense[l] = v <= T ? 1 : 0;
        g->offset[l] = off;
        off += ((g->dense[l] ? v : T) + 7) / 8 * 8;   // slices start at multiples of 8 entries
    }
    g->offset[n_levels] = off;
    for (int a = 0; a < 3; ++a) {
        g->aabb_min[a] = aabb_min[a];
        g->aabb_max[a] = aabb_max[a];
    }
    return check_grid(g);
}

extern "C" nvr_status nvr_encode_fwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const void *table, nvr_dtype table_dtype, void *feat,
                                     nvr_dtype feat_dtype, nvr_stream stream) {
    clear_error();
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(n >= 0, NVR_EINVAL, "n < 0");
    NVR_REQUIRE(table_dtype == NVR_F32 || table_dtype == NVR_F16, NVR_EINVAL,
                "table dtype must be F32 or F16");
    NVR_REQUIRE(feat_dtype >= NVR_F32 && feat_dtype <= NVR_BF16, NVR_EINVAL, "bad feat dtype");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && table && feat, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(table, table_dtype == NVR_F32 ? 8 : 4) &&
                    aligned(feat, 4),
                NVR_EINVAL, "misaligned array");
    return launch_encode_fwd(make_grid_params(g), n, nullptr, n, x, table, table_dtype, feat,
                             feat_dtype, false, hs(stream));
}

extern "C" nvr_status nvr_encode_fwd_grouped(const nvr_grid_desc *g, int64_t n, const float *x,
                                             const void *table, void *feat, nvr_stream stream) {
    clear_error();
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(n >= 0 && n < (1ll << 31), NVR_EINVAL, "n out of range");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && table && feat, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(table, 4) && aligned(feat, 4), NVR_EINVAL,
                "misaligned array");
    // 2048 chunks per level group: the shape the step's tuner settles on for
    // large sample counts
    return launch_encode_fwd(make_grid_params(g), n, nullptr, n, x, table, NVR_F16, feat, NVR_F16,
                             true, hs(stream), nullptr, 2048);
}

extern "C" nvr_status nvr_encode_bwd(const nvr_grid_desc *g, int64_t n, const float *x,
                                     const void *table, nvr_dtype table_dtype,
                                     const float *dfeat, float *dtable, float *dx,
                                     nvr_stream stream) {
    clear_error();
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(n >= 0, NVR_EINVAL, "n < 0");
    NVR_REQUIRE(table_dtype == NVR_F32 || table_dtype == NVR_F16, NVR_EINVAL,
                "table dtype must be F32 or F16");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && table && dfeat && dtable, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(table, table_dtype == NVR_F32 ? 8 : 4) &&
                    aligned(dfeat, 4) && aligned(dtable, 4) && aligned(dx, 4),
                NVR_EINVAL, "misaligned array");
    return launch_encode_bwd(make_grid_params(g), n, nullptr, n, x, table, table_dtype, dfeat,
                             dtable, dx, false, hs(stream));
}
