// Live look-up table of the fast neighbour search (Sec. 4.2, "On-the-fly
// Radiance Fields"): every canonical voxel centre is carried to the live space
// by the node blend of Eq. 1 over the nodes its canonical KNN entry lists, and
// the live voxel it lands in records the canonical index (the largest one on
// collisions, -1 where none lands).  Two launches: lut_fill (-1 everywhere)
// and lut_build (one thread per canonical voxel, an integer atomic max per
// carried voxel, so the result does not depend on the order).  The arithmetic
// is float32 with fused multiply-adds, the hardware exponential and reciprocal
// square root; the antipodal sign is a float32 decision without fusion.
#include <algorithm>

#include "common.hpp"

namespace nvr {
namespace {

struct LutParams {
    float c_lo[3], c_step[3];   // canonical voxel centres: lo + (i + 1/2) step
    float l_lo[3], l_scale[3];  // live voxel coordinates: (v - lo) * scale
    int c_res, l_res, k, n_nodes;
    float inv_r2;
};

__global__ void __launch_bounds__(256)
lut_fill(int64_t n, int32_t *__restrict__ lut) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        lut[i] = -1;
}

// One canonical voxel (ix, iy, iz) = kk: its listed ids (KV = 8 or 4: one 16- or
// 8-byte load, knn aligned to that; KV = 0: element loads for any k), the node
// positions and dual quaternions (STAGED: from the workgroup's copy in local
// memory; otherwise from global memory, two 16-byte loads per node when KV != 0),
// the blend of Eq. 1, and the atomic max of kk on the live voxel it lands in.
template <int KV, bool STAGED>
__device__ __forceinline__ void carry_voxel(const LutParams &p, uint32_t kk, uint32_t ix,
                                            uint32_t iy, uint32_t iz,
                                            const uint16_t *__restrict__ knn,
                                            const float *__restrict__ node_canon,
                                            const float *__restrict__ node_dq,
                                            const float4 *__restrict__ sm,
                                            int32_t *__restrict__ lut) {
    const int k = KV ? KV : p.k;
    const float v[3] = {p.c_lo[0] + ((float)ix + 0.5f) * p.c_step[0],
                        p.c_lo[1] + ((float)iy + 0.5f) * p.c_step[1],
                        p.c_lo[2] + ((float)iz + 0.5f) * p.c_step[2]};
    int id[8];
    if constexpr (KV == 8) {
        const uint4 w4 = *reinterpret_cast<const uint4 *>(knn + 8 * (size_t)kk);
        const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
        for (int j = 0; j < 4; ++j) {
            id[2 * j] = (int)(w[j] & 0xFFFFu);
            id[2 * j + 1] = (int)(w[j] >> 16);
        }
    } else if constexpr (KV == 4) {
        const uint2 w2 = *reinterpret_cast<const uint2 *>(knn + 4 * (size_t)kk);
        id[0] = (int)(w2.x & 0xFFFFu);
        id[1] = (int)(w2.x >> 16);
        id[2] = (int)(w2.y & 0xFFFFu);
        id[3] = (int)(w2.y >> 16);
    } else {
        for (int j = 0; j < k; ++j) id[j] = knn[(size_t)kk * k + j];
    }
    float d2[8];
    float dmin = 3.4e38f;
    for (int j = 0; j < k; ++j) {
        const int i = id[j];
        if (i >= p.n_nodes) id[j] = -1;             // 0xFFFF (or any id past the nodes): none
        d2[j] = 3.4e38f;
        if (id[j] >= 0) {
            float x[3];
            if constexpr (STAGED) {
                const float4 x4 = sm[2 * p.n_nodes + i];
                x[0] = x4.x; x[1] = x4.y; x[2] = x4.z;
            } else {
                x[0] = node_canon[3 * i]; x[1] = node_canon[3 * i + 1]; x[2] = node_canon[3 * i + 2];
            }
            const float dx = v[0] - x[0], dy = v[1] - x[1], dz = v[2] - x[2];
            d2[j] = dx * dx + dy * dy + dz * dz;
            dmin = d2[j] < dmin ? d2[j] : dmin;
        }
    }
    if (id[0] < 0) return;                          // the voxel lists no node
    // blend, aligned to the first listed node's hemisphere
    float q0[4];
    float b[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < k; ++j) {
        if (id[j] < 0) continue;
        float q[8];
        if constexpr (STAGED || KV != 0) {
            const float4 *src = STAGED ? sm + 2 * id[j]
                                       : reinterpret_cast<const float4 *>(node_dq + 8 * id[j]);
            const float4 a = src[0], c = src[1];
            q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w;
            q[4] = c.x; q[5] = c.y; q[6] = c.z; q[7] = c.w;
        } else {
            for (int e = 0; e < 8; ++e) q[e] = node_dq[8 * id[j] + e];
        }
        if (j == 0)
            for (int e = 0; e < 4; ++e) q0[e] = q[e];
        float dot;
        {
#pragma clang fp contract(off)
            // the sign is a float32 decision taken in this order, without fusion
            dot = ((q[0] * q0[0] + q[1] * q0[1]) + q[2] * q0[2]) + q[3] * q0[3];
        }
        const float w = __expf(-(d2[j] - dmin) * p.inv_r2);
        const float sw = dot >= 0.f ? w : -w;
        for (int e = 0; e < 8; ++e) b[e] += sw * q[e];
    }
    const float nn = b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3];
    if (!(nn > 0.f)) return;
    const float inv = rsqrtf(nn);
    const float rw = b[0] * inv, rx = b[1] * inv, ry = b[2] * inv, rz = b[3] * inv;
    const float dw = b[4] * inv, dx = b[5] * inv, dy = b[6] * inv, dz = b[7] * inv;
    // R(c_r) v = v + 2 w (r x v) + 2 r x (r x v)
    const float tx = 2.f * (ry * v[2] - rz * v[1]);
    const float ty = 2.f * (rz * v[0] - rx * v[2]);
    const float tz = 2.f * (rx * v[1] - ry * v[0]);
    const float rv[3] = {v[0] + rw * tx + (ry * tz - rz * ty),
                         v[1] + rw * ty + (rz * tx - rx * tz),
                         v[2] + rw * tz + (rx * ty - ry * tx)};
    // translation 2 vec(c_d conj(c_r))
    const float tr[3] = {2.f * (-dw * rx + dx * rw - dy * rz + dz * ry),
                         2.f * (-dw * ry + dx * rz + dy * rw - dz * rx),
                         2.f * (-dw * rz - dx * ry + dy * rx + dz * rw)};
    int cell[3];
    bool inside = true;
    for (int a = 0; a < 3; ++a) {
        const float u = ((rv[a] + tr[a]) - p.l_lo[a]) * p.l_scale[a];
        const float f = floorf(u);
        inside = inside && f >= 0.f && f < (float)p.l_res;
        cell[a] = inside ? (int)f : 0;
    }
    if (!inside) return;
    const uint32_t f = (uint32_t)cell[0] +
                       (uint32_t)p.l_res * ((uint32_t)cell[1] + (uint32_t)p.l_res * cell[2]);
    atomicMax(lut + f, (int32_t)kk);
}

// Grid-stride loop over the canonical voxels (at most 2^30); the voxel
// coordinates advance by the stride's base-res digits, so only the first voxel
// of each thread takes a division.  STAGED: the workgroup first copies the node
// table into local memory ([n][2] dual-quaternion halves, then [n] positions
// padded to 16 bytes: 48 n bytes).
template <int KV, bool STAGED>
__global__ void __launch_bounds__(512)
lut_build(LutParams p, const uint16_t *__restrict__ knn, const float *__restrict__ node_canon,
          const float *__restrict__ node_dq, int32_t *__restrict__ lut) {
    extern __shared__ float4 sm[];
    if constexpr (STAGED) {
        for (int i = threadIdx.x; i < p.n_nodes; i += blockDim.x) {
            const float *q = node_dq + 8 * i;
            sm[2 * i] = make_float4(q[0], q[1], q[2], q[3]);
            sm[2 * i + 1] = make_float4(q[4], q[5], q[6], q[7]);
            sm[2 * p.n_nodes + i] =
                make_float4(node_canon[3 * i], node_canon[3 * i + 1], node_canon[3 * i + 2], 0.f);
        }
        __syncthreads();
    }
    const uint32_t res = (uint32_t)p.c_res;
    const uint32_t n = res * res * res;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t s_row = stride / res, sx = stride - s_row * res;
    const uint32_t sz = s_row / res, sy = s_row - sz * res;
    uint32_t kk = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t row = kk / res;
    uint32_t ix = kk - row * res, iz = row / res, iy = row - iz * res;
    for (; kk < n; kk += stride) {
        carry_voxel<KV, STAGED>(p, kk, ix, iy, iz, knn, node_canon, node_dq, sm, lut);
        ix += sx;
        const uint32_t cx = ix >= res ? 1u : 0u;
        ix -= cx * res;
        iy += sy + cx;
        const uint32_t cy = iy >= res ? 1u : 0u;
        iy -= cy * res;
        iz += sz + cy;
    }
}

}  // namespace
}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_live_lut(const nvr_lut_desc *d, const uint16_t *knn,
                                   const float *node_canon, const float *node_dq, int32_t *lut,
                                   nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(d != nullptr, NVR_EINVAL, "descriptor is NULL");
    NVR_REQUIRE(d->canon_res >= 1 && d->canon_res <= 1024 && d->live_res >= 1 &&
                    d->live_res <= 1024,
                NVR_EINVAL, "resolutions out of 1..1024");
    NVR_REQUIRE(d->k_nodes >= 1 && d->k_nodes <= 8, NVR_EINVAL, "k_nodes out of 1..8");
    NVR_REQUIRE(d->n_nodes >= 1 && d->n_nodes <= 65535, NVR_EINVAL, "n_nodes out of 1..65535");
    NVR_REQUIRE(d->r_ed > 0.f, NVR_EINVAL, "r_ed must be positive");
    for (int a = 0; a < 3; ++a)
        NVR_REQUIRE(d->canon_max[a] > d->canon_min[a] && d->live_max[a] > d->live_min[a],
                    NVR_EINVAL, "empty box on axis %d", a);
    NVR_REQUIRE(knn && node_canon && node_dq && lut, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(knn, 2) && aligned(node_canon, 4) && aligned(node_dq, 4) &&
                    aligned(lut, 4),
                NVR_EINVAL, "misaligned array");
    LutParams p;
    for (int a = 0; a < 3; ++a) {
        p.c_lo[a] = d->canon_min[a];
        p.c_step[a] = (float)(((double)d->canon_max[a] - d->canon_min[a]) / d->canon_res);
        p.l_lo[a] = d->live_min[a];
        p.l_scale[a] = (float)(d->live_res / ((double)d->live_max[a] - d->live_min[a]));
    }
    p.c_res = d->canon_res;
    p.l_res = d->live_res;
    p.k = d->k_nodes;
    p.n_nodes = d->n_nodes;
    p.inv_r2 = (float)(1.0 / ((double)d->r_ed * d->r_ed));
    const hipStream_t st = hs(stream);
    const int64_t n_live = (int64_t)d->live_res * d->live_res * d->live_res;
    const int64_t n_canon = (int64_t)d->canon_res * d->canon_res * d->canon_res;
    lut_fill<<<grid_for(n_live, 256, 16384), 256, 0, st>>>(n_live, lut);
    NVR_LAUNCHED();
    const bool vec = aligned(node_dq, 16) && aligned(knn, 2 * (size_t)d->k_nodes);
    const int kv = vec && d->k_nodes == 8 ? 8 : vec && d->k_nodes == 4 ? 4 : 0;
    const size_t lds = (size_t)48 * d->n_nodes;
    if (lds <= 65536) {
        // node table staged per workgroup: as many resident workgroups as the
        // 160 KB of local memory per compute unit holds (1..4), each looping
        const int64_t per_cu = std::min<int64_t>(4, std::max<int64_t>(1, 163840 / (int64_t)lds));
        const unsigned g = (unsigned)std::min<int64_t>((n_canon + 511) / 512, 256 * per_cu);
        if (kv == 8)
            lut_build<8, true><<<g, 512, lds, st>>>(p, knn, node_canon, node_dq, lut);
        else if (kv == 4)
            lut_build<4, true><<<g, 512, lds, st>>>(p, knn, node_canon, node_dq, lut);
        else
            lut_build<0, true><<<g, 512, lds, st>>>(p, knn, node_canon, node_dq, lut);
    } else {
        const unsigned g = grid_for(n_canon, 512, 16384);
        if (kv == 8)
            lut_build<8, false><<<g, 512, 0, st>>>(p, knn, node_canon, node_dq, lut);
        else if (kv == 4)
            lut_build<4, false><<<g, 512, 0, st>>>(p, knn, node_canon, node_dq, lut);
        else
            lut_build<0, false><<<g, 512, 0, st>>>(p, knn, node_canon, node_dq, lut);
    }
    NVR_LAUNCHED();
    return NVR_OK;
}
