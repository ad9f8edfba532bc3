// Live look-up table of the fast neighbour search (Sec. 4.2, "On-the-fly
// Radiance Fields"): every canonical voxel centre is carried to the live space
// by the node blend of Eq. 2 over the nodes its canonical KNN entry lists, and
// the live voxel it lands in records the canonical index (the largest one on
// collisions, -1 where none lands).  Two launches: lut_fill (-1 everywhere)
// and lut_build (one thread per canonical voxel, an integer atomic max per
// carried voxel, so the result does not depend on the order).
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

__global__ void __launch_bounds__(256)
lut_build(LutParams p, const uint16_t *__restrict__ knn, const float *__restrict__ node_canon,
          const float *__restrict__ node_dq, int32_t *__restrict__ lut) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)p.c_res * p.c_res * p.c_res;
    for (int64_t kk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; kk < n;
         kk += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(kk % p.c_res), iy = (int)((kk / p.c_res) % p.c_res);
        const int iz = (int)(kk / ((int64_t)p.c_res * p.c_res));
        const float v[3] = {p.c_lo[0] + ((float)ix + 0.5f) * p.c_step[0],
                            p.c_lo[1] + ((float)iy + 0.5f) * p.c_step[1],
                            p.c_lo[2] + ((float)iz + 0.5f) * p.c_step[2]};
        int id[8];
        float d2[8];
        float dmin = 3.4e38f;
        for (int j = 0; j < p.k; ++j) {
            const int i = knn[kk * p.k + j];
            id[j] = i < p.n_nodes ? i : -1;         // 0xFFFF (or any id past the nodes): none
            d2[j] = 3.4e38f;
            if (id[j] >= 0) {
                const float dx = v[0] - node_canon[3 * i], dy = v[1] - node_canon[3 * i + 1];
                const float dz = v[2] - node_canon[3 * i + 2];
                d2[j] = (dx * dx + dy * dy) + dz * dz;
                dmin = d2[j] < dmin ? d2[j] : dmin;
            }
        }
        if (id[0] < 0) continue;                    // the voxel lists no node
        // blend, aligned to the first listed node's hemisphere
        const float *q0 = node_dq + 8 * id[0];
        float b[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < p.k; ++j) {
            if (id[j] < 0) continue;
            const float *q = node_dq + 8 * id[j];
            const float dot = ((q[0] * q0[0] + q[1] * q0[1]) + q[2] * q0[2]) + q[3] * q0[3];
            const float w = expf(-(d2[j] - dmin) * p.inv_r2) * (dot >= 0.f ? 1.f : -1.f);
            for (int e = 0; e < 8; ++e) b[e] += w * q[e];
        }
        const float nrm = sqrtf(((b[0] * b[0] + b[1] * b[1]) + b[2] * b[2]) + b[3] * b[3]);
        if (!(nrm > 0.f)) continue;
        const float inv = 1.f / nrm;
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
        if (!inside) continue;
        const int64_t f = cell[0] + (int64_t)p.l_res * (cell[1] + (int64_t)p.l_res * cell[2]);
        atomicMax(lut + f, (int32_t)kk);
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
    lut_build<<<grid_for(n_canon, 256, 16384), 256, 0, st>>>(p, knn, node_canon, node_dq, lut);
    NVR_LAUNCHED();
    return NVR_OK;
}
