// Key-frame selection (Sec. 4.2, "Online key frame selection") and the
// human/object assembly by depth (Sec. 4.3, rendering).
//
//   vis_bits     Eq. 5 for every (frame, node): one wave per 64 nodes of a
//                frame, the visibility bits formed with a ballot and stored
//                as two 32-bit words; the projection and the comparison are
//                float32 decisions without fused multiply-adds.
//   human_dist   Eq. 6 of a query frame against every pooled frame: one wave
//                per pooled frame, lanes over pose components and visibility
//                words, a butterfly sum.
//   object_dist  Eq. 7: one thread per pooled frame.
//   assemble     the per-pixel depth test of two renderings.
// The pool bookkeeping (admission, replacement, the spatial-temporal choice)
// is host code over at most a few hundred distances.
#include <algorithm>
#include <numeric>
#include <vector>

#include "common.hpp"

namespace nvr {
namespace {

__global__ void __launch_bounds__(256)
vis_bits(int32_t n_nodes, int32_t n_words, int32_t h, int32_t w, float eps,
         const float *__restrict__ nodes, const float *__restrict__ proj,
         const float *__restrict__ depth, uint32_t *__restrict__ bits) {
#pragma clang fp contract(off)
    const int f = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float *P = proj + 12 * f;
    bool vis = false;
    if (i < n_nodes) {
        const float *x = nodes + ((size_t)f * n_nodes + i) * 3;
        const float x0 = x[0], x1 = x[1], x2 = x[2];
        const float up = ((P[0] * x0 + P[1] * x1) + P[2] * x2) + P[3];
        const float vp = ((P[4] * x0 + P[5] * x1) + P[6] * x2) + P[7];
        const float wp = ((P[8] * x0 + P[9] * x1) + P[10] * x2) + P[11];
        if (wp > 0.f) {
            const float u = floorf(up / wp), v = floorf(vp / wp);
            if (u >= 0.f && u < (float)w && v >= 0.f && v < (float)h) {
                const float d = depth[((size_t)f * h + (int)v) * w + (int)u];
                vis = fabsf(wp - d) < eps;
            }
        }
    }
    const uint64_t m = __ballot(vis);
    const int lane = threadIdx.x & 63;
    const int word = (blockIdx.x * blockDim.x + (threadIdx.x & ~63)) >> 5;
    if (lane == 0 && word < n_words) bits[(size_t)f * n_words + word] = (uint32_t)m;
    if (lane == 32 && word + 1 < n_words)
        bits[(size_t)f * n_words + word + 1] = (uint32_t)(m >> 32);
}

__global__ void __launch_bounds__(256)
human_dist(int32_t n, int32_t n_pose, int32_t n_words, const float *__restrict__ pool_theta,
           const uint32_t *__restrict__ pool_bits, const int32_t *__restrict__ pool_t,
           const float *__restrict__ q_theta, const uint32_t *__restrict__ q_bits, int32_t q_t,
           const float *__restrict__ beta, float beta_vis, float beta_h,
           float *__restrict__ E, int32_t *__restrict__ xor_out) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;                             // whole waves leave together
    float acc = 0.f;
    for (int k = lane; k < n_pose; k += 64) {
        const float d = pool_theta[(size_t)j * n_pose + k] - q_theta[k];
        acc += beta[k] * (d * d);
    }
    int cnt = 0;
    for (int k = lane; k < n_words; k += 64)
        cnt += __popc(pool_bits[(size_t)j * n_words + k] ^ q_bits[k]);
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o);
        cnt += __shfl_xor(cnt, o);
    }
    if (lane == 0) {
        const float dt = (float)(pool_t[j] - q_t);
        E[j] = acc + beta_vis * (float)cnt + beta_h * (dt * dt);
        if (xor_out) xor_out[j] = cnt;
    }
}

__global__ void __launch_bounds__(256)
object_dist(int32_t n, const float *__restrict__ pool_d, const int32_t *__restrict__ pool_t,
            const float *__restrict__ q_d, int32_t q_t, float beta_d, float beta_o,
            float *__restrict__ E) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float a = pool_d[3 * j] - q_d[0], b = pool_d[3 * j + 1] - q_d[1];
    const float c = pool_d[3 * j + 2] - q_d[2];
    const float dt = (float)(pool_t[j] - q_t);
    E[j] = beta_d * (a * a + b * b + c * c) + beta_o * (dt * dt);
}

__global__ void __launch_bounds__(256)
assemble(int64_t n, const float *__restrict__ rgb_a, const float *__restrict__ depth_a,
         const float *__restrict__ alpha_a, const float *__restrict__ rgb_b,
         const float *__restrict__ depth_b, const float *__restrict__ alpha_b,
         float *__restrict__ rgb, float *__restrict__ depth) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float aa = alpha_a[i], ab = alpha_b[i];
        const float za = aa > 0.f ? depth_a[i] / aa : 0.f;
        const float zb = ab > 0.f ? depth_b[i] / ab : 0.f;
        const bool ca = aa >= 0.5f, cb = ab >= 0.5f;
        const bool ta = ca && (!cb || za <= zb);
        const bool tb = cb && !ta;
        for (int c = 0; c < 3; ++c) {
            const float x = rgb_a[3 * i + c], y = rgb_b[3 * i + c];
            rgb[3 * i + c] = ta ? x : tb ? y : x + y;
        }
        depth[i] = ta ? za : tb ? zb : (ab > aa ? zb : za);
    }
}

}  // namespace
}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_visibility(int32_t n_frames, int32_t n_nodes, const float *nodes,
                                     const float *proj, const float *depth, int32_t height,
                                     int32_t width, float eps, uint32_t *bits,
                                     nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n_frames >= 0 && n_frames <= 65535, NVR_EINVAL, "n_frames out of 0..65535");
    NVR_REQUIRE(n_nodes >= 0 && n_nodes <= (1 << 24), NVR_EINVAL, "n_nodes out of 0..2^24");
    NVR_REQUIRE(height >= 1 && width >= 1 && (int64_t)height * width <= (1ll << 28), NVR_EINVAL,
                "depth map size out of range");
    NVR_REQUIRE(eps >= 0.f, NVR_EINVAL, "eps must be non-negative");
    if (n_frames == 0 || n_nodes == 0) return NVR_OK;
    NVR_REQUIRE(nodes && proj && depth && bits, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(nodes, 4) && aligned(proj, 4) && aligned(depth, 4) && aligned(bits, 4),
                NVR_EINVAL, "misaligned array");
    const int32_t n_words = (n_nodes + 31) / 32;
    dim3 grid((n_nodes + 255) / 256, n_frames);
    vis_bits<<<grid, 256, 0, hs(stream)>>>(n_nodes, n_words, height, width, eps, nodes, proj,
                                           depth, bits);
    NVR_LAUNCHED();
    return NVR_OK;
}

extern "C" nvr_status nvr_human_distance(int32_t n, int32_t n_pose, int32_t n_words,
                                         const float *pool_theta, const uint32_t *pool_bits,
                                         const int32_t *pool_t, const float *q_theta,
                                         const uint32_t *q_bits, int32_t q_t, const float *beta,
                                         float beta_vis, float beta_h, float *E,
                                         int32_t *xor_count, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n >= 0 && n <= (1 << 24), NVR_EINVAL, "n out of 0..2^24");
    NVR_REQUIRE(n_pose >= 0 && n_pose <= 4096 && n_words >= 0 && n_words <= (1 << 20),
                NVR_EINVAL, "n_pose or n_words out of range");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(pool_t && E && (n_pose == 0 || (pool_theta && q_theta && beta)) &&
                    (n_words == 0 || (pool_bits && q_bits)),
                NVR_EINVAL, "NULL array");
    human_dist<<<(n + 3) / 4, 256, 0, hs(stream)>>>(n, n_pose, n_words, pool_theta, pool_bits,
                                                    pool_t, q_theta, q_bits, q_t, beta, beta_vis,
                                                    beta_h, E, xor_count);
    NVR_LAUNCHED();
    return NVR_OK;
}

extern "C" nvr_status nvr_object_distance(int32_t n, const float *pool_d, const int32_t *pool_t,
                                          const float *q_d, int32_t q_t, float beta_d,
                                          float beta_o, float *E, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n >= 0 && n <= (1 << 24), NVR_EINVAL, "n out of 0..2^24");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(pool_d && pool_t && q_d && E, NVR_EINVAL, "NULL array");
    object_dist<<<(n + 255) / 256, 256, 0, hs(stream)>>>(n, pool_d, pool_t, q_d, q_t, beta_d,
                                                         beta_o, E);
    NVR_LAUNCHED();
    return NVR_OK;
}

extern "C" nvr_status nvr_pool_step(int32_t *pool, int32_t *n_pool, int32_t cap,
                                    const float *dist, int32_t frame, float gamma,
                                    int32_t *action, int32_t *slot) {
    clear_error();
    NVR_REQUIRE(pool && n_pool && action && slot, NVR_EINVAL, "NULL argument");
    NVR_REQUIRE(cap >= 1 && *n_pool >= 0 && *n_pool <= cap, NVR_EINVAL,
                "pool size out of 0..cap or cap < 1");
    const int32_t n = *n_pool;
    if (n == 0) {
        pool[0] = frame;
        *n_pool = 1;
        *action = NVR_POOL_FIRST;
        *slot = 0;
        return NVR_OK;
    }
    NVR_REQUIRE(dist != nullptr, NVR_EINVAL, "NULL distances");
    for (int j = 0; j < n; ++j)
        if (!(dist[j] > gamma)) {
            *action = NVR_POOL_REJECT;
            *slot = -1;
            return NVR_OK;
        }
    if (n < cap) {
        pool[n] = frame;
        *n_pool = n + 1;
        *action = NVR_POOL_APPEND;
        *slot = n;
        return NVR_OK;
    }
    int best = 0;
    for (int j = 1; j < n; ++j)
        if (dist[j] < dist[best]) best = j;
    pool[best] = frame;
    *action = NVR_POOL_REPLACE;
    *slot = best;
    return NVR_OK;
}

extern "C" nvr_status nvr_pool_select(int32_t n_pool, const float *dist, int32_t m,
                                      int32_t *slots, int32_t *n_out) {
    clear_error();
    NVR_REQUIRE(n_pool >= 0 && m >= 0 && n_out && (n_pool == 0 || (dist && slots)), NVR_EINVAL,
                "bad arguments");
    std::vector<int32_t> order(n_pool);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [dist](int32_t a, int32_t b) { return dist[a] < dist[b]; });
    const int32_t k = std::min(m, n_pool);
    for (int32_t j = 0; j < k; ++j) slots[j] = order[j];
    *n_out = k;
    return NVR_OK;
}

extern "C" nvr_status nvr_depth_assemble(int64_t n, const float *rgb_a, const float *depth_a,
                                         const float *alpha_a, const float *rgb_b,
                                         const float *depth_b, const float *alpha_b, float *rgb,
                                         float *depth, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n >= 0 && n < (1ll << 31), NVR_EINVAL, "n out of 0..2^31");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(rgb_a && depth_a && alpha_a && rgb_b && depth_b && alpha_b && rgb && depth,
                NVR_EINVAL, "NULL array");
    assemble<<<grid_for(n, 256, 16384), 256, 0, hs(stream)>>>(n, rgb_a, depth_a, alpha_a, rgb_b,
                                                              depth_b, alpha_b, rgb, depth);
    NVR_LAUNCHED();
    return NVR_OK;
}
