// Hybrid warp of live samples into the canonical space and its backward.
//
// Per sample (one thread): inverse skinning over the k nearest joints, then
// the inverse dual-quaternion blend over the nodes listed for the sample's
// live voxel (the O(1) look-up of the paper's fast search), then the rigid
// transform of the blend.  The joint table lives in LDS; node motions and
// positions are read through the caches (1024 nodes x 44 B).
//
// Backward recomputes the forward and accumulates node-motion gradients in
// an LDS copy of the gradient table (when it fits in 64 KiB), flushed once
// per workgroup with global atomics; otherwise it uses global atomics.
//
// Float32 decisions (no fused multiply-add, one rounding per operation): the
// look-up voxel, the squared joint distances that choose the joints, and the
// sign of <q_r,i, q_r,first>.
#include "common.hpp"

namespace nvr {

constexpr int kMaxJoints = 64;
constexpr int kMaxKJ = 8;
constexpr int kMaxKN = 16;
constexpr int kWarpBlock = 256;

struct WarpParams {
    int n_joints, k_joints, n_nodes, k_nodes, n_frames, lut_res;
    float inv_two_sigma2;      // 1 / (2 sigma_skin^2)
    float inv_r2;              // 1 / r^2
    float lut_lo[3], lut_scale[3];
};

struct Q4 { float w, x, y, z; };

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 add3(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 mul3(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }

// v rotated by unit quaternion (w, u): v + 2w (u x v) + 2 u x (u x v)
__device__ __forceinline__ float3 qrot(float w, float3 u, float3 v) {
    const float3 uv = cross3(u, v);
    return add3(add3(v, mul3(2.f * w, uv)), mul3(2.f, cross3(u, uv)));
}

// ---- float32 decisions: one rounding per operation, no contraction
__device__ __forceinline__ float joint_d2(float3 x, const float *J) {
#pragma clang fp contract(off)
    const float dx = x.x - J[0];
    const float dy = x.y - J[1];
    const float dz = x.z - J[2];
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ int lut_cell(float x, float lo, float scale, int res) {
#pragma clang fp contract(off)
    const float u = (x - lo) * scale;
    const int c = (int)floorf(u);
    return c < 0 ? 0 : (c > res - 1 ? res - 1 : c);
}

__device__ __forceinline__ float sign_dot(const float *q, const float *q0) {
#pragma clang fp contract(off)
    const float dot = ((q[0] * q0[0] + q[1] * q0[1]) + q[2] * q0[2]) + q[3] * q0[3];
    return dot >= 0.f ? 1.f : -1.f;
}

// KJ, KN: compile-time bounds of k_joints and k_nodes (4 or 8, 8 or 16), so
// that every per-sample list is indexed by constants and lives in registers
template <int KJ, int KN>
struct WarpFwd {
    int jsel[KJ];
    float lw[KJ];
    int nid[KN];
    float w[KN];
    float s[KN];
    float3 y;
    float c[8];
    float nr;
    int frame;
    float3 z;
};

// Forward of one sample; `J` is the joint table in global memory: the same
// address for every lane, read through the scalar cache.
template <int KJ, int KN>
__device__ __forceinline__ void warp_one(const WarpParams &p, const float *__restrict__ J,
                                         const nvr_warp_rig &rig, float3 x, int frame,
                                         WarpFwd<KJ, KN> &f) {
    f.frame = frame;
    // --- choose the k nearest joints by float32 squared distance (ties: lower
    // index): each joint passes down the sorted list, swapping with every entry
    // it is strictly nearer than (selects, no divergent branches)
    float bd[KJ];
#pragma unroll
    for (int k = 0; k < KJ; ++k) {
        bd[k] = INFINITY;
        f.jsel[k] = 0x7fffffff;
    }
    for (int j = 0; j < p.n_joints; ++j) {
        float cur = joint_d2(x, J + 3 * j);
        int cj = j;
#pragma unroll
        for (int k = 0; k < KJ; ++k) {
            if (k < p.k_joints) {
                const bool nearer = cur < bd[k];
                const float tb = bd[k];
                const int tj = f.jsel[k];
                bd[k] = nearer ? cur : tb;
                f.jsel[k] = nearer ? cj : tj;
                cur = nearer ? tb : cur;
                cj = nearer ? tj : cj;
            }
        }
    }
    // --- skinning weights and y = sum_j w_j (R_j x + t_j)
    float wsum = 0.f;
#pragma unroll
    for (int k = 0; k < KJ; ++k) {
        f.lw[k] = 0.f;
        if (k < p.k_joints) {
            f.lw[k] = expf(-(bd[k] - bd[0]) * p.inv_two_sigma2);
            wsum += f.lw[k];
        }
    }
    const float iw = 1.f / wsum;
    float3 y = make_float3(0.f, 0.f, 0.f);
    const float *B = rig.bones + (size_t)frame * p.n_joints * 12;
#pragma unroll
    for (int k = 0; k < KJ; ++k) {
        if (k >= p.k_joints) continue;
        f.lw[k] *= iw;
        const float *M = B + 12 * f.jsel[k];
        const float3 yj = make_float3(M[0] * x.x + M[1] * x.y + M[2] * x.z + M[3],
                                      M[4] * x.x + M[5] * x.y + M[6] * x.z + M[7],
                                      M[8] * x.x + M[9] * x.y + M[10] * x.z + M[11]);
        y = add3(y, mul3(f.lw[k], yj));
    }
    f.y = y;
    // --- node set of the live voxel
    int v[3];
    const float xs[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = lut_cell(xs[a], p.lut_lo[a], p.lut_scale[a], p.lut_res);
    const size_t vox = (size_t)v[0] + (size_t)p.lut_res * ((size_t)v[1] + (size_t)p.lut_res * v[2]);
    const uint16_t *ids = rig.lut + ((size_t)frame * p.lut_res * p.lut_res * p.lut_res + vox) * p.k_nodes;
    const float *DQ = rig.node_dq + (size_t)frame * p.n_nodes * 8;
    const float *G = rig.node_pos + (size_t)frame * p.n_nodes * 3;
    float e2[KN];
    float e2min = INFINITY;
#pragma unroll
    for (int k = 0; k < KN; ++k) {
        f.nid[k] = 0;
        e2[k] = INFINITY;
        if (k >= p.k_nodes) continue;
        int id = ids[k];
        id = id < p.n_nodes ? id : p.n_nodes - 1;   // ids are documented to be < n_nodes
        f.nid[k] = id;
        const float3 g = make_float3(G[3 * id], G[3 * id + 1], G[3 * id + 2]);
        const float3 dd = sub3(y, g);
        e2[k] = dot3(dd, dd);
        e2min = fminf(e2min, e2[k]);
    }
    const float *q0 = DQ + 8 * f.nid[0];
    float b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KN; ++k) {
        f.s[k] = 0.f;
        f.w[k] = 0.f;
        if (k >= p.k_nodes) continue;
        const float *q = DQ + 8 * f.nid[k];
        float qq[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) qq[c] = q[c];
        f.s[k] = sign_dot(qq, q0);
        f.w[k] = expf(-(e2[k] - e2min) * p.inv_r2);
        const float sw = f.s[k] * f.w[k];
        // conjugate of both parts: (w, -x, -y, -z)
        b[0] += sw * qq[0];
        b[1] -= sw * qq[1];
        b[2] -= sw * qq[2];
        b[3] -= sw * qq[3];
        b[4] += sw * qq[4];
        b[5] -= sw * qq[5];
        b[6] -= sw * qq[6];
        b[7] -= sw * qq[7];
    }
    const float nr = sqrtf(b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3]);
    f.nr = nr;
    const float inr = 1.f / nr;
#pragma unroll
    for (int c = 0; c < 8; ++c) f.c[c] = b[c] * inr;
    const float3 vr = make_float3(f.c[1], f.c[2], f.c[3]);
    const float3 vd = make_float3(f.c[5], f.c[6], f.c[7]);
    const float wr = f.c[0], wd = f.c[4];
    // translation 2 vec(c_d conj(c_r)) = 2 (w_r v_d - w_d v_r + v_r x v_d)
    const float3 tr = mul3(2.f, add3(sub3(mul3(wr, vd), mul3(wd, vr)), cross3(vr, vd)));
    f.z = add3(qrot(wr, vr, y), tr);
}

template <int KJ, int KN>
__global__ void __launch_bounds__(kWarpBlock)
warp_fwd_kernel(WarpParams p, nvr_warp_rig rig, const float *__restrict__ J, int64_t n,
                const int32_t *__restrict__ n_dev, int64_t cap, const float *__restrict__ x,
                const int32_t *__restrict__ frame, float *__restrict__ xc) {
    const int64_t count = count_of(n, n_dev, cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        WarpFwd<KJ, KN> f;
        const int fr = frame ? frame[i] : 0;
        warp_one<KJ, KN>(p, J, rig, make_float3(x[3 * i], x[3 * i + 1], x[3 * i + 2]), fr, f);
        xc[3 * i] = f.z.x;
        xc[3 * i + 1] = f.z.y;
        xc[3 * i + 2] = f.z.z;
    }
}

// LDS_ACC: node-motion gradients summed per workgroup in LDS; LDS_BONES: bone
// gradients likewise (every sample touches the same few joints, so global
// atomics per sample would serialise on them).
constexpr int kRun = 8;   // consecutive samples per thread in the backward
constexpr int kNodeStride = 9;   // LDS words per node in the backward's gradient table
// adds a joint slot's register sums into the bone-gradient table
#define NVR_FLUSH_BONE(k)                                                                      \
    do {                                                                                       \
        for (int e_ = 0; e_ < 12; ++e_) {                                                      \
            if (LDS_BONES) atomicAdd(bacc + (size_t)bkey[k] * 12 + e_, bsum[k][e_]);           \
            else unsafeAtomicAdd(d_bones + (size_t)bkey[k] * 12 + e_, bsum[k][e_]);            \
        }                                                                                      \
    } while (0)

// adds a node slot's register sums into the node-gradient table
#define NVR_FLUSH_NODE(k)                                                                      \
    do {                                                                                       \
        for (int c_ = 0; c_ < 8; ++c_) {                                                       \
            if (LDS_ACC) atomicAdd(acc + (size_t)nkey[k] * kNodeStride + c_, nsum[k][c_]);     \
            else unsafeAtomicAdd(d_dq + (size_t)nkey[k] * 8 + c_, nsum[k][c_]);               \
        }                                                                                      \
    } while (0)

template <int KJ, int KN, bool LDS_ACC, bool LDS_BONES>
__global__ void __launch_bounds__(kWarpBlock)
warp_bwd_kernel(WarpParams p, nvr_warp_rig rig, const float *__restrict__ J, int64_t n,
                const int32_t *__restrict__ n_dev, int64_t cap, const float *__restrict__ x,
                const int32_t *__restrict__ frame, const float *__restrict__ gz_parts,
                int n_parts, int64_t part_stride, float *__restrict__ d_dq,
                float *__restrict__ d_bones, float *__restrict__ dx_live) {
    extern __shared__ float lds[];
    const int n_bacc = p.n_frames * p.n_joints * 12;
    float *bacc = lds;                                // [n_frames * n_joints * 12] if LDS_BONES
    // [n_frames * n_nodes][kNodeStride] if LDS_ACC: a node's 8 sums padded to 9
    // words, so that lanes adding to different nodes fall into different banks
    float *acc = bacc + (LDS_BONES ? n_bacc : 0);
    const int n_acc = p.n_frames * p.n_nodes * kNodeStride;
    if (LDS_ACC)
        for (int i = threadIdx.x; i < n_acc; i += blockDim.x) acc[i] = 0.f;
    if (LDS_BONES && d_bones != nullptr)
        for (int i = threadIdx.x; i < n_bacc; i += blockDim.x) bacc[i] = 0.f;
    __syncthreads();
    const int64_t count = count_of(n, n_dev, cap);
    // Each thread takes runs of kRun consecutive samples, which nearly always
    // share their nearest joints and often their node list: the bone (node)
    // gradients of a joint (node) slot are summed in registers while its joint
    // (node) stays the same and added to the table when it changes (and at the
    // end), a fraction of the per-sample adds.
    int bkey[KJ], nkey[KN];
    float bsum[KJ][12], nsum[KN][8];
#pragma unroll
    for (int k = 0; k < KN; ++k) {
        nkey[k] = -1;
#pragma unroll
        for (int c = 0; c < 8; ++c) nsum[k][c] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < KJ; ++k) {
        bkey[k] = -1;
#pragma unroll
        for (int e = 0; e < 12; ++e) bsum[k][e] = 0.f;
    }
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kRun; i0 < count;
         i0 += nthreads * kRun)
    for (int r = 0; r < kRun; ++r) {
        const int64_t i = i0 + r;
        if (i >= count) break;
        float3 gz = make_float3(0.f, 0.f, 0.f);
        for (int q = 0; q < n_parts; ++q) {
            const float *g = gz_parts + (size_t)q * part_stride + 3 * i;
            gz = add3(gz, make_float3(g[0], g[1], g[2]));
        }
        if (gz.x == 0.f && gz.y == 0.f && gz.z == 0.f) continue;
        WarpFwd<KJ, KN> f;
        const int fr = frame ? frame[i] : 0;
        const float3 xv = make_float3(x[3 * i], x[3 * i + 1], x[3 * i + 2]);
        warp_one<KJ, KN>(p, J, rig, xv, fr, f);
        const float3 y = f.y;
        const float wr = f.c[0], wd = f.c[4];
        const float3 vr = make_float3(f.c[1], f.c[2], f.c[3]);
        const float3 vd = make_float3(f.c[5], f.c[6], f.c[7]);
        // d z / d c (rotation + translation terms) and d z / d y = R(c_r)
        const float3 vxy = cross3(vr, y);
        float gc[8];
        const float gw_rot = 2.f * dot3(gz, vxy);
        const float3 gv_rot = add3(mul3(2.f * wr, cross3(y, gz)),
                                   mul3(2.f, sub3(add3(mul3(dot3(gz, vr), y), mul3(dot3(vr, y), gz)),
                                                  mul3(2.f * dot3(gz, y), vr))));
        gc[0] = gw_rot + 2.f * dot3(gz, vd);
        const float3 gvr = add3(gv_rot, mul3(2.f, add3(mul3(-wd, gz), cross3(vd, gz))));
        gc[1] = gvr.x;
        gc[2] = gvr.y;
        gc[3] = gvr.z;
        gc[4] = -2.f * dot3(gz, vr);
        const float3 gvd = mul3(2.f, add3(mul3(wr, gz), cross3(gz, vr)));
        gc[5] = gvd.x;
        gc[6] = gvd.y;
        gc[7] = gvd.z;
        // R(c_r)^T gz = rotation by the conjugate
        float3 gy = qrot(wr, make_float3(-vr.x, -vr.y, -vr.z), gz);
        // normalisation c = b / |b_r|
        float dotc = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) dotc += f.c[c] * gc[c];
        const float inr = 1.f / f.nr;
        float gb[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) gb[c] = gc[c] * inr;
#pragma unroll
        for (int c = 0; c < 4; ++c) gb[c] -= f.c[c] * dotc * inr;
        const float cs[8] = {1.f, -1.f, -1.f, -1.f, 1.f, -1.f, -1.f, -1.f};
        const float *DQ = rig.node_dq + (size_t)fr * p.n_nodes * 8;
        const float *G = rig.node_pos + (size_t)fr * p.n_nodes * 3;
#pragma unroll
        for (int k = 0; k < KN; ++k) {
            if (k >= p.k_nodes) continue;
            const int id = f.nid[k];
            const float sw = f.s[k] * f.w[k];
            const float *q = DQ + 8 * id;
            float gwk = 0.f;
            const int key = fr * p.n_nodes + id;
            if (nkey[k] != key) {
                if (nkey[k] >= 0) NVR_FLUSH_NODE(k);
                nkey[k] = key;
#pragma unroll
                for (int c = 0; c < 8; ++c) nsum[k][c] = 0.f;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                nsum[k][c] += sw * cs[c] * gb[c];
                gwk += cs[c] * q[c] * gb[c];
            }
            // weight w_k depends on y: dw/dy = w (-2 (y - g) / r^2)
            const float3 g = make_float3(G[3 * id], G[3 * id + 1], G[3 * id + 2]);
            gy = add3(gy, mul3(f.s[k] * gwk * f.w[k] * (-2.f * p.inv_r2), sub3(y, g)));
        }
        if (d_bones != nullptr) {
            const float gys[3] = {gy.x, gy.y, gy.z};
            const float xh[4] = {xv.x, xv.y, xv.z, 1.f};
#pragma unroll
            for (int k = 0; k < KJ; ++k) {
                if (k >= p.k_joints) continue;
                const int key = fr * p.n_joints + f.jsel[k];
                if (bkey[k] != key) {
                    if (bkey[k] >= 0) NVR_FLUSH_BONE(k);
                    bkey[k] = key;
#pragma unroll
                    for (int e = 0; e < 12; ++e) bsum[k][e] = 0.f;
                }
                const float lw = f.lw[k];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb) bsum[k][4 * a + bb] += lw * gys[a] * xh[bb];
            }
        }
        if (dx_live != nullptr) {
            // y = sum_j lw_j M_j [x; 1], lw = softmax_j(-|x - J_j|^2 / (2 sigma^2)):
            // dx = sum_j lw_j (R_j^T gy + (gy . M_j [x; 1]) (a_j - a_bar)),
            // a_j = -(x - J_j) / sigma^2, a_bar = sum_k lw_k a_k
            const float *B0 = rig.bones + (size_t)fr * p.n_joints * 12;
            const float inv_s2 = 2.f * p.inv_two_sigma2;
            float3 abar = make_float3(0.f, 0.f, 0.f);
#pragma unroll
            for (int k = 0; k < KJ; ++k) {
                if (k >= p.k_joints) continue;
                const float *Jk = J + 3 * f.jsel[k];
                const float3 ak = mul3(-inv_s2, sub3(xv, make_float3(Jk[0], Jk[1], Jk[2])));
                abar = add3(abar, mul3(f.lw[k], ak));
            }
            float3 gx = make_float3(0.f, 0.f, 0.f);
#pragma unroll
            for (int k = 0; k < KJ; ++k) {
                if (k >= p.k_joints) continue;
                const float *M = B0 + 12 * f.jsel[k];
                const float *Jk = J + 3 * f.jsel[k];
                const float3 rt = make_float3(M[0] * gy.x + M[4] * gy.y + M[8] * gy.z,
                                              M[1] * gy.x + M[5] * gy.y + M[9] * gy.z,
                                              M[2] * gy.x + M[6] * gy.y + M[10] * gy.z);
                const float3 yk = make_float3(M[0] * xv.x + M[1] * xv.y + M[2] * xv.z + M[3],
                                              M[4] * xv.x + M[5] * xv.y + M[6] * xv.z + M[7],
                                              M[8] * xv.x + M[9] * xv.y + M[10] * xv.z + M[11]);
                const float3 ak = mul3(-inv_s2, sub3(xv, make_float3(Jk[0], Jk[1], Jk[2])));
                gx = add3(gx, mul3(f.lw[k], add3(rt, mul3(dot3(gy, yk), sub3(ak, abar)))));
            }
            dx_live[3 * i] += gx.x;
            dx_live[3 * i + 1] += gx.y;
            dx_live[3 * i + 2] += gx.z;
        }
    }
#pragma unroll
    for (int k = 0; k < KJ; ++k)
        if (bkey[k] >= 0) NVR_FLUSH_BONE(k);
#pragma unroll
    for (int k = 0; k < KN; ++k)
        if (nkey[k] >= 0) NVR_FLUSH_NODE(k);
#undef NVR_FLUSH_BONE
#undef NVR_FLUSH_NODE
    if (LDS_ACC || LDS_BONES) __syncthreads();
    if (LDS_ACC) {
        for (int i = threadIdx.x; i < n_acc; i += blockDim.x) {
            const int c = i % kNodeStride;
            const float v = acc[i];
            if (c < 8 && v != 0.f) unsafeAtomicAdd(d_dq + (size_t)(i / kNodeStride) * 8 + c, v);
        }
    }
    if (LDS_BONES && d_bones != nullptr) {
        for (int i = threadIdx.x; i < n_bacc; i += blockDim.x) {
            const float v = bacc[i];
            if (v != 0.f) unsafeAtomicAdd(d_bones + i, v);
        }
    }
}

nvr_status make_warp_params(const nvr_warp_desc *w, const nvr_warp_rig *rig, WarpParams *p) {
    NVR_REQUIRE(w && rig, NVR_EINVAL, "NULL warp descriptor or rig");
    NVR_REQUIRE(w->n_joints >= 1 && w->n_joints <= kMaxJoints, NVR_EINVAL, "n_joints out of 1..64");
    NVR_REQUIRE(w->k_joints >= 1 && w->k_joints <= kMaxKJ && w->k_joints <= w->n_joints, NVR_EINVAL,
                "k_joints out of range");
    NVR_REQUIRE(w->n_nodes >= 1 && w->n_nodes <= 65536, NVR_EINVAL, "n_nodes out of 1..65536");
    NVR_REQUIRE(w->k_nodes >= 1 && w->k_nodes <= kMaxKN && w->k_nodes <= w->n_nodes, NVR_EINVAL,
                "k_nodes out of range");
    NVR_REQUIRE(w->n_frames >= 1, NVR_EINVAL, "n_frames < 1");
    NVR_REQUIRE(w->sigma_skin > 0.f && w->r_node > 0.f, NVR_EINVAL, "non-positive widths");
    NVR_REQUIRE(w->lut_res >= 1 && w->lut_res <= 1024, NVR_EINVAL, "lut_res out of 1..1024");
    NVR_REQUIRE(rig->joints && rig->bones && rig->node_dq && rig->node_pos && rig->lut, NVR_EINVAL,
                "NULL rig array");
    p->n_joints = w->n_joints;
    p->k_joints = w->k_joints;
    p->n_nodes = w->n_nodes;
    p->k_nodes = w->k_nodes;
    p->n_frames = w->n_frames;
    p->lut_res = w->lut_res;
    p->inv_two_sigma2 = (float)(1.0 / (2.0 * (double)w->sigma_skin * (double)w->sigma_skin));
    p->inv_r2 = (float)(1.0 / ((double)w->r_node * (double)w->r_node));
    for (int a = 0; a < 3; ++a) {
        NVR_REQUIRE(w->lut_max[a] > w->lut_min[a], NVR_EINVAL, "empty look-up box");
        p->lut_lo[a] = w->lut_min[a];
        p->lut_scale[a] = (float)((double)w->lut_res / ((double)w->lut_max[a] - (double)w->lut_min[a]));
    }
    return NVR_OK;
}

nvr_status launch_warp_fwd(const WarpParams &p, const nvr_warp_rig &rig, int64_t n,
                           const int32_t *n_dev, int64_t cap, const float *x, const int32_t *frame,
                           float *xc, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    const unsigned gr = grid_for(cap, kWarpBlock, 2048);
#define NVR_WARP_FWD(KJ, KN)                                                                  \
    warp_fwd_kernel<KJ, KN><<<gr, kWarpBlock, 0, st>>>(p, rig, rig.joints, n, n_dev, cap, x, \
                                                       frame, xc)
    if (p.k_joints <= 4 && p.k_nodes <= 8) NVR_WARP_FWD(4, 8);
    else if (p.k_joints <= 4) NVR_WARP_FWD(4, 16);
    else if (p.k_nodes <= 8) NVR_WARP_FWD(8, 8);
    else NVR_WARP_FWD(8, 16);
#undef NVR_WARP_FWD
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status launch_warp_bwd(const WarpParams &p, const nvr_warp_rig &rig, int64_t n,
                           const int32_t *n_dev, int64_t cap, const float *x, const int32_t *frame,
                           const float *gz, int n_parts, int64_t part_stride, float *d_dq,
                           float *d_bones, float *dx_live, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    const size_t acc_bytes = sizeof(float) * (size_t)p.n_frames * p.n_nodes * kNodeStride;
    const size_t bone_bytes = sizeof(float) * (size_t)p.n_frames * p.n_joints * 12;
    const size_t base = 0;
    const bool lds_bones = bone_bytes <= 16 * 1024;
    const size_t lb = lds_bones ? bone_bytes : 0;
    const bool lds_acc = acc_bytes + lb <= 64 * 1024;
    const unsigned gr = grid_for(cap, kWarpBlock, lds_acc ? 512 : 2048);
    const size_t lds = base + (lds_bones ? lb : 0) + (lds_acc ? acc_bytes : 0);
#define NVR_WARP_BWD(KJ, KN)                                                                      \
    do {                                                                                          \
        if (lds_acc && lds_bones)                                                                 \
            warp_bwd_kernel<KJ, KN, true, true><<<gr, kWarpBlock, lds, st>>>(                     \
                p, rig, rig.joints, n, n_dev, cap, x, frame, gz, n_parts, part_stride, d_dq,      \
                d_bones, dx_live);                                                                \
        else if (lds_acc)                                                                         \
            warp_bwd_kernel<KJ, KN, true, false><<<gr, kWarpBlock, lds, st>>>(                    \
                p, rig, rig.joints, n, n_dev, cap, x, frame, gz, n_parts, part_stride, d_dq,      \
                d_bones, dx_live);                                                                \
        else if (lds_bones)                                                                       \
            warp_bwd_kernel<KJ, KN, false, true><<<gr, kWarpBlock, lds, st>>>(                    \
                p, rig, rig.joints, n, n_dev, cap, x, frame, gz, n_parts, part_stride, d_dq,      \
                d_bones, dx_live);                                                                \
        else                                                                                      \
            warp_bwd_kernel<KJ, KN, false, false><<<gr, kWarpBlock, lds, st>>>(                   \
                p, rig, rig.joints, n, n_dev, cap, x, frame, gz, n_parts, part_stride, d_dq,      \
                d_bones, dx_live);                                                                \
    } while (0)
    if (p.k_joints <= 4 && p.k_nodes <= 8) NVR_WARP_BWD(4, 8);
    else if (p.k_joints <= 4) NVR_WARP_BWD(4, 16);
    else if (p.k_nodes <= 8) NVR_WARP_BWD(8, 8);
    else NVR_WARP_BWD(8, 16);
#undef NVR_WARP_BWD
    NVR_LAUNCHED();
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_warp_fwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t n,
                                   const int32_t *n_dev, const float *x_live, const int32_t *frame,
                                   float *x_can, nvr_stream stream) {
    clear_error();
    WarpParams p;
    NVR_TRY(make_warp_params(w, rig, &p));
    NVR_REQUIRE(n >= 0, NVR_EINVAL, "n < 0");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x_live && x_can, NVR_EINVAL, "NULL array");
    return launch_warp_fwd(p, *rig, n, n_dev, n, x_live, frame, x_can, hs(stream));
}

extern "C" nvr_status nvr_warp_bwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t n,
                                   const int32_t *n_dev, const float *x_live, const int32_t *frame,
                                   const float *dx_can, int32_t n_parts, float *d_node_dq,
                                   float *d_bones, float *dx_live, nvr_stream stream) {
    clear_error();
    WarpParams p;
    NVR_TRY(make_warp_params(w, rig, &p));
    NVR_REQUIRE(n >= 0, NVR_EINVAL, "n < 0");
    NVR_REQUIRE(n_parts >= 1 && n_parts <= 64, NVR_EINVAL, "n_parts out of 1..64");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x_live && dx_can && d_node_dq, NVR_EINVAL, "NULL array");
    return launch_warp_bwd(p, *rig, n, n_dev, n, x_live, frame, dx_can, n_parts, 3 * n, d_node_dq,
                           d_bones, dx_live, hs(stream));
}

#include "launch.hpp"

namespace nvr {

nvr_status run_warp_fwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t cap,
                        const int32_t *n_dev, const float *x, float *xc, hipStream_t st) {
    WarpParams p;
    NVR_TRY(make_warp_params(w, rig, &p));
    return launch_warp_fwd(p, *rig, cap, n_dev, cap, x, nullptr, xc, st);
}

nvr_status run_warp_bwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t cap,
                        const int32_t *n_dev, const float *x, const float *gz, int n_parts,
                        int64_t part_stride, float *d_dq, float *d_bones, hipStream_t st) {
    WarpParams p;
    NVR_TRY(make_warp_params(w, rig, &p));
    return launch_warp_bwd(p, *rig, cap, n_dev, cap, x, nullptr, gz, n_parts, part_stride, d_dq,
                           d_bones, nullptr, st);
}

}  // namespace nvr
