// Per-ray compositing walks (device), shared by the compositing kernels.
#pragma once
#include "common.hpp"

namespace nvr {

struct RayAcc {
    float c[3];
    float d;
    float tau;   // sum of tau over the composited samples
};

// One composited sample of a ray.
struct Sample {
    float sigma, c0, c1, c2, t, dt;
    int which;      // 0: first list, 1: second list
    int64_t k;      // index in its list
};

// Iterates the samples of ray r in t order over one or two lists (ties go to
// the first list).  Each branch loads its own list's values: selecting a list
// by reference (`which ? b : a`) and loading through the selected pointers
// was compiled with the pointer copy executed for the wrong lanes (a lane
// taking from the second list while the first was not exhausted read the
// first list), so the walk never selects pointers at run time.
struct MergedWalk {
    nvr_samples a, b;
    int64_t i, ie, j, je;
    __device__ __forceinline__ MergedWalk(const nvr_samples &a_, const nvr_samples &b_, bool has_b,
                                          int64_t r)
        : a(a_), b(b_) {
        i = a.off[r];
        ie = a.off[r + 1];
        if (has_b) {
            j = b.off[r];
            je = b.off[r + 1];
        } else {
            j = je = 0;
        }
    }
    __device__ __forceinline__ bool next(Sample &s) {
        const bool take_a = i < ie && (j >= je || a.t[i] <= b.t[j]);
        if (take_a) {
            s.which = 0;
            s.k = i++;
            s.sigma = a.sigma[s.k];
            s.c0 = a.rgb[3 * s.k];
            s.c1 = a.rgb[3 * s.k + 1];
            s.c2 = a.rgb[3 * s.k + 2];
            s.t = a.t[s.k];
            s.dt = a.dt[s.k];
            return true;
        }
        if (j < je) {
            s.which = 1;
            s.k = j++;
            s.sigma = b.sigma[s.k];
            s.c0 = b.rgb[3 * s.k];
            s.c1 = b.rgb[3 * s.k + 1];
            s.c2 = b.rgb[3 * s.k + 2];
            s.t = b.t[s.k];
            s.dt = b.dt[s.k];
            return true;
        }
        return false;
    }
};

__device__ __forceinline__ RayAcc ray_forward(const nvr_samples &a, const nvr_samples &b, bool has_b,
                                              int64_t r, float t_stop) {
    RayAcc acc{{0.f, 0.f, 0.f}, 0.f, 0.f};
    MergedWalk w(a, b, has_b, r);
    Sample s;
    while (w.next(s)) {
        const float tau = s.sigma * s.dt;
        const float T = expf(-acc.tau);
        if (t_stop > 0.f && T < t_stop) break;
        const float wgt = T * (1.f - expf(-tau));
        acc.c[0] += wgt * s.c0;
        acc.c[1] += wgt * s.c1;
        acc.c[2] += wgt * s.c2;
        acc.d += wgt * s.t;
        acc.tau += tau;
    }
    return acc;
}

// dsigma_i = dt_i (T_{i+1} u_i - sum_{k>i} w_k u_k), drgb_i = w_i gC, where the
// suffix sum is (C - C_{<=i}).gC + (D - D_{<=i}) gD.
__device__ __forceinline__ void ray_backward(const nvr_samples &a, const nvr_samples &b, bool has_b,
                                             int64_t r, const float *C, float D, const float *gc,
                                             float gd, float *dsa, float *dra, float *dsb,
                                             float *drb) {
    MergedWalk w(a, b, has_b, r);
    Sample s;
    float csum = 0.f, pc0 = 0.f, pc1 = 0.f, pc2 = 0.f, pd = 0.f;
    while (w.next(s)) {
        const float tau = s.sigma * s.dt;
        const float T = expf(-csum);
        const float Tn = expf(-(csum + tau));
        const float wgt = T * (1.f - expf(-tau));
        pc0 += wgt * s.c0;
        pc1 += wgt * s.c1;
        pc2 += wgt * s.c2;
        pd += wgt * s.t;
        const float u = s.c0 * gc[0] + s.c1 * gc[1] + s.c2 * gc[2] + s.t * gd;
        const float suffix = (C[0] - pc0) * gc[0] + (C[1] - pc1) * gc[1] + (C[2] - pc2) * gc[2] +
                             (D - pd) * gd;
        const float ds = s.dt * (Tn * u - suffix);
        if (s.which == 0) {
            dsa[s.k] = ds;
            dra[3 * s.k] = wgt * gc[0];
            dra[3 * s.k + 1] = wgt * gc[1];
            dra[3 * s.k + 2] = wgt * gc[2];
        } else {
            dsb[s.k] = ds;
            drb[3 * s.k] = wgt * gc[0];
            drb[3 * s.k + 1] = wgt * gc[1];
            drb[3 * s.k + 2] = wgt * gc[2];
        }
        csum += tau;
    }
}

// ---------------------------------------------------------------- group scans
// A ray is composited by a group of kGroup consecutive lanes of a wavefront;
// its samples are taken kGroup at a time, transmittance comes from inclusive
// prefix scans of tau over the group's lanes (shuffles inside the group), with
// a carry across segments.
constexpr int kGroup = 16;

__device__ __forceinline__ float group_scan_incl(float v, int gl) {
#pragma unroll
    for (int d = 1; d < kGroup; d <<= 1) {
        const float u = __shfl_up(v, d, kGroup);
        if (gl >= d) v += u;
    }
    return v;
}
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int d = kGroup / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kGroup);
    return v;
}
// value of lane `src` of the group
__device__ __forceinline__ float group_bcast(float v, int src) { return __shfl(v, src, kGroup); }

// Forward over one list's samples [s0, s1) of a ray; totals on every lane.
// Samples whose transmittance is below t_stop (t_stop > 0) are not
// composited; transmittance is non-increasing, so they form a suffix and the
// walk stops at the first segment that reaches one.
__device__ __forceinline__ RayAcc group_forward(const nvr_samples &L, int64_t s0, int64_t s1, int gl,
                                                float t_stop) {
    float carry = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f, dd = 0.f;
    for (int64_t base = s0; base < s1; base += kGroup) {
        const int64_t s = base + gl;
        const bool v = s < s1;
        float tau = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f, tt = 0.f;
        if (v) {
            tau = L.sigma[s] * L.dt[s];
            r0 = L.rgb[3 * s];
            r1 = L.rgb[3 * s + 1];
            r2 = L.rgb[3 * s + 2];
            tt = L.t[s];
        }
        const float incl = group_scan_incl(tau, gl);
        const float T = expf(-(carry + (incl - tau)));
        const bool keep = v && !(t_stop > 0.f && T < t_stop);
        const float w = keep ? T * (1.f - expf(-tau)) : 0.f;
        c0 += w * r0;
        c1 += w * r1;
        c2 += w * r2;
        dd += w * tt;
        carry += group_sum(keep ? tau : 0.f);
        if (group_sum((v && !keep) ? 1.f : 0.f) > 0.f) break;   // the same on the whole group
    }
    RayAcc acc;
    acc.c[0] = group_sum(c0);
    acc.c[1] = group_sum(c1);
    acc.c[2] = group_sum(c2);
    acc.d = group_sum(dd);
    acc.tau = carry;
    return acc;
}

// Backward over one list's samples of a ray given its totals C, D and the
// loss gradients gc, gd (every lane of the group holds them):
// dsigma_i = dt_i (T_{i+1} u_i - sum_{k>i} w_k u_k), u = c.gc + t gd, where the
// suffix sum is (C.gc + D gd) minus the inclusive prefix of w u.
__device__ __forceinline__ void group_backward(const nvr_samples &L, int64_t s0, int64_t s1, int gl,
                                               const float *C, float D, const float *gc, float gd,
                                               float *ds_out, float *dr_out) {
    const float total = C[0] * gc[0] + C[1] * gc[1] + C[2] * gc[2] + D * gd;
    float carry_tau = 0.f, carry_wu = 0.f;
    for (int64_t base = s0; base < s1; base += kGroup) {
        const int64_t s = base + gl;
        const bool v = s < s1;
        float tau = 0.f, dt = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f, tt = 0.f;
        if (v) {
            dt = L.dt[s];
            tau = L.sigma[s] * dt;
            r0 = L.rgb[3 * s];
            r1 = L.rgb[3 * s + 1];
            r2 = L.rgb[3 * s + 2];
            tt = L.t[s];
        }
        const float incl = group_scan_incl(tau, gl);
        const float T = expf(-(carry_tau + (incl - tau)));
        const float Tn = expf(-(carry_tau + incl));
        const float w = v ? T * (1.f - expf(-tau)) : 0.f;
        const float u = r0 * gc[0] + r1 * gc[1] + r2 * gc[2] + tt * gd;
        const float wu_incl = group_scan_incl(w * u, gl);
        const float suffix = total - (carry_wu + wu_incl);
        if (v) {
            ds_out[s] = dt * (Tn * u - suffix);
            dr_out[3 * s] = w * gc[0];
            dr_out[3 * s + 1] = w * gc[1];
            dr_out[3 * s + 2] = w * gc[2];
        }
        carry_tau += group_bcast(incl, kGroup - 1);
        carry_wu += group_bcast(wu_incl, kGroup - 1);
    }
}

nvr_status launch_fill_zero(float *p, int64_t n, hipStream_t st);
nvr_status launch_composite_loss(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                 const float *C_t, const float *D_t, const float *mask,
                                 float lambda_d, const nvr_train_state *state, float *loss,
                                 float *C_out, float *D_out, float *dsa, float *dra, float *dsb,
                                 float *drb, hipStream_t st, int blocks = 0,
                                 float *partials = nullptr);
// most workgroups launch_composite_loss uses; partials (nullable) holds one
// float per workgroup, and makes the loss a fixed-order sum of them
constexpr int kMaxLossBlocks = 65536;
nvr_status launch_composite_fwd(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                float t_stop, float *C, float *D, float *TN, hipStream_t st);

}  // namespace nvr
