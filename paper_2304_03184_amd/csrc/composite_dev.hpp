// Per-ray compositing walks (device), shared by the compositing kernels.
#pragma once
#include "common.hpp"

namespace nvr {

struct RayAcc {
    float c[3];
    float d;
    float tau;   // sum of tau over the composited samples
};

// Iterates the samples of ray r in t order over one or two lists.
struct MergedWalk {
    const nvr_samples &a, &b;
    bool has_b;
    int64_t i, ie, j, je;
    __device__ MergedWalk(const nvr_samples &a_, const nvr_samples &b_, bool hb, int64_t r)
        : a(a_), b(b_), has_b(hb) {
        i = a.off[r];
        ie = a.off[r + 1];
        if (has_b) {
            j = b.off[r];
            je = b.off[r + 1];
        } else {
            j = je = 0;
        }
    }
    // returns false when exhausted; sets which (0: a, 1: b) and idx
    __device__ __forceinline__ bool next(int &which, int64_t &idx) {
        if (i < ie && (j >= je || a.t[i] <= b.t[j])) {
            which = 0;
            idx = i++;
            return true;
        }
        if (j < je) {
            which = 1;
            idx = j++;
            return true;
        }
        return false;
    }
};

__device__ __forceinline__ RayAcc ray_forward(const nvr_samples &a, const nvr_samples &b, bool has_b,
                                              int64_t r, float t_stop) {
    RayAcc acc{{0.f, 0.f, 0.f}, 0.f, 0.f};
    MergedWalk w(a, b, has_b, r);
    int which;
    int64_t k;
    while (w.next(which, k)) {
        const nvr_samples &L = which ? b : a;
        const float tau = L.sigma[k] * L.dt[k];
        const float T = expf(-acc.tau);
        if (t_stop > 0.f && T < t_stop) break;
        const float wgt = T * (1.f - expf(-tau));
        acc.c[0] += wgt * L.rgb[3 * k];
        acc.c[1] += wgt * L.rgb[3 * k + 1];
        acc.c[2] += wgt * L.rgb[3 * k + 2];
        acc.d += wgt * L.t[k];
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
    int which;
    int64_t k;
    float csum = 0.f, pc0 = 0.f, pc1 = 0.f, pc2 = 0.f, pd = 0.f;
    while (w.next(which, k)) {
        const nvr_samples &L = which ? b : a;
        const float tau = L.sigma[k] * L.dt[k];
        const float T = expf(-csum);
        const float Tn = expf(-(csum + tau));
        const float wgt = T * (1.f - expf(-tau));
        const float c0 = L.rgb[3 * k], c1 = L.rgb[3 * k + 1], c2 = L.rgb[3 * k + 2];
        const float tk = L.t[k];
        pc0 += wgt * c0;
        pc1 += wgt * c1;
        pc2 += wgt * c2;
        pd += wgt * tk;
        const float u = c0 * gc[0] + c1 * gc[1] + c2 * gc[2] + tk * gd;
        const float suffix = (C[0] - pc0) * gc[0] + (C[1] - pc1) * gc[1] + (C[2] - pc2) * gc[2] +
                             (D - pd) * gd;
        float *ds = which ? dsb : dsa;
        float *dr = which ? drb : dra;
        ds[k] = L.dt[k] * (Tn * u - suffix);
        dr[3 * k] = wgt * gc[0];
        dr[3 * k + 1] = wgt * gc[1];
        dr[3 * k + 2] = wgt * gc[2];
        csum += tau;
    }
}

nvr_status launch_fill_zero(float *p, int64_t n, hipStream_t st);
nvr_status launch_composite_loss(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                 const float *C_t, const float *D_t, const float *mask,
                                 float lambda_d, const nvr_train_state *state, float *loss,
                                 float *C_out, float *D_out, float *dsa, float *dra, float *dsb,
                                 float *drb, hipStream_t st);
nvr_status launch_composite_fwd(int64_t n_rays, const nvr_samples &a, const nvr_samples *b,
                                float t_stop, float *C, float *D, float *TN, hipStream_t st);

}  // namespace nvr
