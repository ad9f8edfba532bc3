"""Volume-rendering compositing along each ray, FP64 (test infrastructure only).

The paper renders its density fields by NeRF volume rendering (Sec. 1 and the
overview; the back-end also renders depth maps, Sec. 4.3) without writing the
formula down.  The reading taken is NeRF's quadrature, for the samples of one
ray in order of t:

    tau_i = sigma_i * delta_i,  T_i = exp(-sum_{j<i} tau_j),
    alpha_i = 1 - exp(-tau_i),  w_i = T_i * alpha_i,
    C = sum_i w_i c_i,  D = sum_i w_i t_i (un-normalised),  T_N = exp(-sum_i tau_i)

with a black background and D = 0 for an empty ray.  A forward-only render may
drop every sample whose T_i falls below a threshold (early termination).

Backward (closed form), with u_i = c_i . gC + t_i * gD:

    dL/dc_i     = w_i * gC
    dL/dsigma_i = delta_i * ( T_{i+1} * u_i - sum_{k>i} w_k u_k )

where the suffix sum equals (C - C_{<=i}) . gC + (D - D_{<=i}) * gD.

Samples are given packed ray-major: ray r owns samples off[r] .. off[r+1]-1.
A merged ray (two fields sharing it) is composited over the union of both
sample lists sorted by t, human samples first on ties; each keeps its own delta.
"""
from __future__ import annotations

import numpy as np


def forward(off, sigma, rgb, t, dt, t_stop: float = 0.0):
    """Returns C (R,3), D (R,), TN (R,) and per-sample w (n,) in FP64.

    ``t_stop`` > 0 drops every sample with T_i < t_stop (render only)."""
    off = np.asarray(off, np.int64)
    sigma = np.asarray(sigma, np.float64)
    rgb = np.asarray(rgb, np.float64)
    t = np.asarray(t, np.float64)
    dt = np.asarray(dt, np.float64)
    R = off.size - 1
    C = np.zeros((R, 3))
    D = np.zeros(R)
    TN = np.ones(R)
    w = np.zeros(sigma.size)
    for r in range(R):
        a, b = off[r], off[r + 1]
        if b == a:
            continue
        tau = sigma[a:b] * dt[a:b]
        csum = np.concatenate([[0.0], np.cumsum(tau)])
        Ti = np.exp(-csum[:-1])
        wi = Ti * (1.0 - np.exp(-tau))
        if t_stop > 0.0:
            wi = np.where(Ti >= t_stop, wi, 0.0)
        w[a:b] = wi
        C[r] = wi @ rgb[a:b]
        D[r] = wi @ t[a:b]
        TN[r] = np.exp(-csum[-1])
    return C, D, TN, w


def backward(off, sigma, rgb, t, dt, dC, dD):
    """Closed-form gradients (dsigma (n,), drgb (n,3)) of a scalar loss whose
    gradient with respect to C, D is dC (R,3), dD (R,)."""
    off = np.asarray(off, np.int64)
    sigma = np.asarray(sigma, np.float64)
    rgb = np.asarray(rgb, np.float64)
    t = np.asarray(t, np.float64)
    dt = np.asarray(dt, np.float64)
    dC = np.asarray(dC, np.float64)
    dD = np.asarray(dD, np.float64)
    R = off.size - 1
    dsig = np.zeros(sigma.size)
    drgb = np.zeros((sigma.size, 3))
    for r in range(R):
        a, b = off[r], off[r + 1]
        if b == a:
            continue
        tau = sigma[a:b] * dt[a:b]
        csum = np.concatenate([[0.0], np.cumsum(tau)])
        Ti = np.exp(-csum[:-1])
        Tn = np.exp(-csum[1:])                      # T_{i+1}
        wi = Ti * (1.0 - np.exp(-tau))
        u = rgb[a:b] @ dC[r] + t[a:b] * dD[r]
        wu = wi * u
        suffix = np.concatenate([np.cumsum(wu[::-1])[::-1][1:], [0.0]])  # sum_{k>i}
        dsig[a:b] = dt[a:b] * (Tn * u - suffix)
        drgb[a:b] = wi[:, None] * dC[r][None, :]
    return dsig, drgb


def product_form(off, sigma, dt):
    """T_i as the product of (1 - alpha_j), j < i: an independent restatement
    used only to pin the exp-of-sum form."""
    off = np.asarray(off, np.int64)
    sigma = np.asarray(sigma, np.float64)
    dt = np.asarray(dt, np.float64)
    out = np.ones(sigma.size)
    for r in range(off.size - 1):
        acc = 1.0
        for i in range(off[r], off[r + 1]):
            out[i] = acc
            acc *= 1.0 - (1.0 - np.exp(-sigma[i] * dt[i]))
    return out


def merge_two(off_a, t_a, off_b, t_b):
    """Merge two ray-major sample lists ray by ray on t (ties: list a first).

    Returns (off (R+1,), src (n,) 0/1, idx (n,)): merged sample k comes from
    list ``src[k]`` at index ``idx[k]``.  Both lists must be sorted in t per
    ray (the marcher emits them so)."""
    off_a = np.asarray(off_a, np.int64)
    off_b = np.asarray(off_b, np.int64)
    R = off_a.size - 1
    src, idx, off = [], [], [0]
    for r in range(R):
        i, j = off_a[r], off_b[r]
        ie, je = off_a[r + 1], off_b[r + 1]
        while i < ie or j < je:
            if j >= je or (i < ie and t_a[i] <= t_b[j]):
                src.append(0)
                idx.append(i)
                i += 1
            else:
                src.append(1)
                idx.append(j)
                j += 1
        off.append(len(src))
    return np.asarray(off, np.int64), np.asarray(src, np.int64), np.asarray(idx, np.int64)
