"""Density and colour networks of one field, FP64 (test infrastructure only).

Each field feeds its encoded features to a geometry network E_g and a colour
network E_c (Sec. 4.2, "Separated instant neural representation"; the human
field the same after the warp).  Widths and activations are not stated in the
paper; the reading taken (Instant-NGP's published design):

* bias-free linear layers, ReLU on hidden layers;
* density network enc -> hidden... -> 16 outputs o; the density is
  sigma = exp(o_0), with o_0 clamped to [-15, 15] (derivative 0 outside);
* colour network input [o (all 16), SH(d)] -> hidden... -> 3, then sigmoid.

Parameters are one flat vector: every layer's W (out x in, row-major), density
layers first, then colour layers, in order.
"""
from __future__ import annotations

import numpy as np

SIGMA_CLAMP = 15.0


def split_params(params, shapes):
    out, p = [], 0
    params = np.asarray(params, np.float64)
    for o, i in shapes:
        out.append(params[p:p + o * i].reshape(o, i))
        p += o * i
    if p != params.size:
        raise ValueError("parameter vector does not match the layer shapes")
    return out


def _n_density_layers(fcfg):
    return len(fcfg.density_hidden) + 1


def forward(fcfg, params, feat, sh):
    """feat (n, L*F), sh (n, n_sh) -> sigma (n,), rgb (n,3), cache."""
    Ws = split_params(params, fcfg.layer_shapes())
    nd = _n_density_layers(fcfg)
    acts = [np.asarray(feat, np.float64)]
    h = acts[0]
    for k in range(nd):
        h = h @ Ws[k].T
        if k < nd - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    o = h
    o0 = o[:, 0]
    sigma = np.exp(np.clip(o0, -SIGMA_CLAMP, SIGMA_CLAMP))
    g = np.concatenate([o, np.asarray(sh, np.float64)], axis=1)
    acts.append(g)
    for k in range(nd, len(Ws)):
        g = g @ Ws[k].T
        if k < len(Ws) - 1:
            g = np.maximum(g, 0.0)
        acts.append(g)
    rgb = 1.0 / (1.0 + np.exp(-g))
    return sigma, rgb, dict(acts=acts, Ws=Ws, sigma=sigma, rgb=rgb, o0=o0)


def backward(fcfg, cache, dsigma, drgb):
    """Returns (dparams flat, dfeat (n, L*F))."""
    Ws, acts = cache["Ws"], cache["acts"]
    nd = _n_density_layers(fcfg)
    nl = len(Ws)
    dW = [None] * nl
    g = np.asarray(drgb, np.float64) * cache["rgb"] * (1.0 - cache["rgb"])
    # colour layers: acts[nd+1] is the colour input, acts[nd+1+j] the outputs
    for k in range(nl - 1, nd - 1, -1):
        a_in = acts[k + 1]
        dW[k] = g.T @ a_in
        g = g @ Ws[k]
        if k > nd:                       # input of this layer came out of a ReLU
            g = g * (a_in > 0.0)
    do = g[:, :fcfg.density_out].copy()
    inside = np.abs(cache["o0"]) < SIGMA_CLAMP
    do[:, 0] += np.asarray(dsigma, np.float64) * cache["sigma"] * inside
    g = do
    for k in range(nd - 1, -1, -1):
        a_in = acts[k]
        dW[k] = g.T @ a_in
        g = g @ Ws[k]
        if k > 0:
            g = g * (a_in > 0.0)
    return np.concatenate([w.reshape(-1) for w in dW]), g
