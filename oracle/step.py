"""Whole training step and forward-only render, FP64 (test infrastructure only).

Per training iteration the back-end samples rays, warps human samples into the
canonical space, encodes, evaluates the networks, volume-renders and back-
propagates the colour / depth loss (Sec. 4.2 and 4.3).  This module chains the
other oracle modules in that order for one or two fields:

    march (per field, over the rays the field covers)
    -> [warp]  (human field)
    -> [deformation network: x_c = x_t + MLP([enc_d(x_t), theta])]  (human field, if given)
    -> encode -> SH(view direction) -> networks
    -> composite (two fields on a shared ray: merged by t)
    -> loss -> composite backward -> network backward -> encode backward
    -> [deformation-network backward] -> [warp backward]
    -> Adam (tables skip zero-gradient entries; the deformation network's table
       and parameters are trained with its field).

Motion priors (and the pose theta) are inputs (they come from the tracker,
Sec. 4.1): their gradients are returned but not applied.
"""
from __future__ import annotations

from dataclasses import dataclass, field as dfield

import numpy as np

from . import composite, deform, grid, march, network, optim, sh, warp


@dataclass
class DeformState:
    """The deformation network of a warped field (Sec. 4.2, hybrid deformation)."""
    lay: object                       # grid.Layout of its own 32-wide encoding
    theta: np.ndarray                 # (72,) pose
    table: np.ndarray                 # (n_entries, 2) float64 master
    params: np.ndarray                # flat float64 master
    m_t: np.ndarray = None
    v_t: np.ndarray = None
    m_p: np.ndarray = None
    v_p: np.ndarray = None

    def __post_init__(self):
        self.theta = np.asarray(self.theta, np.float64).copy()
        self.table = np.asarray(self.table, np.float64).copy()
        self.params = np.asarray(self.params, np.float64).copy()
        self.m_t = np.zeros_like(self.table)
        self.v_t = np.zeros_like(self.table)
        self.m_p = np.zeros_like(self.params)
        self.v_p = np.zeros_like(self.params)


@dataclass
class FieldState:
    fcfg: object
    table: np.ndarray                 # (n_entries, F) float64 master
    params: np.ndarray                # flat float64 master
    occ_words: np.ndarray = None
    rig: dict = None                  # warp inputs for a human field
    deform: DeformState = None        # its deformation network (needs rig)
    m_t: np.ndarray = None
    v_t: np.ndarray = None
    m_p: np.ndarray = None
    v_p: np.ndarray = None
    lay: object = None

    def __post_init__(self):
        self.table = np.asarray(self.table, np.float64).copy()
        self.params = np.asarray(self.params, np.float64).copy()
        self.lay = grid.Layout.from_field(self.fcfg)
        self.m_t = np.zeros_like(self.table)
        self.v_t = np.zeros_like(self.table)
        self.m_p = np.zeros_like(self.params)
        self.v_p = np.zeros_like(self.params)


@dataclass
class StepState:
    fields: list
    step: int = 0
    loss_scale: float = 1.0
    history: list = dfield(default_factory=list)


def march_field(work, st: FieldState, o, d, ray_lo=0, ray_hi=None):
    f = st.fcfg
    R = o.shape[0]
    ray_hi = R if ray_hi is None else ray_hi
    delta = march.step_size(work, f)
    m = march.march(o[ray_lo:ray_hi], d[ray_lo:ray_hi], f.aabb_min, f.aabb_max,
                    work.near, work.far, delta, work.max_steps,
                    st.occ_words if f.occ_res > 0 else None, f.occ_res)
    count = np.zeros(R, np.int64)
    count[ray_lo:ray_hi] = m["count"]
    off = np.concatenate([[0], np.cumsum(count)]).astype(np.int64)
    m["off"] = off
    m["ray"] = m["ray"] + ray_lo
    m["count"] = count
    return m


def field_forward(st: FieldState, x, dirs, grid_box=None, frame=None):
    """``xc`` in the cache is where the field's encoding is read: the warped
    point, moved by the deformation network when the field has one."""
    f = st.fcfg
    xw = x if st.rig is None else warp.warp(x, st.rig, grid_box[0], grid_box[1], frame)
    xc, dcache = xw, None
    if st.deform is not None:
        D = st.deform
        xc, dcache = deform.forward(D.params, xw, D.theta, D.table, D.lay)
    feat = grid.encode(xc, st.table, st.lay)
    shv = sh.sh_encode(dirs, f.sh_degree)
    sigma, rgb, cache = network.forward(f, st.params, feat, shv)
    return sigma, rgb, dict(xc=xc, xw=xw, deform=dcache, net=cache, x=x, frame=frame)


def field_backward(st: FieldState, cache, dsigma, drgb, grid_box=None):
    dparams, dfeat = network.backward(st.fcfg, cache["net"], dsigma, drgb)
    want_dx = st.rig is not None
    dtable, dxc = grid.encode_backward(cache["xc"], st.table, dfeat, st.lay, want_dx)
    out = dict(table=dtable, params=dparams)
    if want_dx:
        dxw = dxc
        if st.deform is not None:
            dp, dt, dxw, dth = deform.backward(cache["deform"], dxc)
            out.update(deform_params=dp, deform_table=dt, theta=dth)
        d_dq, d_bones = warp.warp_backward(cache["x"], st.rig, grid_box[0], grid_box[1],
                                           dxw, cache["frame"])
        out.update(node_dq=d_dq, bones=d_bones, dxc=dxc, dxw=dxw)
    return out


def forward_all(work, state: StepState, o, d, ranges, grid_box=None, t_stop=0.0):
    """Forward of every field over its ray range, then (merged) compositing.
    ``ranges`` lists (ray_lo, ray_hi) per field."""
    per = []
    for st, (lo, hi) in zip(state.fields, ranges):
        m = march_field(work, st, o, d, lo, hi)
        dirs = d[m["ray"]]
        sigma, rgb, cache = field_forward(st, m["x"], dirs, grid_box)
        per.append(dict(m=m, sigma=sigma, rgb=rgb, cache=cache))
    if len(per) == 1:
        p = per[0]
        off, sig, col = p["m"]["off"], p["sigma"], p["rgb"]
        t, dt = p["m"]["t"], p["m"]["dt"]
        src = np.zeros(sig.size, np.int64)
        idx = np.arange(sig.size)
    else:
        a, b = per
        off, src, idx = composite.merge_two(a["m"]["off"], a["m"]["t"], b["m"]["off"],
                                            b["m"]["t"])
        sig = np.where(src == 0, a["sigma"][np.where(src == 0, idx, 0)],
                       b["sigma"][np.where(src == 1, idx, 0)])
        col = np.where((src == 0)[:, None], a["rgb"][np.where(src == 0, idx, 0)],
                       b["rgb"][np.where(src == 1, idx, 0)])
        t = np.where(src == 0, a["m"]["t"][np.where(src == 0, idx, 0)],
                     b["m"]["t"][np.where(src == 1, idx, 0)])
        dt = np.where(src == 0, a["m"]["dt"][np.where(src == 0, idx, 0)],
                      b["m"]["dt"][np.where(src == 1, idx, 0)])
    C, D, TN, w = composite.forward(off, sig, col, t, dt, t_stop)
    return dict(per=per, off=off, src=src, idx=idx, sigma=sig, rgb=col, t=t, dt=dt,
                C=C, D=D, TN=TN, w=w)


def train_step(work, state: StepState, o, d, C_t, D_t, ranges, grid_box=None,
               adam=None, apply=True, mask=None):
    """One fwd + bwd (+ Adam if ``apply``); ``mask`` is the per-ray M(r) of
    Eq. 8 (None: every ray).  Returns dict(loss, grads per field, C, D, fwd)."""
    adam = adam or optim.Adam()
    fw = forward_all(work, state, o, d, ranges, grid_box)
    L, dC, dD = optim.loss(fw["C"], fw["D"], C_t, D_t, work.lambda_depth, mask)
    dsig, drgb = composite.backward(fw["off"], fw["sigma"], fw["rgb"], fw["t"], fw["dt"],
                                    dC * state.loss_scale, dD * state.loss_scale)
    grads = []
    for fi, (st, p) in enumerate(zip(state.fields, fw["per"])):
        sel = fw["src"] == fi
        n = p["sigma"].size
        ds = np.zeros(n)
        dr = np.zeros((n, 3))
        ds[fw["idx"][sel]] = dsig[sel]
        dr[fw["idx"][sel]] = drgb[sel]
        grads.append(field_backward(st, p["cache"], ds, dr, grid_box))
    trained = ("table", "params", "deform_table", "deform_params")
    flat, where = [], []
    for k, g in enumerate(grads):
        for key in trained:
            if key in g:
                flat.append(g[key])
                where.append((k, key))
    unscaled, finite = optim.unscale_and_check(flat, state.loss_scale)
    for (k, key), u in zip(where, unscaled):
        grads[k][key] = u
    for g in grads:
        for key in ("node_dq", "bones", "dxc", "dxw", "theta"):
            if key in g:
                g[key] = g[key] / state.loss_scale
    if apply:
        if finite:
            state.step += 1
            for st, g in zip(state.fields, grads):
                adam.update(st.table, g["table"], st.m_t, st.v_t, state.step, skip_zero=True)
                adam.update(st.params, g["params"], st.m_p, st.v_p, state.step)
                if st.deform is not None:
                    D = st.deform
                    adam.update(D.table, g["deform_table"], D.m_t, D.v_t, state.step,
                                skip_zero=True)
                    adam.update(D.params, g["deform_params"], D.m_p, D.v_p, state.step)
        else:
            state.loss_scale *= 0.5
    state.history.append(L)
    return dict(loss=L, grads=grads, C=fw["C"], D=fw["D"], fwd=fw, finite=finite)


def render(work, state: StepState, o, d, ranges, grid_box=None, t_stop=1e-4):
    fw = forward_all(work, state, o, d, ranges, grid_box, t_stop)
    return fw["C"], fw["D"]
