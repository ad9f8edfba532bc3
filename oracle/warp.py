"""Hybrid warp of live samples into the canonical space, FP64 (test infrastructure only).

Paper definitions followed:

* node influence weight w(x_i, v) = exp(-|v - x_i|^2 / r^2), r = 0.1
  (Sec. 4.1, after Eq. 1);
* the forward blend DQB(v) = sum_i w(x_i, v) dq_i and v~ = SE3(DQB(v)) v
  (Sec. 4.1, Eq. 1);
* the inverse warp of a live sample v_l: deformed nodes x_i^t = dq_i^t x_i,
  v_t = SE3(DQB^-1(v_l)) v_l (Sec. 4.2, Eq. 4), the blend using nodes near the
  point, found in O(1) through a voxel look-up table that lists the neighbour
  node ids of every live voxel (Sec. 4.2, "On-the-fly Radiance Fields").

Readings where the paper is silent or leaves a choice:

* Hybrid order.  Canonical -> live is the skeleton motion after the node
  motion (the double-layer representation of Sec. 4.1), so live -> canonical is
  inverse skinning first, then the inverse node blend.  ``bones`` are given
  already inverted: per joint the live->canonical rigid map y = R x + t.
* Skinning weights (SMPL's per-vertex weights are not available): the 4
  joints nearest to the live point (ties: lower joint index), weights
  exp(-(|x-J_j|^2 - d_min^2) / (2 sigma_s^2)) normalised to sum 1,
  sigma_s = 0.1; y = sum_j w_j (R_j x + t_j).
* Node set: the K ids stored for the live voxel that contains the live sample
  (voxel = clamp(floor((x - lo) * res/side), 0, res-1), linear index
  vx + res*(vy + res*vz)); the first id is the node nearest to that voxel.
* DQB^-1: the blend of the conjugated dual quaternions (both parts
  conjugated, which is the inverse rigid motion), b = sum_i s_i w_i conj(dq_i),
  with w_i = exp(-(|y - g_i|^2 - d_min^2)/r^2) over the node set (g_i the
  deformed node positions; the d_min shift is a uniform scale the blend is
  invariant to, and keeps far points from underflowing), s_i = +1 if
  <q_r,i, q_r,first> >= 0 else -1 (antipodal alignment to the first node).
  Normalise c = b / |b_r|; z = R(c_r) y + 2 vec(c_d conj(c_r)) (the dual-
  quaternion skinning translation, valid when c_d is not orthogonal to c_r).
* Gradients: d z / d dq_i through the blend (the deformed node positions are
  separate inputs), and d z / d bones through y, including y's influence on the
  node weights.  The shift d_min carries no gradient (the blend is scale
  invariant).

Three steps decide integers from floating point and are evaluated in IEEE
float32, one rounding per operation, no fused multiply-add, in this order:
the look-up voxel (as the marcher's occupancy voxel), the squared joint
distances ((dx*dx + dy*dy) + dz*dz) that pick the 4 joints, and the sign dot
product (((w*w1 + x*x1) + y*y1) + z*z1).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32
R_ED = 0.1
SIGMA_SKIN = 0.1


# --------------------------------------------------------------------------
# quaternion helpers (w, x, y, z)
# --------------------------------------------------------------------------
def qmul(a, b):
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def qconj(q):
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def qrot(q, v):
    """q (0,v) q* for a unit quaternion q."""
    pv = np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], -1)
    return qmul(qmul(q, pv), qconj(q))[..., 1:]


def dq_apply(dq, p):
    """Rigid motion of a unit dual quaternion applied to points."""
    qr, qd = dq[..., :4], dq[..., 4:]
    return qrot(qr, p) + 2.0 * qmul(qd, qconj(qr))[..., 1:]


# --------------------------------------------------------------------------
# float32 decisions
# --------------------------------------------------------------------------
def lut_voxel(x, lo, hi, res):
    x = np.asarray(x, f32)
    side = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    sc = (res / side).astype(f32)
    u = (x - np.asarray(lo, f32)[None, :]) * sc[None, :]
    v = np.clip(np.floor(u), 0, res - 1).astype(np.int64)
    return v[:, 0] + res * (v[:, 1] + res * v[:, 2])


def nearest_joints(x, joints, k):
    x = np.asarray(x, f32)
    J = np.asarray(joints, f32)
    dx = x[:, None, 0] - J[None, :, 0]
    dy = x[:, None, 1] - J[None, :, 1]
    dz = x[:, None, 2] - J[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    return np.argsort(d2, axis=1, kind="stable")[:, :k]


def sign_to_first(qr_nodes):
    """qr_nodes (n,K,4) float32 -> (n,K) +-1."""
    q = np.asarray(qr_nodes, f32)
    q0 = q[:, :1, :]
    dot = ((q[..., 0] * q0[..., 0] + q[..., 1] * q0[..., 1]) + q[..., 2] * q0[..., 2]) \
        + q[..., 3] * q0[..., 3]
    return np.where(dot >= 0, 1.0, -1.0)


# --------------------------------------------------------------------------
# forward / backward
# --------------------------------------------------------------------------
def _gather(rig, frame, n):
    fr = np.zeros(n, np.int64) if frame is None else np.asarray(frame, np.int64)
    return fr


def warp(x, rig, grid_lo, grid_hi, frame=None, k_joints=4, r=R_ED, sigma_s=SIGMA_SKIN,
         want_cache=False):
    """x (n,3) live samples; rig: dict(joints (24,3), bones (F,24,3,4),
    node_dq (F,M,8), node_pos (F,M,3), knn (F,res^3,K)).  Returns z (n,3)."""
    # joint and voxel choices are float32 decisions on the rounded position;
    # the arithmetic runs in float64 on the position as given
    x32 = np.asarray(x, f32)
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    fr = _gather(rig, frame, n)
    J = np.asarray(rig["joints"], np.float64)
    bones = np.asarray(rig["bones"], np.float64)
    dq_all = np.asarray(rig["node_dq"], np.float64)
    pos_all = np.asarray(rig["node_pos"], np.float64)
    knn = np.asarray(rig["knn"])
    res = round(knn.shape[1] ** (1.0 / 3.0))
    # --- inverse skinning
    jsel = nearest_joints(x32, rig["joints"], k_joints)                # (n,4)
    d2 = ((x[:, None, :] - J[jsel]) ** 2).sum(-1)
    lw = np.exp(-(d2 - d2.min(1, keepdims=True)) / (2.0 * sigma_s ** 2))
    lw = lw / lw.sum(1, keepdims=True)
    M = bones[fr[:, None], jsel]                                       # (n,4,3,4)
    xh = np.concatenate([x, np.ones((n, 1))], 1)
    yj = np.einsum("nkab,nb->nka", M, xh)
    y = np.einsum("nk,nka->na", lw, yj)
    # --- node set from the live voxel
    vox = lut_voxel(x32, grid_lo, grid_hi, res)
    nid = knn[fr, vox].astype(np.int64)                                # (n,K)
    dq = dq_all[fr[:, None], nid]                                      # (n,K,8)
    g = pos_all[fr[:, None], nid]                                      # (n,K,3)
    s = sign_to_first(np.asarray(rig["node_dq"], f32)[fr[:, None], nid][..., :4])
    e2 = ((y[:, None, :] - g) ** 2).sum(-1)
    w = np.exp(-(e2 - e2.min(1, keepdims=True)) / r ** 2)
    conj = dq * np.array([1, -1, -1, -1, 1, -1, -1, -1], float)
    b = np.einsum("nk,nkc->nc", s * w, conj)
    nr = np.linalg.norm(b[:, :4], axis=1)
    c = b / nr[:, None]
    z = dq_apply(c, y)
    if not want_cache:
        return z
    return z, dict(x=x, xh=xh, jsel=jsel, lw=lw, M=M, y=y, nid=nid, dq=dq, g=g, s=s,
                   w=w, conj=conj, b=b, nr=nr, c=c, fr=fr, r=r)


def _grad_c(c, y, gz):
    """Gradient of z = qrot(c_r, y) + 2 vec(c_d conj(c_r)) w.r.t. c (8), y (3)."""
    qr, qd = c[:, :4], c[:, 4:]
    w0, v = qr[:, :1], qr[:, 1:]
    # rotation term: z_rot = y + 2 w (v x y) + 2 v x (v x y)
    vxy = np.cross(v, y)
    # d z_rot / d w0 = 2 (v x y)
    g_w = 2.0 * np.sum(gz * vxy, 1, keepdims=True)
    # d/dv of 2w (v x y): for gz: 2w (y x gz); of 2 v x (v x y): use identity
    # v x (v x y) = v (v.y) - y (v.v)  -> grad wrt v: (v.y) gz + v (gz.y)... expand:
    # d/dv [gz . (v (v.y) - y |v|^2)] = gz.v * y + (v.y) gz - 2 (gz.y) v
    g_v = 2.0 * w0 * np.cross(y, gz) + 2.0 * (np.sum(gz * v, 1, keepdims=True) * y
                                             + np.sum(v * y, 1, keepdims=True) * gz
                                             - 2.0 * np.sum(gz * y, 1, keepdims=True) * v)
    # translation term: t = 2 (w_r v_d - w_d v_r + v_r x v_d)
    wr, vr = qr[:, :1], qr[:, 1:]
    wd, vd = qd[:, :1], qd[:, 1:]
    g_wr_t = 2.0 * np.sum(gz * vd, 1, keepdims=True)
    g_vr_t = 2.0 * (-wd * gz + np.cross(vd, gz))
    g_wd_t = -2.0 * np.sum(gz * vr, 1, keepdims=True)
    g_vd_t = 2.0 * (wr * gz + np.cross(gz, vr))
    gc = np.concatenate([g_w + g_wr_t, g_v + g_vr_t, g_wd_t, g_vd_t], 1)
    # d z / d y = R(c_r): gy = R^T gz = rotation by conj(c_r)
    gy = qrot(qconj(qr), gz)
    return gc, gy


def warp_backward(x, rig, grid_lo, grid_hi, gz, frame=None, k_joints=4, r=R_ED,
                  sigma_s=SIGMA_SKIN, want_dx=False):
    """Gradients of sum(gz . z): returns (d_node_dq (F,M,8), d_bones (F,24,3,4)),
    and with ``want_dx`` also dx (n,3), the gradient with respect to the live
    positions (through the skinning blend, its weights and the node weights;
    the float32 joint / voxel choices are locally constant)."""
    z, C = warp(x, rig, grid_lo, grid_hi, frame, k_joints, r, sigma_s, want_cache=True)
    gz = np.asarray(gz, np.float64)
    gc, gy = _grad_c(C["c"], C["y"], gz)
    nr = C["nr"][:, None]
    c = C["c"]
    # c = b / |b_r|
    dot = np.sum(c * gc, 1, keepdims=True)           # c_r.g_cr + c_d.g_cd
    gb = gc / nr
    gb[:, :4] -= c[:, :4] * dot / nr
    conj_sign = np.array([1, -1, -1, -1, 1, -1, -1, -1], float)
    sw = C["s"] * C["w"]
    gdq = sw[:, :, None] * (gb[:, None, :] * conj_sign)             # (n,K,8)
    d_dq = np.zeros_like(np.asarray(rig["node_dq"], np.float64))
    np.add.at(d_dq, (C["fr"][:, None].repeat(C["nid"].shape[1], 1), C["nid"]), gdq)
    # y -> node weights: dw_i/dy = w_i * (-2 (y - g_i) / r^2)
    gw = C["s"] * np.einsum("nkc,nc->nk", C["conj"], gb)              # dL/dw_i
    gy = gy + np.einsum("nk,nka->na", gw * C["w"], -2.0 * (C["y"][:, None, :] - C["g"]) / r ** 2)
    # y = sum_j lw_j (M_j xh)
    gM = C["lw"][:, :, None, None] * gy[:, None, :, None] * C["xh"][:, None, None, :]
    d_bones = np.zeros_like(np.asarray(rig["bones"], np.float64))
    np.add.at(d_bones, (C["fr"][:, None].repeat(C["jsel"].shape[1], 1), C["jsel"]), gM)
    if not want_dx:
        return d_dq, d_bones
    # y = sum_j lw_j M_j xh with lw = softmax_j(-|x - J_j|^2 / (2 sigma^2)):
    # dy/dx = sum_j lw_j R_j + sum_j (M_j xh) (a_j - a_bar)^T lw_j,
    # a_j = -(x - J_j) / sigma^2, a_bar = sum_k lw_k a_k
    Jsel = np.asarray(rig["joints"], np.float64)[C["jsel"]]           # (n,4,3)
    a = -(C["x"][:, None, :] - Jsel) / sigma_s ** 2
    a_bar = np.einsum("nk,nka->na", C["lw"], a)
    R = C["M"][..., :3]                                                # (n,4,3,3)
    yj = np.einsum("nkab,nb->nka", C["M"], C["xh"])
    gx = np.einsum("nk,nkab,na->nb", C["lw"], R, gy)
    gx += np.einsum("nk,nk,nka->na", C["lw"], np.einsum("nka,na->nk", yj, gy),
                    a - a_bar[:, None, :])
    return d_dq, d_bones, gx
