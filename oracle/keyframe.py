"""Key-frame selection and the human/object assembly, FP64 (test infrastructure only).

Paper definitions followed (Sec. 4.2, "Online key frame selection"; values
from Sec. 4.3, implementation details):

* Eq. 5: node i of frame t is visible, s_i^t = 1, when its depth z' differs
  from the depth map D^t at its projected pixel by less than eps = 0.01;
* Eq. 6: human frame distance E_h = sum_k beta_pose,k (theta_1,k -
  theta_2,k)^2 + beta_vis sum_i (s_i^1 xor s_i^2) + beta_h (t_1 - t_2)^2, with
  beta_pose 0.1 on torso joints and 0.02 on limb joints, beta_vis = 0.01,
  beta_h = 0.02 (theta: 24 joints x 3 axis-angle components; t: frame index);
* Eq. 7: object frame distance E_o = beta_d |d_1 - d_2|^2 + beta_o (t_1 -
  t_2)^2, beta_d = 1, beta_o = 0.02 (d: the object translation);
* the spatial pool: the first frame enters; a later frame enters when its E to
  every pooled frame exceeds gamma = 2.5; the pool holds at most 100 frames;
* the spatial-temporal pool of the rendering-aware refinement: m = 10 frames of
  the spatial pool closest to the rendering view plus the m latest frames;
* the human and object renderings are combined per pixel by depth.

Readings where the paper is silent or inconsistent:

* the projection is a 3 x 4 matrix P = K [R | t] (world to pixels, camera z
  forward); (u', v', w') = P (x, 1), z' = w' (the camera depth), pixel
  (floor(u'/w'), floor(v'/w')) with pixel centres at half-integers, row-major
  depth maps D[v][u]; a node with w' <= 0 or projecting outside the image is
  not visible.  These decide integers and are evaluated in IEEE float32, one
  rounding per operation, no fused multiply-add, in the order
  ((P_r0 x + P_r1 y) + P_r2 z) + P_r3, then the divisions, then
  |w' - D| < eps;
* torso joints (weight 0.1) are the trunk of the 24-joint skeleton: pelvis,
  the three spine joints, neck, both collars and head (0, 3, 6, 9, 12, 13, 14,
  15); the other 16 joints are limbs (0.02);
* E is a distance (larger = more diverse: frames enter when E > gamma), so the
  "similarity" of the eviction and selection rules is read as small E: when the
  pool is full, an entering frame replaces the pooled frame with the smallest
  E to it (ties: the lower slot), and the m pooled frames with the smallest E
  to the query (ties: the lower slot) are selected; the rendering view is
  represented by a frame record (its pose, visibility and time);
* visibility bits are packed 32 per word, node i at word i >> 5, bit i & 31;
* assembly: a field covers a pixel when its opacity 1 - T_N is at least 1/2,
  its surface depth is D / (1 - T_N); the pixel takes the colour and depth of
  the nearer covering field (ties: the first); with no covering field the
  colours add (both over the black background) and the depth is that of the
  more opaque field's normalised depth, or 0 when both opacities are 0.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32

EPS_VIS = 0.01
BETA_TORSO, BETA_LIMB = 0.1, 0.02
BETA_VIS, BETA_H = 0.01, 0.02
BETA_D, BETA_O = 1.0, 0.02
GAMMA = 2.5
POOL_CAP = 100
M_SELECT = 10
TORSO_JOINTS = (0, 3, 6, 9, 12, 13, 14, 15)


def beta_pose(n_joints=24):
    """Per-component pose weights [3 n_joints] (axis-angle components of joint j
    at 3j..3j+2)."""
    b = np.full(n_joints, BETA_LIMB)
    b[list(TORSO_JOINTS)] = BETA_TORSO
    return np.repeat(b, 3)


def visibility(nodes, P, depth, eps=EPS_VIS):
    """Eq. 5 for nodes [M][3] (world positions) of one frame: bool [M]."""
    x = np.asarray(nodes, f32)
    P = np.asarray(P, f32)
    D = np.asarray(depth, f32)
    h, w = D.shape

    def row(r):
        return ((P[r, 0] * x[:, 0] + P[r, 1] * x[:, 1]) + P[r, 2] * x[:, 2]) + P[r, 3]

    up, vp, wp = row(0), row(1), row(2)
    front = wp > f32(0)
    safe = np.where(front, wp, f32(1))
    u = np.floor(up / safe)
    v = np.floor(vp / safe)
    inside = front & (u >= 0) & (u < w) & (v >= 0) & (v < h)
    ui = np.where(inside, u, 0).astype(np.int64)
    vi = np.where(inside, v, 0).astype(np.int64)
    d = D[vi, ui]
    return inside & (np.abs(wp - d) < f32(eps))


def pack_bits(b):
    """bool [M] -> uint32 [ceil(M / 32)], node i at word i >> 5, bit i & 31."""
    b = np.asarray(b, bool)
    words = np.zeros((len(b) + 31) // 32, np.uint64)
    for i in np.nonzero(b)[0]:
        words[i >> 5] |= np.uint64(1) << np.uint64(i & 31)
    return words.astype(np.uint32)


def xor_count(bits1, bits2):
    """Number of nodes whose visibility differs (sum of s^1 xor s^2)."""
    x = np.bitwise_xor(np.asarray(bits1, np.uint32), np.asarray(bits2, np.uint32))
    return int(sum(bin(int(v)).count("1") for v in x))


def human_distance(theta1, theta2, bits1, bits2, t1, t2, beta=None, beta_vis=BETA_VIS,
                   beta_h=BETA_H):
    """Eq. 6."""
    th1 = np.asarray(theta1, np.float64)
    th2 = np.asarray(theta2, np.float64)
    b = beta_pose(len(th1) // 3) if beta is None else np.asarray(beta, np.float64)
    return float(np.sum(b * (th1 - th2) ** 2) + beta_vis * xor_count(bits1, bits2)
                 + beta_h * float(t1 - t2) ** 2)


def object_distance(d1, d2, t1, t2, beta_d=BETA_D, beta_o=BETA_O):
    """Eq. 7."""
    dd = np.asarray(d1, np.float64) - np.asarray(d2, np.float64)
    return float(beta_d * np.sum(dd * dd) + beta_o * float(t1 - t2) ** 2)


def pool_step(pool, dist_to_pool, frame, gamma=GAMMA, cap=POOL_CAP):
    """One admission decision.  pool: list of frame ids (slots in order);
    dist_to_pool[j]: E(frame, pool[j]).  Returns (new pool, action, slot) with
    action 'first', 'append', 'replace' or 'reject'."""
    pool = list(pool)
    if not pool:
        return [frame], "first", 0
    e = np.asarray(dist_to_pool, np.float64)
    if not np.all(e > gamma):
        return pool, "reject", -1
    if len(pool) < cap:
        pool.append(frame)
        return pool, "append", len(pool) - 1
    slot = int(np.argmin(e))            # first minimum: the lower slot on ties
    pool[slot] = frame
    return pool, "replace", slot


def select(pool, dist_to_query, latest, m=M_SELECT):
    """Spatial-temporal pool: the m pooled frames with the smallest E to the
    query (ties: lower slot), then the m latest frame ids."""
    e = np.asarray(dist_to_query, np.float64)
    order = sorted(range(len(pool)), key=lambda j: (e[j], j))[:m]
    return [pool[j] for j in order], list(latest)[-m:]


def assemble(rgb_a, depth_a, alpha_a, rgb_b, depth_b, alpha_b):
    """Per-pixel depth test of two renderings (colour [n][3], un-normalised
    depth [n], opacity 1 - T_N [n]): colour [n][3], depth [n]."""
    ca, cb = np.asarray(rgb_a, np.float64), np.asarray(rgb_b, np.float64)
    da, db = np.asarray(depth_a, np.float64), np.asarray(depth_b, np.float64)
    aa, ab = np.asarray(alpha_a, np.float64), np.asarray(alpha_b, np.float64)
    za = np.where(aa > 0, da / np.where(aa > 0, aa, 1.0), 0.0)
    zb = np.where(ab > 0, db / np.where(ab > 0, ab, 1.0), 0.0)
    cov_a, cov_b = aa >= 0.5, ab >= 0.5
    take_a = cov_a & (~cov_b | (za <= zb))
    take_b = cov_b & ~take_a
    rgb = np.where(take_a[:, None], ca, np.where(take_b[:, None], cb, ca + cb))
    z_none = np.where(ab > aa, zb, za)             # 0 when both opacities are 0
    depth = np.where(take_a, za, np.where(take_b, zb, z_none))
    return rgb, depth
