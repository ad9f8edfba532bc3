"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *draws* inputs: rays, occupancy bitfields, table and weight
initialisations, skeleton / embedded-graph poses, neighbour look-up grids and
colour / depth targets.  It holds none of the method's arithmetic (no hash
encoding, no network, no compositing, no blended warp): both the FP64 oracle and
the HIP path consume the arrays produced here, and neither is imported here.

Every generator takes a ``numpy.random.Generator`` (PCG64) so that a seed fully
determines an input.  Arrays are returned in the dtypes the library consumes
(float32 positions / directions / parameters, uint32 bitfield words, uint16
node ids).

Workload shapes follow the five configurations the implementation is measured
on (sizes only; derived quantities such as level resolutions are computed by
each side itself):

* ``cfg1`` plain static FP32 field: 4096 rays from a radius-2 sphere aimed at
  the origin, 64 uniform samples in [1, 3], L=8, F=2, T=2^14, N 16->512.
* ``cfg2`` Instant-NGP-scale object field: 2^18 rays, <=128 samples/ray,
  128^3 occupancy (~30 % set), L=16, F=2, T=2^19, N 16->2048.
* ``cfg3`` dynamic human field behind the hybrid warp (24 joints, 1024 nodes).
* ``cfg4`` human (T=2^19) + object (T=2^18) fields, 180k / 80k rays of which
  20k are shared.
* ``cfg5`` key-frame refinement and a 1920x1080 novel view.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "FieldCfg", "WorkCfg", "config", "rng_for",
    "sphere_rays", "noise_occupancy", "occupancy_from_points", "pack_bits",
    "uniform_table", "xavier_params", "smooth_colour_targets", "uniform_targets",
    "human_rig", "object_points", "keyframe_scene", "human_workload", "two_field_workload",
    "keyframe_workload", "deform_inputs", "DEFORM_SHAPES",
]


# ----------------------------------------------------------------------------
# configuration records (sizes only)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class FieldCfg:
    """Sizes of one radiance field (hash grid + two tiny networks)."""
    n_levels: int = 16          # L
    n_features: int = 2         # F
    log2_table: int = 19        # log2 T
    res_min: int = 16           # N_min
    res_max: int = 2048         # N_max
    aabb_min: tuple = (-1.0, -1.0, -1.0)
    aabb_max: tuple = (1.0, 1.0, 1.0)
    density_hidden: tuple = (64,)
    density_out: int = 16
    colour_hidden: tuple = (64, 64)
    sh_degree: int = 4          # number of SH bands; d bands give d*d coefficients
    occ_res: int = 128          # occupancy bitfield resolution (0: no occupancy test)

    @property
    def enc_width(self) -> int:
        return self.n_levels * self.n_features

    @property
    def n_sh(self) -> int:
        return self.sh_degree * self.sh_degree

    def layer_shapes(self):
        """(out, in) of every linear layer, density network first."""
        shapes = []
        d = [self.enc_width, *self.density_hidden, self.density_out]
        shapes += [(d[i + 1], d[i]) for i in range(len(d) - 1)]
        c = [self.density_out + self.n_sh, *self.colour_hidden, 3]
        shapes += [(c[i + 1], c[i]) for i in range(len(c) - 1)]
        return shapes

    @property
    def n_params(self) -> int:
        return sum(o * i for o, i in self.layer_shapes())


@dataclass(frozen=True)
class WorkCfg:
    name: str
    n_rays: int
    fields: tuple
    near: float = 0.0
    far: float = 1.0e30
    max_steps: int = 128        # samples per ray on the full box diagonal
    fixed_step: float = 0.0     # >0: use this step instead of sqrt(3)*side/max_steps
    lambda_depth: float = 0.0
    warp: bool = False
    seed: int = 0
    extra: dict = field(default_factory=dict)


def config(k: int, scale: float = 1.0) -> WorkCfg:
    """Workload configuration ``k`` (1..5).  ``scale`` shrinks the ray count
    (e.g. 1/64 for the oracle-sized runs) without touching the field sizes."""
    seed = 20230400 + k
    def rays(n):
        return max(1, int(round(n * scale)))
    if k == 1:
        f = FieldCfg(n_levels=8, log2_table=14, res_max=512,
                     aabb_min=(-1.5,) * 3, aabb_max=(1.5,) * 3,
                     colour_hidden=(64,), sh_degree=2, occ_res=0)
        return WorkCfg("cfg1_plain_static_fp32", rays(4096), (f,), near=1.0, far=3.0,
                       max_steps=64, fixed_step=2.0 / 64.0, seed=seed)
    if k == 2:
        return WorkCfg("cfg2_ngp_object_2p18", rays(1 << 18), (FieldCfg(),), seed=seed)
    if k == 3:
        return WorkCfg("cfg3_human_hybrid_warp_2p18", rays(1 << 18), (FieldCfg(),),
                       warp=True, seed=seed,
                       extra=dict(n_joints=24, k_joints=4, n_nodes=1024, k_nodes=8,
                                  knn_res=128))
    if k == 4:
        human = FieldCfg()
        obj = FieldCfg(log2_table=18)
        return WorkCfg("cfg4_human_object_180k_80k", rays(240000), (human, obj),
                       warp=True, lambda_depth=1.0, seed=seed,
                       extra=dict(n_joints=24, k_joints=4, n_nodes=1024, k_nodes=8,
                                  knn_res=128, human_only=rays(160000),
                                  shared=rays(20000), object_only=rays(60000)))
    if k == 5:
        f = FieldCfg(aabb_min=(-1.5,) * 3, aabb_max=(1.5,) * 3)
        return WorkCfg("cfg5_keyframes_2p20_render_1080p", rays(1 << 20), (f,),
                       lambda_depth=1.0, seed=seed,
                       extra=dict(n_keyframes=8, kf_w=1280, kf_h=720,
                                  render_w=1920, render_h=1080, t_stop=1e-4))
    raise ValueError(f"unknown configuration {k}")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------
def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def sphere_rays(n: int, rng, radius: float = 2.0, aim_lo=(-0.25,) * 3,
                aim_hi=(0.25,) * 3):
    """Origins uniform on a sphere of ``radius``, each aimed at a point drawn
    uniformly in the box [aim_lo, aim_hi].  Returned as float32 (n,3) arrays;
    directions are unit length in float64 before the cast."""
    u = _unit(rng.normal(size=(n, 3)))
    o = radius * u
    c = rng.uniform(aim_lo, aim_hi, size=(n, 3))
    d = _unit(c - o)
    return o.astype(np.float32), d.astype(np.float32)


# ----------------------------------------------------------------------------
# occupancy
# ----------------------------------------------------------------------------
def pack_bits(occ: np.ndarray) -> np.ndarray:
    """Pack a boolean (R,R,R) grid indexed [z,y,x] into uint32 words; voxel
    (x,y,z) has linear index x + R*(y + R*z) and lives in bit (idx & 31) of
    word idx >> 5."""
    flat = occ.reshape(-1).astype(np.uint64)
    n = flat.size
    words = np.zeros((n + 31) // 32, dtype=np.uint64)
    idx = np.arange(n)
    np.add.at(words, idx >> 5, flat << (idx & 31).astype(np.uint64))
    return words.astype(np.uint32)


def noise_occupancy(res: int, rng, frac: float = 0.30, n_waves: int = 8,
                    bernoulli: bool = False):
    """Smooth-noise occupancy: the sum of ``n_waves`` random 3-D sinusoids with
    1..4 cycles across the box, thresholded at its (1-frac) quantile.  With
    ``bernoulli`` every voxel is set independently with probability ``frac``.
    Returns (bool grid [z,y,x], packed uint32 words)."""
    if bernoulli:
        occ = rng.uniform(size=(res, res, res)) < frac
        return occ, pack_bits(occ)
    g = (np.arange(res) + 0.5) / res
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    s = np.zeros((res, res, res))
    for _ in range(n_waves):
        k = rng.uniform(1.0, 4.0, size=3) * rng.choice([-1, 1], size=3)
        ph = rng.uniform(0, 2 * math.pi)
        s += np.sin(2 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
    thr = np.quantile(s, 1.0 - frac)
    occ = s > thr
    return occ, pack_bits(occ)


def occupancy_from_points(points: np.ndarray, radius: float, res: int,
                          aabb_min, aabb_max):
    """Voxels whose centre lies within ``radius`` of any point."""
    from scipy.spatial import cKDTree
    lo = np.asarray(aabb_min, float)
    hi = np.asarray(aabb_max, float)
    g = (np.arange(res) + 0.5) / res
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    centres = lo + np.stack([x, y, z], -1).reshape(-1, 3) * (hi - lo)
    tree = cKDTree(points)
    dist, _ = tree.query(centres, k=1)
    occ = (dist <= radius).reshape(res, res, res)
    return occ, pack_bits(occ)


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------
def uniform_table(n_entries: int, n_features: int, rng, lo=-0.1, hi=0.1):
    return rng.uniform(lo, hi, size=(n_entries, n_features)).astype(np.float32)


# layer shapes (out, in) of the deformation network: [32-wide encoding, 72-wide
# pose] -> 4 x 128 -> 3
DEFORM_SHAPES = ((128, 104), (128, 128), (128, 128), (128, 128), (3, 128))


def xavier_params(shapes, rng):
    """Xavier-uniform U[-a, a], a = sqrt(6/(fan_in+fan_out)), for each (out,in)
    layer; concatenated row-major into one float32 vector."""
    parts = []
    for o, i in shapes:
        a = math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=(o, i)).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------
# targets
# ----------------------------------------------------------------------------
def deform_inputs(n_entries: int, rng, pose_scale=0.3, out_scale=0.05):
    """Inputs of a deformation network (Sec. 4.2; widths in Sec. 4.3): pose
    theta (72, normal with std pose_scale), its 2-feature table (uniform_table)
    and Xavier weights for DEFORM_SHAPES with the output layer scaled by
    out_scale, so the residual starts at about a centimetre.  Returns (theta,
    table, params), float32."""
    theta = rng.normal(scale=pose_scale, size=72).astype(np.float32)
    table = uniform_table(n_entries, 2, rng)
    params = xavier_params(DEFORM_SHAPES, rng)
    n_out = DEFORM_SHAPES[-1][0] * DEFORM_SHAPES[-1][1]
    params[-n_out:] *= np.float32(out_scale)
    return theta, table, params


def uniform_targets(n: int, rng):
    return rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)


def smooth_colour_targets(o, d, rng, n_waves: int = 4):
    """Smooth colours of a ray: 0.5 + 0.5*sin of random linear forms in
    (origin, direction), per channel.  Learnable, multi-view consistent enough
    for a throughput workload."""
    x = np.concatenate([o, d], axis=1).astype(np.float64)
    out = np.zeros((x.shape[0], 3))
    for c in range(3):
        acc = np.zeros(x.shape[0])
        for _ in range(n_waves):
            k = rng.normal(size=6)
            acc += np.sin(x @ k + rng.uniform(0, 2 * math.pi))
        out[:, c] = 0.5 + 0.5 * np.tanh(acc / n_waves)
    return out.astype(np.float32)


# ----------------------------------------------------------------------------
# skeleton + embedded graph (human field)
# ----------------------------------------------------------------------------
# A 24-joint stick figure (metres, y up), joint order pelvis-first; parents only
# serve to place capsules for node sampling.
_JOINTS = np.array([
    [0.00, 0.00, 0.00], [0.09, -0.08, 0.0], [-0.09, -0.08, 0.0], [0.00, 0.12, 0.0],
    [0.10, -0.48, 0.0], [-0.10, -0.48, 0.0], [0.00, 0.25, 0.0], [0.10, -0.86, 0.0],
    [-0.10, -0.86, 0.0], [0.00, 0.38, 0.0], [0.10, -0.92, 0.08], [-0.10, -0.92, 0.08],
    [0.00, 0.55, 0.0], [0.08, 0.50, 0.0], [-0.08, 0.50, 0.0], [0.00, 0.68, 0.0],
    [0.18, 0.52, 0.0], [-0.18, 0.52, 0.0], [0.45, 0.52, 0.0], [-0.45, 0.52, 0.0],
    [0.70, 0.52, 0.0], [-0.70, 0.52, 0.0], [0.80, 0.52, 0.0], [-0.80, 0.52, 0.0]])
_PARENT = [-1, 0, 0, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 9, 9, 12, 13, 14, 16, 17, 18, 19, 20, 21]
_RADIUS = [0.12, 0.08, 0.08, 0.12, 0.06, 0.06, 0.12, 0.05, 0.05, 0.12, 0.04, 0.04,
           0.06, 0.06, 0.06, 0.09, 0.05, 0.05, 0.045, 0.045, 0.04, 0.04, 0.04, 0.04]


def _rodrigues(axis, angle):
    axis = _unit(axis)
    K = np.zeros(axis.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2] = -axis[..., 2], axis[..., 1]
    K[..., 1, 0], K[..., 1, 2] = axis[..., 2], -axis[..., 0]
    K[..., 2, 0], K[..., 2, 1] = -axis[..., 1], axis[..., 0]
    s = np.sin(angle)[..., None, None]
    c = np.cos(angle)[..., None, None]
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + s * K + (1 - c) * (K @ K)


def _quat_from_axis_angle(axis, angle):
    axis = _unit(axis)
    h = 0.5 * angle
    return np.concatenate([np.cos(h)[..., None], np.sin(h)[..., None] * axis], -1)


def _qmul(a, b):
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def human_rig(rng, n_nodes=1024, k_nodes=8, knn_res=128, max_bone_deg=30.0,
              max_node_deg=5.0, max_node_trans=0.05, aabb_min=(-1.0,) * 3,
              aabb_max=(1.0,) * 3, n_frames=1):
    """Synthetic posed human for the hybrid warp.

    Returns a dict of float32 / uint16 arrays:

    * ``joints`` (24,3): joint centres (live = canonical: every bone rotates
      about its own joint centre).
    * ``bones`` (F,24,3,4): per-joint live->canonical rigid transforms [R|t],
      rotation about the joint centre, axis uniform, angle U[0, 30 deg].
    * ``node_dq`` (F,M,8): embedded-graph node motions as dual quaternions
      (real w,x,y,z then dual w,x,y,z): a rotation about the node of angle
      U[0, 5 deg] (axis uniform) and a translation uniform in a 5 cm ball.
    * ``node_pos`` (F,M,3): the deformed node positions (node + translation).
    * ``knn`` (F,R^3,K) uint16: for each live voxel centre (linear index
      x + R*(y + R*z) over the box) the K nodes nearest to it, sorted by
      distance, where a node's live position is its deformed position carried
      by the forward motion of the bone nearest to the node (the generator's own
      rigging; ties are measure-zero for these random positions).
    * ``node_live`` (F,M,3): those live node positions (for occupancy).
    * ``node_canon`` (M,3): canonical node positions.
    """
    from scipy.spatial import cKDTree
    J = _JOINTS.copy()
    nj = J.shape[0]
    # canonical nodes sampled inside capsules around bones (parent->child)
    segs = [(J[_PARENT[j]], J[j], _RADIUS[j]) for j in range(1, nj)]
    lens = np.array([np.linalg.norm(b - a) + 1e-3 for a, b, _ in segs])
    which = rng.choice(len(segs), size=n_nodes, p=lens / lens.sum())
    tpar = rng.uniform(size=n_nodes)
    dirs = _unit(rng.normal(size=(n_nodes, 3)))
    rad = rng.uniform(size=n_nodes) ** (1 / 3)
    canon = np.empty((n_nodes, 3))
    owner = np.empty(n_nodes, int)
    for n in range(n_nodes):
        a, b, r = segs[which[n]]
        canon[n] = a + tpar[n] * (b - a) + dirs[n] * rad[n] * r
        owner[n] = which[n] + 1
    lo = np.asarray(aabb_min, float)
    hi = np.asarray(aabb_max, float)
    g = (np.arange(knn_res) + 0.5) / knn_res
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    centres = lo + np.stack([xx, yy, zz], -1).reshape(-1, 3) * (hi - lo)

    bones_f, dq_f, pos_f, knn_f, live_f = [], [], [], [], []
    for _ in range(n_frames):
        ang = np.deg2rad(rng.uniform(0, max_bone_deg, size=nj))
        R = _rodrigues(rng.normal(size=(nj, 3)), ang)       # live->canonical rotation
        t = J - np.einsum("jab,jb->ja", R, J)                 # about the joint centre
        bones = np.concatenate([R, t[..., None]], -1)          # (24,3,4)
        # node motions: rotate about the node, then translate
        nang = np.deg2rad(rng.uniform(0, max_node_deg, size=n_nodes))
        q = _quat_from_axis_angle(rng.normal(size=(n_nodes, 3)), nang)
        tr = _unit(rng.normal(size=(n_nodes, 3))) * (
            max_node_trans * rng.uniform(size=(n_nodes, 1)) ** (1 / 3))
        Rn = _rodrigues(q[:, 1:] / np.maximum(np.linalg.norm(q[:, 1:], axis=1,
                                                             keepdims=True), 1e-300),
                        nang)
        T = canon - np.einsum("nab,nb->na", Rn, canon) + tr    # global translation
        qd = 0.5 * _qmul(np.concatenate([np.zeros((n_nodes, 1)), T], 1), q)
        dq = np.concatenate([q, qd], 1)
        pos = canon + tr
        # live node positions: forward motion of the owning bone (inverse of [R|t])
        Ro = R[owner]
        live = np.einsum("nba,nb->na", Ro, pos - t[owner])
        tree = cKDTree(live)
        _, nn = tree.query(centres, k=k_nodes)
        bones_f.append(bones)
        dq_f.append(dq)
        pos_f.append(pos)
        knn_f.append(nn.astype(np.uint16))
        live_f.append(live)
    return dict(joints=J.astype(np.float32),
                bones=np.stack(bones_f).astype(np.float32),
                node_dq=np.stack(dq_f).astype(np.float32),
                node_pos=np.stack(pos_f).astype(np.float32),
                knn=np.stack(knn_f),
                node_live=np.stack(live_f).astype(np.float32),
                node_canon=canon.astype(np.float32))


def object_points(rng, centre=(0.55, 0.45, 0.15), half=(0.12, 0.08, 0.10), n=4000):
    """Points filling a small box (a hand-held object) for its occupancy."""
    c = np.asarray(centre)
    h = np.asarray(half)
    return (c + rng.uniform(-1, 1, size=(n, 3)) * h).astype(np.float32)


# ----------------------------------------------------------------------------
# key-frame scene (analytic spheres + back plane)
# ----------------------------------------------------------------------------
def keyframe_scene(rng, n_spheres=6):
    """Scene parameters: sphere centres/radii, a back plane z = -1.2 and a smooth
    colour field 1/(1+exp(-s(x))) with s a sum of 8 random 3-D sinusoids."""
    cen = rng.uniform(-0.7, 0.7, size=(n_spheres, 3))
    rad = rng.uniform(0.1, 0.4, size=n_spheres)
    waves = [(rng.normal(size=(3, 3)) * 3.0, rng.uniform(0, 2 * math.pi, size=3))
             for _ in range(8)]
    return dict(centres=cen, radii=rad, plane_z=-1.2, waves=waves)


def scene_colour(scene, p):
    s = np.zeros(p.shape[:-1] + (3,))
    for k, ph in scene["waves"]:
        s += np.sin(p @ k.T + ph)
    return 1.0 / (1.0 + np.exp(-s / 2.0))


def scene_trace(scene, o, d):
    """Nearest hit distance along each ray (inf if none) and the hit colour."""
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    best = np.full(o.shape[0], np.inf)
    for c, r in zip(scene["centres"], scene["radii"]):
        oc = o - c
        b = np.sum(oc * d, 1)
        cc = np.sum(oc * oc, 1) - r * r
        disc = b * b - cc
        ok = disc > 0
        tt = np.where(ok, -b - np.sqrt(np.where(ok, disc, 0)), np.inf)
        tt = np.where(tt > 0, tt, np.inf)
        best = np.minimum(best, tt)
    tp = (scene["plane_z"] - o[:, 2]) / np.where(np.abs(d[:, 2]) > 1e-12, d[:, 2], 1e-12)
    tp = np.where(tp > 0, tp, np.inf)
    best = np.minimum(best, tp)
    hit = o + np.where(np.isfinite(best), best, 0)[:, None] * d
    col = scene_colour(scene, hit)
    col[~np.isfinite(best)] = 0.0
    return best, col


def look_at_cameras(n, radius=2.0, arc_deg=90.0, height=0.3):
    """Camera-to-world rotations and centres on an arc looking at the origin."""
    out = []
    for i in range(n):
        a = math.radians(-arc_deg / 2 + arc_deg * i / max(n - 1, 1))
        c = np.array([radius * math.sin(a), height, radius * math.cos(a)])
        fwd = _unit(-c)
        right = _unit(np.cross(fwd, [0, 1, 0]))
        up = np.cross(right, fwd)
        R = np.stack([right, up, fwd], 1)   # columns: x right, y up, z forward
        out.append((R, c))
    return out


def pixel_rays(R, c, w, h, f, pix=None):
    """Unit-direction rays of a pinhole camera (principal point at the centre).
    ``pix`` selects linear pixel ids; default all pixels, row-major."""
    if pix is None:
        pix = np.arange(w * h)
    u = (pix % w) + 0.5
    v = (pix // w) + 0.5
    dc = np.stack([(u - w / 2) / f, -(v - h / 2) / f, np.ones_like(u, dtype=float)], 1)
    d = _unit(dc @ R.T)
    o = np.broadcast_to(c, d.shape).copy()
    return o.astype(np.float32), d.astype(np.float32)


def keyframe_occupancy(scene, res, aabb_min, aabb_max, band_voxels=2.0):
    """Voxels inside a sphere or whose centre lies within ``band_voxels`` voxel
    sizes of a sphere surface or of the back plane."""
    lo = np.asarray(aabb_min, float)
    hi = np.asarray(aabb_max, float)
    vox = float(np.max((hi - lo) / res))
    g = (np.arange(res) + 0.5) / res
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    p = lo + np.stack([x, y, z], -1) * (hi - lo)
    occ = np.abs(p[..., 2] - scene["plane_z"]) <= band_voxels * vox
    for c, r in zip(scene["centres"], scene["radii"]):
        occ |= np.linalg.norm(p - c, axis=-1) - r <= band_voxels * vox
    return occ, pack_bits(occ)


def _inside(p, box):
    lo, hi = np.asarray(box[0], float), np.asarray(box[1], float)
    return np.all((p >= lo) & (p <= hi), axis=-1)


def keyframe_batch(scene, cams, n_rays, rng, box, w=1280, h=720, f=1000.0, depth_noise=0.005):
    """One training batch drawn uniformly over the pixels of the key frames:
    rays, target colours and along-ray depths (the z-depth in the camera gets
    N(0, depth_noise) noise, then is converted to the distance along the ray),
    and the loss mask: 1 for rays whose first hit lies inside ``box`` (the
    field's box; other targets are out of the field's reach)."""
    cam = rng.integers(0, len(cams), size=n_rays)
    pix = rng.integers(0, w * h, size=n_rays)
    o = np.empty((n_rays, 3), np.float32)
    d = np.empty((n_rays, 3), np.float32)
    cosz = np.empty(n_rays)
    for k, (R, c) in enumerate(cams):
        sel = np.nonzero(cam == k)[0]
        if sel.size == 0:
            continue
        ok, dk = pixel_rays(R, c, w, h, f, pix[sel])
        o[sel], d[sel] = ok, dk
        cosz[sel] = dk.astype(np.float64) @ R[:, 2]
    t, col = scene_trace(scene, o, d)
    hit = np.isfinite(t)
    zdepth = np.where(hit, t * cosz, 0.0) + rng.normal(0.0, depth_noise, size=n_rays)
    D = np.where(hit, zdepth / cosz, 0.0)
    p = o.astype(np.float64) + np.where(hit, t, 0.0)[:, None] * d.astype(np.float64)
    mask = hit & _inside(p, box)
    return (o, d, col.astype(np.float32), D.astype(np.float32), mask.astype(np.float32))


def keyframe_eval_view(scene, box, w=160, h=90, f=125.0, angle_deg=20.0, radius=2.0,
                       height=0.3):
    """A novel view between key frames (same arc, angle in degrees from the
    arc centre): rays, ground-truth colours and the mask of pixels whose first
    hit lies inside ``box``."""
    a = math.radians(angle_deg)
    c = np.array([radius * math.sin(a), height, radius * math.cos(a)])
    fwd = _unit(-c)
    right = _unit(np.cross(fwd, [0, 1, 0]))
    up = np.cross(right, fwd)
    R = np.stack([right, up, fwd], 1)
    o, d = pixel_rays(R, c, w, h, f)
    t, col = scene_trace(scene, o, d)
    hit = np.isfinite(t)
    p = o.astype(np.float64) + np.where(hit, t, 0.0)[:, None] * d.astype(np.float64)
    return o, d, col.astype(np.float32), hit & _inside(p, box)


def keyframe_workload(seed_offset=0):
    """Key-frame refinement inputs: (work, field cfg, scene, 8 key-frame
    cameras, packed analytic occupancy, rng).  The caller draws the table and
    weights from ``rng`` next (table first), and the batch of step i from
    ``keyframe_step_rng(work, i)``."""
    work = config(5)
    fcfg = work.fields[0]
    rng = rng_for(work.seed + seed_offset)
    scene = keyframe_scene(rng)
    cams = look_at_cameras(8)
    _, words = keyframe_occupancy(scene, fcfg.occ_res, fcfg.aabb_min, fcfg.aabb_max)
    return work, fcfg, scene, cams, words, rng


def keyframe_step_rng(work, step):
    return rng_for(work.seed * 1000 + 7 + step)


def human_workload(scale=1.0, seed_offset=0):
    """The human field behind the hybrid warp at ``scale`` of its ray count:
    (work, field cfg, rig, rays o, d, smooth colour targets, packed live-space
    occupancy, rng).  The caller draws the table and weights from ``rng`` next."""
    work = config(3, scale)
    f = work.fields[0]
    ex = work.extra
    rng = rng_for(work.seed + seed_offset)
    rig = human_rig(rng, n_nodes=ex["n_nodes"], k_nodes=ex["k_nodes"], knn_res=ex["knn_res"])
    o, d = sphere_rays(work.n_rays, rng, aim_lo=(-0.3, -0.8, -0.2), aim_hi=(0.3, 0.8, 0.2))
    _, occ = occupancy_from_points(rig["node_live"][0], 0.12, f.occ_res, f.aabb_min, f.aabb_max)
    C = smooth_colour_targets(o, d, rng)
    return work, f, rig, o, d, C, occ, rng


def two_field_workload(scale=1.0 / 64, seed_offset=0):
    """Human (hybrid warp) + object fields over uneven ray ranges with shared
    rays, at ``scale`` of the full ray counts: (work, (human cfg, object cfg),
    rig, rays o, d, targets C, D, ray ranges, packed occupancies, rng).  The
    caller draws the two tables and weights from ``rng`` next (human table,
    human weights, object table, object weights)."""
    work = config(4, scale)
    fh, fo = work.fields
    ex = work.extra
    rng = rng_for(work.seed + seed_offset)
    rig = human_rig(rng, n_nodes=ex["n_nodes"], k_nodes=ex["k_nodes"], knn_res=ex["knn_res"])
    n = work.n_rays
    h_end = ex["human_only"] + ex["shared"]
    o_begin = ex["human_only"]
    o, d = sphere_rays(n, rng, aim_lo=(-0.3, -0.8, -0.2), aim_hi=(0.6, 0.8, 0.3))
    _, occ_h = occupancy_from_points(rig["node_live"][0], 0.12, fh.occ_res, fh.aabb_min,
                                     fh.aabb_max)
    _, occ_o = occupancy_from_points(object_points(rng), 0.1, fo.occ_res, fo.aabb_min,
                                     fo.aabb_max)
    C = uniform_targets(n, rng)
    D = rng.uniform(1.0, 3.0, size=n).astype(np.float32)
    return work, (fh, fo), rig, o, d, C, D, [(0, h_end), (o_begin, n)], (occ_h, occ_o), rng
