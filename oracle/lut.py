"""Live look-up-table construction, FP64 (test infrastructure only).

The fast neighbour search of Sec. 4.2 ("On-the-fly Radiance Fields"): a
canonical KNN field lists, for every canonical voxel k, its K nearest embedded-
graph nodes (built once); at frame t every canonical voxel centre v_k is carried
to the live space by the node blend of Eq. 1 and the live voxel f it lands in
records k, so that a live sample finds its canonical voxel, and through it its
nodes, in O(1).

Paper definitions followed:

* Eq. 1: DQB(v) = sum over the listed nodes i of w(x_i, v) dq_i, and
  v~ = SE3(DQB(v)) v, with x_i the canonical node positions and dq_i the node
  motions of frame t;
* w(x_i, v) = exp(-|v - x_i|^2 / r^2), r = 0.1 (Sec. 4.1).

Readings where the paper is silent:

* weights are taken as exp(-(|v - x_i|^2 - d_min^2) / r^2) with d_min the
  nearest listed node: a uniform scale the blend is invariant to, which keeps
  far voxels from underflowing;
* antipodal alignment of the blended dual quaternions to the first listed
  node (as in the inverse warp), then normalisation by the real part's norm;
  SE3 applied as R(c_r) v + 2 vec(c_d conj(c_r));
* voxel centres v_k = lo + (i + 1/2) side / res per axis, k = ix + res (iy +
  res iz); a voxel with no listed node (id -1) is not carried;
* the live voxel is floor((v~ - lo_live) res_live / side_live) per axis; a point
  outside the live box is dropped;
* collisions (several canonical voxels in one live voxel): the largest k is
  kept; holes (no canonical voxel): -1.

The GPU forms the live positions in float32, so voxels landing within rounding
distance of a live voxel face may go either way: ``margin`` reports, per
canonical voxel, the distance (in live voxels) of v~ to the nearest face, which
the comparison uses to tell decided voxels from undecided ones.
"""
from __future__ import annotations

import numpy as np

from . import warp

R_ED = warp.R_ED


def voxel_centres(lo, hi, res):
    """Canonical voxel centres [res^3][3], index ix + res (iy + res iz)."""
    lo = np.asarray(lo, np.float64)
    step = (np.asarray(hi, np.float64) - lo) / res
    i = np.arange(res ** 3)
    idx = np.stack([i % res, (i // res) % res, i // (res * res)], 1)
    return lo + (idx + 0.5) * step


def forward_dqb(v, ids, node_canon, node_dq, r=R_ED):
    """Eq. 1 for points v [n][3] with listed node ids [n][K] (nearest first, -1 =
    none).  Returns (live positions [n][3], carried [n] bool)."""
    v = np.asarray(v, np.float64)
    ids = np.asarray(ids, np.int64)
    have = ids >= 0
    safe = np.where(have, ids, 0)
    xi = np.asarray(node_canon, np.float64)[safe]                 # n,K,3
    d2 = np.sum((v[:, None, :] - xi) ** 2, axis=-1)
    d2 = np.where(have, d2, np.inf)
    dmin = np.min(d2, axis=1, keepdims=True)
    carried = have[:, 0]
    w = np.where(have, np.exp(-(d2 - np.where(carried[:, None], dmin, 0.0)) / (r * r)), 0.0)
    dq = np.asarray(node_dq, np.float64)[safe]                    # n,K,8
    s = warp.sign_to_first(dq[..., :4])                           # n,K (float32 decision)
    b = np.sum((s * w)[..., None] * dq, axis=1)                   # n,8
    nrm = np.linalg.norm(b[:, :4], axis=1, keepdims=True)
    c = b / np.where(nrm > 0, nrm, 1.0)
    live = warp.dq_apply(c, v)
    return live, carried


def live_coords(live, lo, hi, res):
    """Continuous live-voxel coordinates (v~ - lo) res / side [n][3]."""
    lo = np.asarray(lo, np.float64)
    return (np.asarray(live, np.float64) - lo) * (res / (np.asarray(hi, np.float64) - lo))


def assemble(u, carried, res):
    """Live look-up table from continuous live-voxel coordinates u [n][3] of the
    canonical voxels 0..n-1: int64 [res^3], the largest canonical index per live
    voxel, -1 where none lands."""
    u = np.asarray(u, np.float64)
    cell = np.floor(u).astype(np.int64)
    inside = carried & np.all((cell >= 0) & (cell < res), axis=1)
    k = np.nonzero(inside)[0]
    f = cell[k, 0] + res * (cell[k, 1] + res * cell[k, 2])
    lut = np.full(res ** 3, -1, np.int64)
    np.maximum.at(lut, f, k)
    return lut


def build(canon_lo, canon_hi, canon_res, knn, node_canon, node_dq, live_lo, live_hi, live_res,
          r=R_ED):
    """The live table and, per canonical voxel, its live coordinates and the
    distance of its live position to the nearest live-voxel face (in voxels)."""
    v = voxel_centres(canon_lo, canon_hi, canon_res)
    live, carried = forward_dqb(v, knn, node_canon, node_dq, r)
    u = live_coords(live, live_lo, live_hi, live_res)
    frac = u - np.floor(u)
    margin = np.min(np.minimum(frac, 1.0 - frac), axis=1)
    return assemble(u, carried, live_res), u, carried, margin
