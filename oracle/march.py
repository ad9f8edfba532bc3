"""Ray clipping and occupancy-skipping sample placement (test infrastructure only).

The paper trains and renders its fields "based on Instant-NGP" (Sec. 4.3)
and never describes the marcher.  The reading taken:

* clip the ray o + t d to the field's box by the slab method, intersected with
  [near, far];
* place samples at cell midpoints t_i = t_n + (i + 1/2) * delta while
  t_i < t_f, at most ``max_steps`` of them, every sample with the same delta
  (delta = sqrt(3) * side / max_steps unless a fixed step is given);
* keep a sample iff its occupancy voxel v = clamp(floor((x - lo) * res/side),
  0, res-1), linear index vx + res*(vy + res*vz), has its bit set
  (bit idx & 31 of 32-bit word idx >> 5); no bitfield keeps every sample.

These steps turn floating point into integers (how many samples, which voxel),
so they are evaluated in IEEE float32 with one rounding per +, -, *, /
(no fused multiply-add) in exactly this order:

    inv_a = 1 / d_a
    t0_a = (lo_a - o_a) * inv_a ; t1_a = (hi_a - o_a) * inv_a
    t_n = max(min(t0,t1) over a, near) ; t_f = min(max(t0,t1) over a, far)
    t_i = t_n + (float(i) + 0.5) * delta
    x_a = o_a + t_i * d_a
    v_a = clamp(floor((x_a - lo_a) * scale_a), 0, res - 1)

with scale_a = float32(res / side_a) rounded once from float64.  The sample
positions x are outputs of the marcher at that precision; everything
downstream of them is float64 here.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def clip(o, d, lo, hi, near, far):
    o = np.asarray(o, f32)
    d = np.asarray(d, f32)
    lo = np.asarray(lo, f32)
    hi = np.asarray(hi, f32)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = f32(1.0) / d
        t0 = (lo[None, :] - o) * inv
        t1 = (hi[None, :] - o) * inv
    tmin = np.minimum(t0, t1)
    tmax = np.maximum(t0, t1)
    tn = np.maximum(np.maximum(np.maximum(tmin[:, 0], tmin[:, 1]), tmin[:, 2]), f32(near))
    tf = np.minimum(np.minimum(np.minimum(tmax[:, 0], tmax[:, 1]), tmax[:, 2]), f32(far))
    return tn.astype(f32), tf.astype(f32)


def occ_scale(res, lo, hi):
    side = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    return (res / side).astype(f32)


def march(o, d, lo, hi, near, far, delta, max_steps, occ_words=None, occ_res=0):
    """Returns dict(off (R+1,) int64, ray (n,), t (n,) f32, dt (n,) f32,
    x (n,3) f32, count (R,))."""
    o = np.asarray(o, f32)
    d = np.asarray(d, f32)
    lo32 = np.asarray(lo, f32)
    R = o.shape[0]
    tn, tf = clip(o, d, lo, hi, near, far)
    i = np.arange(max_steps, dtype=f32)
    t = tn[:, None] + (i[None, :] + f32(0.5)) * f32(delta)           # (R,S)
    keep = t < tf[:, None]
    x = o[:, None, :] + t[:, :, None] * d[:, None, :]                # (R,S,3)
    if occ_words is not None and occ_res > 0:
        sc = occ_scale(occ_res, lo, hi)
        u = (x - lo32[None, None, :]) * sc[None, None, :]
        v = np.clip(np.floor(u), 0, occ_res - 1).astype(np.int64)
        idx = v[..., 0] + occ_res * (v[..., 1] + occ_res * v[..., 2])
        words = np.asarray(occ_words, np.uint32)
        bit = (words[idx >> 5] >> (idx & 31).astype(np.uint32)) & np.uint32(1)
        keep &= bit.astype(bool)
    count = keep.sum(axis=1)
    off = np.concatenate([[0], np.cumsum(count)]).astype(np.int64)
    ray = np.repeat(np.arange(R), count)
    return dict(off=off, ray=ray, t=t[keep].astype(f32),
                dt=np.full(int(off[-1]), f32(delta), f32),
                x=x[keep].astype(f32), count=count)


def march_dense(o, d, lo, hi, near, far, delta, max_steps, occ_words=None, occ_res=0):
    """Every sample inside the clipped segment, plus the occupancy bit of each
    (used to pin: skipping == dense evaluation with sigma forced to 0)."""
    full = march(o, d, lo, hi, near, far, delta, max_steps)
    if occ_words is None or occ_res == 0:
        return full, np.ones(full["t"].size, bool)
    sc = occ_scale(occ_res, lo, hi)
    u = (full["x"] - np.asarray(lo, f32)[None, :]) * sc[None, :]
    v = np.clip(np.floor(u), 0, occ_res - 1).astype(np.int64)
    idx = v[:, 0] + occ_res * (v[:, 1] + occ_res * v[:, 2])
    words = np.asarray(occ_words, np.uint32)
    bit = ((words[idx >> 5] >> (idx & 31).astype(np.uint32)) & np.uint32(1)).astype(bool)
    return full, bit


def step_size(work, fcfg):
    """delta for a workload: the fixed step if given, else sqrt(3)*side/max_steps."""
    if work.fixed_step > 0:
        return float(np.float32(work.fixed_step))
    side = max(h - l for l, h in zip(fcfg.aabb_min, fcfg.aabb_max))
    return float(np.float32(np.sqrt(3.0) * side / work.max_steps))
