"""Shared helpers of the GPU parity tests (inputs from synth, references from
the oracle; nothing here runs the method's arithmetic itself)."""
import numpy as np

import synth
from oracle import grid as ogrid

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def f16_round(a):
    return np.asarray(a, np.float32).astype(np.float16).astype(np.float64)


def bf16_round(a):
    x = np.ascontiguousarray(np.asarray(a, np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def field_inputs(k, n_rays, seed_offset=0, occ_res=None):
    """Rays, targets, table, params (and occupancy) of workload k at n_rays."""
    w = synth.config(k)
    f = w.fields[0]
    if occ_res is not None:
        f = synth.FieldCfg(**{**f.__dict__, "occ_res": occ_res})
    w = synth.WorkCfg(**{**w.__dict__, "n_rays": n_rays, "fields": (f,)})
    rng = synth.rng_for(w.seed + seed_offset)
    if k == 1:
        o, d = synth.sphere_rays(n_rays, rng)
    else:
        o, d = synth.sphere_rays(n_rays, rng)
    occ_words = None
    if f.occ_res > 0:
        _, occ_words = synth.noise_occupancy(f.occ_res, rng)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, f.n_features, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    Ct = synth.uniform_targets(n_rays, rng)
    return dict(work=w, fcfg=f, o=o, d=d, occ=occ_words, table=table, params=params, Ct=Ct,
                lay=lay, rng=rng)


def decided_rays(work, fcfg, rig, o, d, occ_words, grid_box, margin, want, ray_lo=0,
                 deform=None):
    """Indices (first ``want``) of the rays all of whose kept samples land,
    under the oracle's float64 warp, at least ``margin`` metres from every cell
    face of every level of the field's encoding.  On such rays the float32
    canonical positions of the GPU warp (a few 1e-7 m away) pick the same cells,
    so the encoding's position gradient (discontinuous across faces) is the
    same function on both sides.  With ``deform`` = (layout, theta, table,
    params) of a deformation network, the warped points must also keep the
    margin on its encoding's ladder, and the deformed points on the field's.
    Only synth inputs and oracle arithmetic are used to choose them."""
    from oracle import deform as odef, march as omarch, warp as owarp
    m = omarch.march(o, d, fcfg.aabb_min, fcfg.aabb_max, work.near, work.far,
                     omarch.step_size(work, fcfg), work.max_steps, occ_words, fcfg.occ_res)
    xc = owarp.warp(m["x"], rig, grid_box[0], grid_box[1])
    lay = ogrid.Layout.from_field(fcfg)
    checks = [(xc, lay)]
    if deform is not None:
        dlay, theta, table, params = deform
        xd, _ = odef.forward(params, xc, theta, table, dlay)
        checks = [(xc, dlay), (xd, lay)]
    ok = np.ones(xc.shape[0], bool)
    for pts, ly in checks:
        for N in ly.res:
            u = np.clip((pts - ly.lo) / ly.side, 0.0, 1.0) * N
            ok &= (np.abs(u - np.round(u)) * ly.side / N >= margin).all(axis=1)
    bad = np.bincount(m["ray"], weights=(~ok).astype(np.float64), minlength=o.shape[0])
    good = np.nonzero((bad == 0) & (m["count"] > 0))[0]
    assert good.size >= want, f"only {good.size} decided rays"
    return good[:want]
