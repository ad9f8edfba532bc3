"""GPU side of the multi-step training checks: the same seeded workloads as
tests/golden/make_curves.py, run through the C-ABI library."""
import math
import os

import numpy as np
import torch

import synth
from oracle import grid as ogrid

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_curve(name):
    return np.loadtxt(os.path.join(GOLDEN, name), ndmin=2)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def human_object_losses(precision, steps, use_graph=False, deform=False):
    from paper_2304_03184_amd import field as F, ops as O
    work, (fh, fo), rig, o, d, C, D, ranges, (occ_h, occ_o), rng = synth.two_field_workload()
    table_h = synth.uniform_table(ogrid.Layout.from_field(fh).n_entries, 2, rng)
    params_h = synth.xavier_params(fh.layer_shapes(), rng)
    table_o = synth.uniform_table(ogrid.Layout.from_field(fo).n_entries, 2, rng)
    params_o = synth.xavier_params(fo.layer_shapes(), rng)
    ex = work.extra
    R = O.Rig.from_numpy(rig)
    wd = O.warp_desc(n_nodes=ex["n_nodes"], lut_res=ex["knn_res"])
    dfm = None
    if deform:
        g = O.grid_desc_of(fh)
        theta, dtab, dpar = synth.deform_inputs(g.n_entries, synth.rng_for(work.seed + 91))
        dfm = F.Deform(g, theta, dtab, dpar)
    fld_h = F.Field(work, fh, table_h, params_h, occ_words=occ_h, rig=R, warp_desc=wd,
                    ray_range=ranges[0], deform=dfm)
    fld_o = F.Field(work, fo, table_o, params_o, occ_words=occ_o, ray_range=ranges[1])
    tr = F.Trainer([fld_h, fld_o], work.n_rays, work.n_rays * 128, precision=precision,
                   lambda_depth=work.lambda_depth, use_graph=use_graph)
    tr.set_batch(_dev(o), _dev(d), _dev(C), _dev(D))
    losses = [float(tr.step().item()) for _ in range(steps)]
    tr.close()
    return np.array(losses)


def psnr(c, gt, mask):
    e = (np.asarray(c, np.float64) - gt)[mask]
    return -10.0 * math.log10(float(np.mean(e * e)))


def keyframe_run(precision, steps, n_rays, eval_every, use_graph=True, deterministic=False):
    """Losses per step and {step: PSNR of the novel view} of key-frame training."""
    from paper_2304_03184_amd import field as F
    work, f, scene, cams, occ, rng = synth.keyframe_workload()
    table = synth.uniform_table(ogrid.Layout.from_field(f).n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    fld = F.Field(work, f, table, params, occ_words=occ)
    tr = F.Trainer([fld], n_rays, n_rays * 128, precision=precision,
                   lambda_depth=work.lambda_depth, use_graph=use_graph,
                   deterministic=deterministic)
    bo = torch.empty((n_rays, 3), device="cuda")
    bd = torch.empty((n_rays, 3), device="cuda")
    bC = torch.empty((n_rays, 3), device="cuda")
    bD = torch.empty(n_rays, device="cuda")
    bM = torch.empty(n_rays, device="cuda")
    tr.set_batch(bo, bd, bC, bD, bM)   # fixed buffers: the captured graph stays valid
    box = (f.aabb_min, f.aabb_max)
    eo, ed, egt, emask = synth.keyframe_eval_view(scene, box)
    eo_d, ed_d = _dev(eo), _dev(ed)
    losses, psnrs = [], {}
    for i in range(steps):
        o, d, C, D, M = synth.keyframe_batch(scene, cams, n_rays, synth.keyframe_step_rng(work, i),
                                             box)
        bo.copy_(torch.from_numpy(o))
        bd.copy_(torch.from_numpy(d))
        bC.copy_(torch.from_numpy(C))
        bD.copy_(torch.from_numpy(D))
        bM.copy_(torch.from_numpy(M))
        losses.append(tr.step().clone())   # the loss buffer is reused by the next step
        if (i + 1) % eval_every == 0:
            rgb, _ = tr.render(eo_d, ed_d, t_stop=1e-4)
            psnrs[i] = psnr(rgb.cpu().numpy(), egt, emask)
    out = torch.cat(losses).cpu().numpy().astype(np.float64)
    tr.close()
    return out, psnrs
