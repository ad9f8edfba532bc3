"""Writes the FP64 oracle's multi-step training curves that the GPU tests
compare against (test infrastructure; calls only ``oracle/`` and ``synth/``).

* ``curve_human_object_r64.txt``: the two-field workload (human field behind
  the hybrid warp + object field, shared rays composited as one merged list,
  colour + depth loss, Eq. 8) at 1/64 of its ray counts, one fixed batch,
  Adam, loss per step.
* ``curve_human_object_deform_r64.txt``: the same with the pose-conditioned
  deformation network between the human field's warp and its encoding
  (Sec. 4.2; its own 16-level grid on the human field's ladder, inputs from
  ``synth.deform_inputs``), trained with the fields.
* ``curve_human_object_deform_r64_perturbed.txt`` (``--perturb EPS``): the
  same oracle run with every warped position moved by U[-EPS, EPS] per
  coordinate (EPS the size of the float32 warp's rounding), which measures how
  fast the training trajectory itself separates under float32-sized errors.
* ``curve_human_object_deform_r64_gradnoise.txt`` (``--perturb-grad REL``):
  the same oracle run with an error of relative norm REL added to every
  gradient array before each Adam update (each non-zero entry gets
  REL * rms * U[-sqrt 3, sqrt 3], rms over the array's non-zero entries; zero
  entries stay zero), REL = 5e-2 being the BF16 step's gradient bar: the
  separation to expect from gradients carrying errors of that size.
* ``curve_keyframes_4096.txt``: key-frame refinement (rays drawn per step from
  eight 1280x720 key frames of the analytic scene, colour + depth loss with
  the mask M(r) of Eq. 8 set for rays whose first hit lies in the field's box,
  Adam), 4096 rays per step; loss per step and the PSNR (over the pixels whose
  hit lies in the box) of a 160x90 novel view rendered with early termination
  every ``--eval-every`` steps.

Usage (from the repository root):
    python tests/golden/make_curves.py human_object --steps 500
    python tests/golden/make_curves.py human_object_deform --steps 200
    python tests/golden/make_curves.py human_object_deform --steps 200 --perturb 2.5e-7
    python tests/golden/make_curves.py human_object_deform --steps 200 --perturb-grad 5e-2
    python tests/golden/make_curves.py keyframes --steps 2000 --eval-every 250
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import optim, grid as ogrid, step as ostep  # noqa: E402


def human_object_state(deform=False):
    work, (fh, fo), rig, o, d, C, D, ranges, (occ_h, occ_o), rng = synth.two_field_workload()
    table_h = synth.uniform_table(ogrid.Layout.from_field(fh).n_entries, 2, rng)
    params_h = synth.xavier_params(fh.layer_shapes(), rng)
    table_o = synth.uniform_table(ogrid.Layout.from_field(fo).n_entries, 2, rng)
    params_o = synth.xavier_params(fo.layer_shapes(), rng)
    dfm = None
    if deform:
        lay = ogrid.Layout.from_field(fh)
        theta, table, params = synth.deform_inputs(lay.n_entries, synth.rng_for(work.seed + 91))
        dfm = ostep.DeformState(lay, theta, table, params)
    st = ostep.StepState([ostep.FieldState(fh, table_h, params_h, occ_words=occ_h, rig=rig,
                                           deform=dfm),
                          ostep.FieldState(fo, table_o, params_o, occ_words=occ_o)])
    return work, st, o, d, C, D, ranges


def keyframe_state():
    work, f, scene, cams, occ, rng = synth.keyframe_workload()
    table = synth.uniform_table(ogrid.Layout.from_field(f).n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    st = ostep.StepState([ostep.FieldState(f, table, params, occ_words=occ)])
    return work, f, scene, cams, st


def psnr(c, gt, mask):
    e = (np.asarray(c, np.float64) - gt)[mask]
    return -10.0 * math.log10(float(np.mean(e * e)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["human_object", "human_object_deform", "keyframes"])
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--rays", type=int, default=4096)
    ap.add_argument("--eval-every", type=int, default=250)
    ap.add_argument("--perturb", type=float, default=0.0,
                    help="move every warped position by U[-eps, eps] (seeded) per coordinate; "
                         "the curve file name gets a _perturbed suffix")
    ap.add_argument("--perturb-grad", type=float, default=0.0,
                    help="add an error of relative norm rel (seeded, uniform per non-zero entry) "
                         "to every gradient array before each Adam update; the curve file name "
                         "gets a _gradnoise suffix")
    ap.add_argument("--lr-decay", type=float, default=1.0,
                    help="update k uses lr * decay^(k-1); the key-frame curve file name "
                         "gets a _decay suffix when < 1")
    args = ap.parse_args()
    t0 = time.time()
    if args.which in ("human_object", "human_object_deform"):
        deform = args.which == "human_object_deform"
        work, st, o, d, C, D, ranges = human_object_state(deform)
        box = ((-1.0,) * 3, (1.0,) * 3)
        suffix = "_perturbed" if args.perturb > 0 else ("_gradnoise" if args.perturb_grad > 0 else "")
        adam = optim.Adam()
        if args.perturb_grad > 0:
            gnoise = np.random.default_rng(7)
            rel = args.perturb_grad

            class NoisyAdam(optim.Adam):
                def update(self, p, g, m, v, step, skip_zero=False):
                    nz = g != 0.0
                    if nz.any():
                        rms = math.sqrt(float(np.mean(g[nz] ** 2)))
                        u = gnoise.uniform(-math.sqrt(3.0), math.sqrt(3.0), size=np.shape(g))
                        g = np.where(nz, g + rel * rms * u, 0.0)
                    return super().update(p, g, m, v, step, skip_zero=skip_zero)

            adam = NoisyAdam()
        path = os.path.join(HERE, f"curve_{args.which}_r64{suffix}.txt")
        if args.perturb > 0:
            from oracle import warp as owarp
            noise = np.random.default_rng(5)
            orig = owarp.warp

            def noisy(x, *a, **k):
                out = orig(x, *a, **k)
                if k.get("want_cache"):       # the backward's own recomputation
                    return out
                return out + noise.uniform(-args.perturb, args.perturb, size=out.shape)

            owarp.warp = noisy
        rows = []
        for i in range(args.steps):
            r = ostep.train_step(work, st, o, d, C, D, ranges, box, adam=adam, apply=True)
            rows.append((i, r["loss"]))
            print(f"step {i} loss {r['loss']:.8f} ({time.time() - t0:.0f} s)", flush=True)
        with open(path, "w") as fh:
            fh.write("# FP64 oracle: two-field workload at 1/64 of its rays (3750 rays, human\n"
                     "# [0, 2812), object [2500, 3750)), one fixed batch, Adam lr 1e-2,\n"
                     "# colour + depth loss (Eq. 8, lambda_d = 1)"
                     f"{'; deformation network on the human field' if deform else ''}"
                     f"{f'; warped positions moved by U[-{args.perturb:g}, {args.perturb:g}]' if args.perturb > 0 else ''}"
                     f"{f'; gradient errors of relative norm {args.perturb_grad:g}' if args.perturb_grad > 0 else ''}.\n"
                     f"# written by: python tests/golden/make_curves.py {args.which} --steps {args.steps}"
                     f"{f' --perturb {args.perturb:g}' if args.perturb > 0 else ''}"
                     f"{f' --perturb-grad {args.perturb_grad:g}' if args.perturb_grad > 0 else ''}\n"
                     "# columns: step loss\n")
            for i, l in rows:
                fh.write(f"{i} {l:.10e}\n")
    else:
        work, f, scene, cams, st = keyframe_state()
        box = (f.aabb_min, f.aabb_max)
        eo, ed, egt, emask = synth.keyframe_eval_view(scene, box)
        decay = args.lr_decay < 1.0
        path = os.path.join(HERE, f"curve_keyframes_{args.rays}{'_decay' if decay else ''}.txt")
        adam = optim.Adam(lr_decay=args.lr_decay)
        rows = []
        for i in range(args.steps):
            o, d, C, D, M = synth.keyframe_batch(scene, cams, args.rays,
                                                 synth.keyframe_step_rng(work, i), box)
            r = ostep.train_step(work, st, o, d, C, D, [(0, args.rays)], adam=adam, apply=True,
                                 mask=M)
            p = float("nan")
            if (i + 1) % args.eval_every == 0:
                rc, _ = ostep.render(work, st, eo, ed, [(0, eo.shape[0])], t_stop=1e-4)
                p = psnr(rc, egt, emask)
            rows.append((i, r["loss"], p))
            print(f"step {i} loss {r['loss']:.8f} psnr {p:.4f} ({time.time() - t0:.0f} s)",
                  flush=True)
        with open(path, "w") as fh:
            fh.write("# FP64 oracle: key-frame refinement, rays drawn per step from eight\n"
                     f"# 1280x720 key frames of the analytic scene, {args.rays} rays per step,\n"
                     f"# Adam lr 1e-2 (times {args.lr_decay:.9g}^(k-1) at update k), masked colour\n"
                     "# + depth loss (Eq. 8, lambda_d = 1); PSNR over the in-box pixels of a\n"
                     "# 160x90 novel view (t_stop 1e-4) every "
                     f"{args.eval_every} steps (nan elsewhere).\n"
                     f"# written by: python tests/golden/make_curves.py keyframes --steps {args.steps} "
                     f"--rays {args.rays} --eval-every {args.eval_every}"
                     f"{f' --lr-decay {args.lr_decay!r}' if decay else ''}\n"
                     "# columns: step loss psnr_db\n")
            for i, l, p in rows:
                fh.write(f"{i} {l:.10e} {p:.6f}\n")
    print("wrote", path, f"in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
