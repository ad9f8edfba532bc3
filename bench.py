"""Throughput benchmark of the radiance-field training step on one MI355X.

Workload: the Instant-NGP-scale static object field (2^18 rays per step,
<= 128 samples per ray through a 128^3 occupancy bitfield with ~30 % of the
voxels set; hash grid L=16, F=2, T=2^19, N 16 -> 2048; density 32->64->16;
colour (16+16)->64->64->3).  Inputs are seeded synthetic data, resident in
HBM before timing.

A step is one whole pass of the hot path: march with occupancy skipping,
hash encode, density + colour networks, compositing, loss, backward through
all of them, Adam.  The headline is the fused bf16 step (fp16 tables with fp32
masters, MFMA networks, level-split encoder, captured HIP graph); the plain
fp32 step (one launch per stage, fp32 tables) is timed beside it, as is a
forward-only 1920x1080 render of the same field.  The dominant kernel is timed
alone with HIP events on the stream it runs on for the roofline figure, and
the FP64 oracle is timed on a bounded sample of the same workload on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(n_rays, seed_offset=0):
    import synth
    w = synth.config(2)
    f = w.fields[0]
    rng = synth.rng_for(w.seed + seed_offset)
    o, d = synth.sphere_rays(n_rays, rng)
    _, occ = synth.noise_occupancy(f.occ_res, rng)
    return w, f, rng, o, d, occ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--rays", type=int, default=1 << 18)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-render", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the human, two-field and key-frame configurations")
    ap.add_argument("--kf-train-steps", type=int, default=600)
    ap.add_argument("--only", choices=["human", "two_fields", "keyframes"],
                    help="run only this configuration (for profiling) and print its record")
    ap.add_argument("--cpu-rays", type=int, default=32768)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (byte-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(data-parallel sharding is described in the design notes); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2304_03184_amd import _lib as L, field as F, ops as O

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    L.lib()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    if args.only:
        fn = {"human": lambda: bench_human(O, L, F, torch, dev, args.steps, args.warmup),
              "two_fields": lambda: bench_two_fields(O, L, F, torch, dev, args.steps, args.warmup),
              "keyframes": lambda: bench_keyframes(O, L, F, torch, dev, args.steps, args.warmup,
                                                   args.kf_train_steps)}[args.only]
        print(json.dumps({"only": args.only, **fn()}), flush=True)
        return

    R = args.rays
    w, f, rng, o, d, occ = make_inputs(R)
    n_entries = O.grid_desc_of(f).n_entries
    table = synth.uniform_table(n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    Ct = synth.smooth_colour_targets(o, d, rng)
    cap = R * 48        # per-field sample capacity (observed ~25 kept samples per ray)
    o_d, d_d, C_d = dev(o), dev(d), dev(Ct)

    def timed_steps(precision, steps, warmup, graph):
        fld = F.Field(w, f, table, params, occ_words=occ)
        # the BF16 step tunes its launch shapes in its first (warm-up) step
        tr = F.Trainer([fld], R, cap, precision=precision, use_graph=graph,
                       autotune=precision == L.NVR_BF16)
        tr.set_batch(o_d, d_d, C_d)
        for _ in range(warmup):
            tr.step()
        torch.cuda.synchronize()
        n_samples = tr.sample_count()
        assert n_samples <= cap, "sample capacity overflow"
        t0 = time.perf_counter()
        for _ in range(steps):
            tr.step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        loss = float(tr.loss.item())
        return tr, fld, dt, n_samples, loss

    log(f"[bench] bf16 fused step: {R} rays, warmup {args.warmup}, steps {args.steps}")
    tr, fld, dt_bf, n_samp, loss_bf = timed_steps(L.NVR_BF16, args.steps, args.warmup, True)
    shape = tr.launch_shape(0)
    log(f"[bench] bf16 fused: {dt_bf * 1e3:.3f} ms/step, {n_samp} samples, loss {loss_bf:.5f}, "
        f"launch shape {shape}")

    # ---------------------------------------------------------------- dominant kernel
    # the level-split hash-grid scatter (encode backward) on this step's own samples
    roof = None
    try:
        roof = time_encode_kernels(O, L, torch, fld, w, f, o_d, d_d, occ, cap)
    except Exception as e:  # measurement is reported as missing, never invented
        log(f"[bench] roofline measurement failed: {e}")

    # ---------------------------------------------------------------- occupancy upkeep
    occupancy = None
    try:
        occupancy = time_occupancy(L, F, torch, w, f, table, params)
    except Exception as e:  # measurement is reported as missing, never invented
        log(f"[bench] occupancy update measurement failed: {e}")

    # ---------------------------------------------------------------- live look-up table
    live_lut = None
    try:
        live_lut = [time_live_lut(O, torch), time_live_lut(O, torch, res=512, k=4)]
    except Exception as e:  # measurement is reported as missing, never invented
        log(f"[bench] live look-up table measurement failed: {e}")

    # ---------------------------------------------------------------- deformation network
    deform = None
    try:
        deform = time_deform(O, L, torch)
    except Exception as e:  # measurement is reported as missing, never invented
        log(f"[bench] deformation network measurement failed: {e}")

    # ---------------------------------------------------------------- key-frame selection
    keyframe = None
    try:
        keyframe = time_keyframe(O, torch)
    except Exception as e:  # measurement is reported as missing, never invented
        log(f"[bench] key-frame measurement failed: {e}")

    # ---------------------------------------------------------------- render
    render = None
    if not args.no_render:
        render = time_render(O, L, F, torch, w, f, table, params, occ, dev)

    tr.close()

    # ---------------------------------------------------------------- other configurations
    extra = {}
    if not args.no_extra:
        for name, fn in (("human_warp", lambda: bench_human(O, L, F, torch, dev, 10, 3)),
                         ("two_fields", lambda: bench_two_fields(O, L, F, torch, dev, 10, 3)),
                         ("keyframes", lambda: bench_keyframes(O, L, F, torch, dev, 10, 3,
                                                               args.kf_train_steps))):
            try:
                extra[name] = fn()
            except Exception as e:  # reported as missing, never invented
                log(f"[bench] {name} failed: {e}")
                extra[name] = {"error": str(e)}

    log(f"[bench] fp32 plain step: {args.plain_steps} steps")
    tr32, _, dt_32, n32, loss_32 = timed_steps(L.NVR_F32, args.plain_steps, 1, False)
    tr32.close()
    log(f"[bench] fp32 plain: {dt_32 * 1e3:.3f} ms/step")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_rays)

    out = {
        "metric": "training rays/s (fwd+bwd) & render Mpix/s, BF16 fused vs FP32 plain",
        "value": R / dt_bf,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_bf * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded rays, occupancy, tables, weights, targets)",
        "config": {"workload": w.name, "rays_per_step": R, "samples_per_step": n_samp,
                   "levels": f.n_levels, "log2_table": f.log2_table, "res": [f.res_min, f.res_max],
                   "occupancy": f"{f.occ_res}^3 noise, 30% set", "graph": True,
                   "launch_shape": dict(zip(["gather_chunks", "mlp_fwd_blocks", "mlp_bwd_blocks",
                                             "emit_chunks", "composite_blocks", "tuned",
                                             "emit_chunk_samples"], shape))},
        "fp32_plain": {"rays_per_s": R / dt_32, "ms_per_step": dt_32 * 1e3,
                       "speedup_bf16_over_fp32": dt_32 / dt_bf, "loss": loss_32},
        "render": render,
        "configs": extra,
        "occupancy_update": occupancy,
        "live_lut": live_lut,
        "keyframe": keyframe,
        "deform": deform,
        "roofline": roof,
        "step_roofline": step_roofline(f, R, n_samp, n_entries,
                                       sum(a * b for a, b in f.layer_shapes()), dt_bf),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


MFMA_PEAK_FLOPS = 2.5e15    # dense fp16 / bf16 MFMA


def step_roofline(f, R, n, n_entries, n_params, t_step):
    """Step time if every stage ran at its own bound (HBM bytes at 8 TB/s or
    MFMA flops at 2.5 PFLOP/s, whichever is longer), from per-unit algorithmic
    figures; the measured step is reported as a fraction of it."""
    L_ = f.n_levels
    fwd_flop = sum(2 * a * b for a, b in f.layer_shapes())   # one forward, unpadded
    stages = {   # name: (bytes, flops)
        "march": (24 * n + 28 * R, 0),                        # t, dt, x, ray id; rays in
        "gather": ((12 + L_ * 8 * 4 + 2 * 2 * L_) * n, 0),    # 588 B / sample at L = 16
        "mlp_fwd": ((4 * L_ + 16) * n, fwd_flop * n),         # fp16 features in, sigma + rgb out
        "composite_loss": (40 * n + 40 * R, 10 * n),
        "mlp_bwd": ((4 * L_ + 16 + 8 * L_) * n, 3 * fwd_flop * n),  # recompute + dX + dW
        "scatter": ((12 + 8 * L_ + L_ * 8 * 2 * 4) * n, 0),   # 1164 B / sample at L = 16
        "adam": (34 * (2 * n_entries + n_params), 0),
    }
    out, total = {}, 0.0
    for k, (by, fl) in stages.items():
        t = max(by / (HBM_PEAK_GBS * 1e9), fl / MFMA_PEAK_FLOPS)
        out[k] = {"bytes": by, "flops": fl, "ms": t * 1e3}
        total += t
    return {"rays_per_s": R / total, "ms_per_step": total * 1e3,
            "measured_frac": total / t_step, "stages": out}


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "binned_scatter_object_2p18_traffic.json")
SCATTER_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2304_03184_amd",
                           "csrc", "scatter.hip")


def measured_traffic():
    """HBM bytes per call of the binned scatter from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs recorded under profiles/ (scaled by the same counters on a
    copy of known size); None once scatter.hip differs from the source the
    counters were taken on."""
    import hashlib
    import json as _json
    try:
        rec = _json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha1(open(SCATTER_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("scatter_hip_sha1") != sha:
        return None
    return rec["hbm_bytes_per_call"]


def calibrate_copy(torch, gib=1):
    """A plain device copy of known size (gib GiB read + gib GiB written), three
    times, for scaling the HBM byte counters."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copied {gib} GiB three times")


def time_encode_kernels(O, L, torch, fld, w, f, o_d, d_d, occ, cap):
    """Times the hash-grid kernels alone with HIP events on the current stream,
    on this workload's own samples.  The roofline entry is the binned
    table-gradient scatter with feature gradients in the level-group layout the
    step keeps them in (count, scan, tile-bucketed append, per-tile LDS sum,
    split-tile reduce; in the step the gather forms the counts instead).  Beside
    it: the same call on row-major gradients (regrouped first), the level-split
    gather in both layouts, and the random-gather probe at the table's own
    footprint, the practical ceiling of the gather."""
    import ctypes as C
    md = O.march_desc_of(w, f)
    m = O.march(md, o_d, d_d, fld.occ, capacity=cap)
    n = m["n"]
    x = m["x"].contiguous()
    g = fld.grid
    L_ = f.n_levels
    lpg = (L_ + 7) // 8
    rng = np.random.default_rng(5)
    dfeat = torch.from_numpy(rng.normal(size=(n, 2 * L_)).astype(np.float32) * 1e-3).cuda()
    dgrp = torch.zeros((8, n, 2 * lpg), dtype=torch.float32, device="cuda")
    for l in range(L_):
        dgrp[l % 8, :, 2 * (l // 8):2 * (l // 8) + 2] = dfeat[:, 2 * l:2 * l + 2]
    dtab = torch.zeros_like(fld.table)
    nb = L.lib().nvr_encode_bwd_workspace(C.byref(g), n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    feat_g = torch.empty((8, n, 2 * lpg), dtype=torch.float16, device="cuda")
    probe_out = torch.empty((8, n), dtype=torch.int32, device="cuda")
    th = fld.table_half

    def bwd_grouped():
        L.call("nvr_encode_bwd_binned_grouped", C.byref(g), n, O._p(x), O._p(th), O._p(dgrp),
               O._p(dtab), None, O._p(ws), O._stream())

    def bwd_rowmajor():
        L.call("nvr_encode_bwd_binned", C.byref(g), n, O._p(x), O._p(th), O._p(dfeat),
               O._p(dtab), None, O._p(ws), O._stream())

    def fwd_grouped():
        L.call("nvr_encode_fwd_grouped", C.byref(g), n, O._p(x), O._p(th), O._p(feat_g),
               O._stream())

    def fwd_rowmajor():
        O.encode_fwd(g, x, th, torch.float16)

    def probe():
        L.call("nvr_probe_gather", O._p(th), th.numel() * th.element_size(), n, 4 * lpg, 1,
               O._p(probe_out), O._stream())

    def timed(fn, reps=10):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_bwd = timed(bwd_grouped)
    t_bwd_rm = timed(bwd_rowmajor)
    t_fwd = timed(fwd_grouped)
    t_fwd_rm = timed(fwd_rowmajor)
    t_probe = timed(probe)
    # algorithmic bytes per sample (per-unit figures of the scatter and gather):
    #   backward: position 12 B + dfeat 2L x 4 B + L x 8 corners x F=2 fp32 gradient
    #             contributions of 4 B (the 1,024 B / sample table-gradient RMW at L = 16)
    #   forward:  position 12 B + L x 8 corners x 4 B (fp16 x 2) + 2L fp16 features
    bwd_bpu = 12 + 4 * 2 * L_ + L_ * 8 * 2 * 4
    fwd_bpu = 12 + L_ * 8 * 4 + 2 * 2 * L_
    log(f"[bench] binned scatter {t_bwd * 1e3:.3f} ms (row-major gradients "
        f"{t_bwd_rm * 1e3:.3f} ms), gather {t_fwd * 1e3:.3f} ms (row-major "
        f"{t_fwd_rm * 1e3:.3f} ms), random-gather probe {t_probe * 1e3:.3f} ms over {n} samples")
    achieved = bwd_bpu * n / t_bwd / 1e9
    loads = 8 * n * 4 * lpg   # 16-byte probe loads: 4 per level, every level group
    return {"kernel": "hash-grid backward: binned table-gradient scatter, gradients in the "
                      "level-group layout (nvr_encode_bwd_binned_grouped: zero_u32 + "
                      "scatter_count + scatter_scan + scatter_emit + scatter_accum + "
                      "scatter_reduce)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "samples_per_launch": n, "bytes_per_sample": bwd_bpu,
            "avg_launch_ms": t_bwd * 1e3,
            "row_major_call": {"entry": "nvr_encode_bwd_binned (adds scatter_planarize)",
                               "avg_launch_ms": t_bwd_rm * 1e3,
                               "achieved_GBs": bwd_bpu * n / t_bwd_rm / 1e9},
            "encode_fwd": {"kernel": "encode_fwd_split (level-split gather, fp16 table, fp16 "
                                     "features in the level-group layout; "
                                     "nvr_encode_fwd_grouped)",
                           "avg_launch_ms": t_fwd * 1e3, "bytes_per_sample": fwd_bpu,
                           "achieved_GBs": fwd_bpu * n / t_fwd / 1e9,
                           "frac": fwd_bpu * n / t_fwd / 1e9 / HBM_PEAK_GBS,
                           "row_major_ms": t_fwd_rm * 1e3,
                           "gather_probe": {
                               "what": "random aligned 16-byte loads over the same fp16 table "
                                       "split into 8 XCD slices, as many as the gather's "
                                       "x-edge loads (4 per level per sample)",
                               "avg_launch_ms": t_probe * 1e3,
                               "loads_per_s": loads / t_probe,
                               "GBs_16B": loads * 16 / t_probe / 1e9,
                               "gather_frac_of_probe": t_probe / t_fwd}}}


def time_occupancy(L, F, torch, w, f, table, params, m=1 << 19):
    """One occupancy-grid update of the field (128^3 density grid, m probes at
    random cells, BF16 path), timed with HIP events on the current stream."""
    res = f.occ_res
    n = res ** 3
    rng = np.random.default_rng(31)
    cells = rng.integers(0, n, size=m).astype(np.int32)
    v = np.stack([cells % res, (cells // res) % res, cells // (res * res)], 1)
    lo, hi = np.asarray(f.aabb_min, np.float64), np.asarray(f.aabb_max, np.float64)
    pts = (lo + (v + rng.uniform(size=(m, 3))) * (hi - lo) / res).astype(np.float32)
    fld = F.Field(w, f, table, params)
    grid = torch.from_numpy(rng.uniform(0, 2, size=n).astype(np.float32)).cuda()
    bits = torch.zeros((n + 31) // 32, dtype=torch.int32, device="cuda")
    c_d, p_d = torch.from_numpy(cells).cuda(), torch.from_numpy(pts).cuda()
    for _ in range(3):
        F.occupancy_update(fld, L.NVR_BF16, c_d, p_d, grid, bits)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    reps = 10
    e0.record()
    for _ in range(reps):
        F.occupancy_update(fld, L.NVR_BF16, c_d, p_d, grid, bits)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    # algorithmic bytes: the grid read and written once and the bitfield written
    # (8 B + 1/8 B per cell); per probe its cell and position (16 B), the
    # gather's 16 levels x 8 corners x 4 B and the grid update (8 B)
    by = n * (8 + 1 / 8) + m * (16 + f.n_levels * 8 * 4 + 8)
    log(f"[bench] occupancy update: {t * 1e3:.3f} ms ({m} probes, {n} cells)")
    return {"cells": n, "probes": m, "precision": "bf16", "ms": t * 1e3,
            "bytes_per_update": by, "achieved_GBs": by / t / 1e9,
            "ms_per_step_if_every_16_steps": t * 1e3 / 16}


def time_live_lut(O, torch, res=128, k=8, knn_res=128):
    """Live look-up table of the human field's neighbour search: res^3 canonical
    and live voxels, k of the rig's 1024 nodes listed per voxel, timed with HIP
    events on the current stream.  The canonical KNN field is computed at
    knn_res^3 (the k nodes nearest each voxel centre) and, for a finer res,
    repeated over the res / knn_res finer voxels of each cell."""
    import synth
    from scipy.spatial import cKDTree
    rig = synth.human_rig(np.random.default_rng(33), knn_res=8)
    canon, dq = rig["node_canon"], rig["node_dq"][0]
    g = (np.arange(knn_res) + 0.5) / knn_res * 2.0 - 1.0
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    centres = np.stack([xx, yy, zz], -1).reshape(-1, 3)
    _, ids = cKDTree(canon.astype(np.float64)).query(centres, k=k)
    knn = torch.from_numpy(ids.astype(np.uint16).view(np.int16)).cuda()
    if res != knn_res:
        s = res // knn_res
        knn = knn.view(knn_res, 1, knn_res, 1, knn_res, 1, k).expand(
            knn_res, s, knn_res, s, knn_res, s, k).reshape(res ** 3, k)
    c_d, q_d = torch.from_numpy(canon).cuda(), torch.from_numpy(dq).cuda()
    box = ((-1.0,) * 3, (1.0,) * 3)
    for _ in range(3):
        lut = O.live_lut(knn, c_d, q_d, box, res, box, res)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    reps = 20 if res <= 128 else 5
    e0.record()
    for _ in range(reps):
        lut = O.live_lut(knn, c_d, q_d, box, res, box, res)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    n = res ** 3
    filled = float((lut >= 0).float().mean().item())
    del knn, lut
    # algorithmic bytes: the KNN field read once (2 k B per canonical voxel), the
    # table filled and then updated once per carried voxel (8 B per voxel); the
    # node data (1024 x 44 B) stays in cache
    by = n * (2 * k + 8)
    log(f"[bench] live look-up table {res}^3, {k} nodes: {t * 1e6:.1f} us ({filled:.2f} filled)")
    return {"canon_res": res, "live_res": res, "k_nodes": k, "n_nodes": len(canon),
            "knn_res": knn_res, "us": t * 1e6, "filled": filled, "bytes": by,
            "achieved_GBs": by / t / 1e9, "voxels_per_s": n / t}


def time_deform(O, L, torch, n=1 << 18):
    """Pose-conditioned deformation network on n points (the field's ladder for
    its own 2^19-entry table, 104 -> 4 x 128 -> 3) through the public entry
    points, forward and backward (which runs the forward first), float32 tiled
    kernels and matrix cores, timed with HIP events."""
    import ctypes as C
    rng = np.random.default_rng(37)
    g = L.GridDesc()
    L.call("nvr_grid_init", C.byref(g), 16, 2, 19, 16, 2048, (C.c_float * 3)(-1, -1, -1),
           (C.c_float * 3)(1, 1, 1))
    n_entries = int(g.offset[16])
    table = torch.from_numpy(rng.uniform(-0.1, 0.1, size=(n_entries, 2)).astype(np.float32)).cuda()
    n_par = int(L.lib().nvr_deform_param_count())
    params = (torch.rand(n_par, device="cuda") * 2 - 1) * 0.1
    x = torch.from_numpy(rng.uniform(-0.9, 0.9, size=(n, 3)).astype(np.float32)).cuda()
    theta = torch.randn(72, device="cuda") * 0.3
    dvc = torch.randn((n, 3), device="cuda")

    def timed(fn, reps=10):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    flops_fwd = 2.0 * n * n_par
    out = {"points": n}
    for name, math in (("f32_tiled", L.NVR_F32), ("f16_matrix_cores", L.NVR_F16)):
        fwd = timed(lambda: O.deform_fwd(g, x, theta, table, params, math=math))
        bwd = timed(lambda: O.deform_bwd(g, x, theta, table, params, dvc, math=math))
        # the backward recomputes the forward: 3 x the forward's products
        out[name] = {"fwd_ms": fwd, "bwd_ms": bwd,
                     "fwd_tflops": flops_fwd / (fwd * 1e-3) / 1e12,
                     "bwd_tflops": 3 * flops_fwd / (bwd * 1e-3) / 1e12}
        log(f"[bench] deformation net {n} points ({name}): fwd {fwd:.3f} ms, "
            f"bwd {bwd:.3f} ms")
    return out


def time_keyframe(O, torch):
    """Key-frame selection kernels and the depth-test assembly, timed with HIP
    events on the current stream: Eq. 5 visibility of 1024 nodes against a
    640x576 depth map for one frame and for a full pool of 100 frames, Eq. 6
    of a query against 100 pooled frames, the assembly of two 1920x1080
    renderings."""
    import synth
    rng = np.random.default_rng(35)
    F, M, H, W, fl = 100, 1024, 576, 640, 500.0
    P = []
    for R, c in synth.look_at_cameras(F, radius=2.0, arc_deg=180.0):
        K = np.array([[fl, 0.0, W / 2], [0.0, -fl, H / 2], [0.0, 0.0, 1.0]])
        P.append(K @ np.concatenate([R.T, (-R.T @ c)[:, None]], 1))
    P = torch.from_numpy(np.stack(P).astype(np.float32)).cuda()
    X = torch.from_numpy(rng.uniform(-0.8, 0.8, size=(F, M, 3)).astype(np.float32)).cuda()
    D = torch.from_numpy(rng.uniform(1.0, 3.0, size=(F, H, W)).astype(np.float32)).cuda()
    theta = torch.randn((F, 72), device="cuda") * 0.3
    beta = torch.full((72,), 0.02, device="cuda")
    t = torch.arange(F, dtype=torch.int32, device="cuda")
    bits = O.visibility(X, P, D)
    n_pix = 1920 * 1080
    g = torch.Generator(device="cuda").manual_seed(36)
    ca, cb = (torch.rand((n_pix, 3), device="cuda", generator=g) for _ in range(2))
    aa, ab = (torch.rand(n_pix, device="cuda", generator=g) for _ in range(2))
    da, db = aa * 2.0, ab * 1.5

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    out = {
        "visibility_1_frame_us": timed(lambda: O.visibility(X[:1], P[:1], D[:1])),
        "visibility_100_frames_us": timed(lambda: O.visibility(X, P, D)),
        "human_distance_pool_100_us": timed(
            lambda: O.human_distance(theta, bits, t, theta[0], bits[0], 7, beta)),
        "assemble_1080p_us": timed(lambda: O.depth_assemble(ca, da, aa, cb, db, ab)),
        "nodes": M, "depth_map": [W, H], "pool": F,
    }
    # the assembly reads 2 x 20 B and writes 16 B per pixel
    out["assemble_GBs"] = n_pix * 56 / (out["assemble_1080p_us"] * 1e-6) / 1e9
    log(f"[bench] key-frame: visibility {out['visibility_1_frame_us']:.1f} us (1 frame), "
        f"{out['visibility_100_frames_us']:.1f} us (100), distances "
        f"{out['human_distance_pool_100_us']:.1f} us, assembly {out['assemble_1080p_us']:.1f} us")
    return out


def time_render(O, L, F, torch, w, f, table, params, occ, dev):
    """Forward-only 1920x1080 render of the field (128 samples max, t_stop 1e-4)."""
    import synth
    (Rm, c), = synth.look_at_cameras(1, radius=2.0)[:1]
    o, d = synth.pixel_rays(Rm, c, 1920, 1080, 1500.0)
    fld = F.Field(w, f, table, params, occ_words=occ)
    tr = F.Trainer([fld], o.shape[0], 1 << 26, precision=L.NVR_BF16)
    od, dd = dev(o), dev(d)
    for _ in range(2):
        tr.render(od, dd, t_stop=1e-4)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        tr.render(od, dd, t_stop=1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    tr.close()
    mpix = 1920 * 1080 / dt / 1e6
    log(f"[bench] render 1920x1080: {dt * 1e3:.3f} ms, {mpix:.1f} Mpix/s")
    return {"resolution": [1920, 1080], "ms_per_frame": dt * 1e3, "mpix_per_s": mpix,
            "t_stop": 1e-4, "dtype": "bf16"}


def _f16(a):
    return np.asarray(a, np.float32).astype(np.float16).astype(np.float64)


def _timed(torch, tr, steps, warmup):
    for _ in range(warmup):
        tr.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _deform_state(fl):
    """The oracle's copy of a field's deformation network (the fp16 table copy
    and the fp16-rounded weights the matrix-core forward reads)."""
    from oracle import grid as ogrid, step as ostep
    D = fl.deform
    if D is None:
        return None
    return ostep.DeformState(ogrid.Layout.from_field(fl.fcfg), D.theta.cpu().numpy(),
                             D.table_half.float().cpu().numpy(), _f16(D.params.cpu().numpy()))


def _sampled_colour_error(torch, tr, flds, w, o, d, ranges, pick, box=None):
    """Forward colours / depths of the picked rays after training vs the FP64
    oracle given the same fp16 tables and fp16-rounded weights."""
    from oracle import step as ostep
    R = o.shape[0]
    Cg = torch.empty((R, 3), device="cuda")
    Dg = torch.empty(R, device="cuda")
    tr.forward(C_out=Cg, D_out=Dg)
    torch.cuda.synchronize()
    states = [ostep.FieldState(fl.fcfg, fl.table_half.float().cpu().numpy().astype(np.float64),
                               _f16(fl.params.cpu().numpy()),
                               occ_words=fl.occ.cpu().numpy().view(np.uint32)
                               if fl.occ is not None else None,
                               rig=getattr(fl, "rig_np", None),
                               deform=_deform_state(fl)) for fl in flds]
    sub = []
    for lo, hi in ranges:   # each field's rays among the picked (sorted) ones
        idx = np.nonzero((pick >= lo) & (pick < hi))[0]
        sub.append((int(idx[0]), int(idx[-1]) + 1) if idx.size else (0, 0))
    ref = ostep.forward_all(w, ostep.StepState(states), o[pick], d[pick], sub, box)
    ec = float(np.abs(Cg.cpu().numpy()[pick] - ref["C"]).max())
    ed = float(np.abs(Dg.cpu().numpy()[pick] - ref["D"]).max())
    return ec, ed


def _human_step(O, L, F, torch, dev, steps, warmup, with_deform):
    import synth
    w, f, rig, o, d, Ct, occ, rng = synth.human_workload()
    g = O.grid_desc_of(f)
    table = synth.uniform_table(g.n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    D = None
    if with_deform:
        # the deformation network's own encoding on the field's ladder
        theta, dtab, dpar = synth.deform_inputs(g.n_entries, synth.rng_for(w.seed + 90))
        D = F.Deform(O.grid_desc_of(f), theta, dtab, dpar)
    R, ex = w.n_rays, w.extra
    wd = O.warp_desc(n_nodes=ex["n_nodes"], k_nodes=ex["k_nodes"], lut_res=ex["knn_res"])
    fld = F.Field(w, f, table, params, occ_words=occ, rig=O.Rig.from_numpy(rig), warp_desc=wd,
                  deform=D)
    fld.rig_np = rig
    cap = R * 64
    tr = F.Trainer([fld], R, cap, precision=L.NVR_BF16, use_graph=True, autotune=True)
    tr.set_batch(dev(o), dev(d), dev(Ct))
    dt = _timed(torch, tr, steps, warmup)
    n = tr.sample_count()
    assert n <= cap, "sample capacity overflow"
    pick = np.sort(synth.rng_for(31).choice(R, size=64, replace=False))
    ec, ed = _sampled_colour_error(torch, tr, [fld], w, o, d, [(0, R)], pick,
                                   ((-1.0,) * 3, (1.0,) * 3))
    tr.close()
    assert ec < 2e-2 and ed < 2e-2, f"human field: sampled colour error {ec}, depth {ed}"
    return w, dt, n, ec, ed, pick


def bench_human(O, L, F, torch, dev, steps, warmup):
    """The human field behind the hybrid deformation at full size (2^18 rays,
    24 joints, 1024 nodes listed 8 per voxel of a 128^3 look-up, then the
    pose-conditioned deformation network on its own hash grid), fused BF16 step
    in a captured graph with tuned shapes; the same step without the network
    beside it; sampled parity after training."""
    w, dt, n, ec, ed, pick = _human_step(O, L, F, torch, dev, steps, warmup, True)
    _, dt0, n0, ec0, ed0, _ = _human_step(O, L, F, torch, dev, steps, warmup, False)
    R, ex = w.n_rays, w.extra
    log(f"[bench] human field (warp + deformation network): {dt * 1e3:.3f} ms/step, {n} samples, "
        f"sampled C err {ec:.2e}; warp only {dt0 * 1e3:.3f} ms/step")
    return {"workload": w.name, "rays_per_step": R, "samples_per_step": n,
            "ms_per_step": dt * 1e3, "rays_per_s": R / dt, "nodes": ex["n_nodes"],
            "joints": ex["n_joints"], "lut_res": ex["knn_res"], "graph": True,
            "deformation_network": "104 -> 4 x 128 -> 3, matrix cores, own 16-level grid",
            "warp_only": {"ms_per_step": dt0 * 1e3, "rays_per_s": R / dt0,
                          "samples_per_step": n0, "colour_max_abs": ec0},
            "sampled_parity": {"rays": int(pick.size), "colour_max_abs": ec, "depth_max_abs": ed,
                               "bar": 2e-2}}


def bench_two_fields(O, L, F, torch, dev, steps, warmup):
    """Human + object fields at full size (180k / 80k rays, 20k shared rays
    composited over the t-merged samples of both), colour + depth loss, one
    captured BF16 graph step with tuned shapes; sampled parity after training."""
    import synth
    w, (fh, fo), rig, o, d, C, D, ranges, (occ_h, occ_o), rng = \
        synth.two_field_workload(scale=1.0)
    table_h = synth.uniform_table(O.grid_desc_of(fh).n_entries, 2, rng)
    params_h = synth.xavier_params(fh.layer_shapes(), rng)
    table_o = synth.uniform_table(O.grid_desc_of(fo).n_entries, 2, rng)
    params_o = synth.xavier_params(fo.layer_shapes(), rng)
    ex = w.extra
    wd = O.warp_desc(n_nodes=ex["n_nodes"], k_nodes=ex["k_nodes"], lut_res=ex["knn_res"])
    fld_h = F.Field(w, fh, table_h, params_h, occ_words=occ_h, rig=O.Rig.from_numpy(rig),
                    warp_desc=wd, ray_range=ranges[0])
    fld_h.rig_np = rig
    fld_o = F.Field(w, fo, table_o, params_o, occ_words=occ_o, ray_range=ranges[1])
    R = w.n_rays
    cap = 180000 * 64
    tr = F.Trainer([fld_h, fld_o], R, cap, precision=L.NVR_BF16, lambda_depth=w.lambda_depth,
                   use_graph=True, autotune=True)
    tr.set_batch(dev(o), dev(d), dev(C), dev(D))
    dt = _timed(torch, tr, steps, warmup)
    nh, no = tr.sample_count(0), tr.sample_count(1)
    assert nh <= cap and no <= cap, "sample capacity overflow"
    g = synth.rng_for(32)
    pick = np.sort(np.concatenate([g.choice(ex["human_only"], 24, replace=False),
                                   ex["human_only"] + g.choice(ex["shared"], 24, replace=False),
                                   ranges[0][1] + g.choice(ex["object_only"], 16, replace=False)]))
    ec, ed = _sampled_colour_error(torch, tr, [fld_h, fld_o], w, o, d, ranges, pick,
                                   ((-1.0,) * 3, (1.0,) * 3))
    tr.close()
    assert ec < 2e-2 and ed < 2e-2, f"two fields: sampled colour error {ec}, depth {ed}"
    log(f"[bench] two fields: {dt * 1e3:.3f} ms/step, {nh} + {no} samples, "
        f"sampled C err {ec:.2e}")
    return {"workload": w.name, "rays_per_step": R, "rays": {"human": ranges[0][1],
            "object": R - ranges[1][0], "shared": ex["shared"]},
            "samples_per_step": {"human": nh, "object": no}, "ms_per_step": dt * 1e3,
            "rays_per_s": R / dt, "loss": "colour + depth (lambda_d = 1)", "graph": True,
            "sampled_parity": {"rays": int(pick.size), "colour_max_abs": ec, "depth_max_abs": ed,
                               "bar": 2e-2}}


def bench_keyframes(O, L, F, torch, dev, steps, warmup, train_steps):
    """Key-frame refinement at full size: 2^20 rays per step drawn over eight
    1280x720 RGB-D key frames, fused BF16 step (captured graph, tuned shapes);
    then `train_steps` steps on that batch and a forward-only 1920x1080 novel
    view of the trained field with early termination at T < 1e-4."""
    import synth
    from oracle import step as ostep
    work, f, scene, cams, occ, rng = synth.keyframe_workload()
    table = synth.uniform_table(O.grid_desc_of(f).n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    box = (f.aabb_min, f.aabb_max)
    R = work.n_rays
    o, d, C, D, M = synth.keyframe_batch(scene, cams, R, synth.keyframe_step_rng(work, 0), box)
    fld = F.Field(work, f, table, params, occ_words=occ)
    cap = R * 16
    tr = F.Trainer([fld], R, cap, precision=L.NVR_BF16, lambda_depth=work.lambda_depth,
                   use_graph=True, autotune=True)
    tr.set_batch(dev(o), dev(d), dev(C), dev(D), dev(M))
    dt = _timed(torch, tr, steps, warmup)
    n = tr.sample_count()
    assert n <= cap, "sample capacity overflow"
    for _ in range(train_steps):
        tr.step()
    loss = float(tr.loss.item())
    # the novel view between key frames, full HD
    W, H, fx = work.extra["render_w"], work.extra["render_h"], 1500.0
    eo, ed_, egt, emask = synth.keyframe_eval_view(scene, box, w=W, h=H, f=fx)
    eo_d, ed_d = dev(eo), dev(ed_)
    rgb, depth = tr.render(eo_d, ed_d, t_stop=work.extra["t_stop"])
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        tr.render(eo_d, ed_d, t_stop=work.extra["t_stop"])
    torch.cuda.synchronize()
    dt_r = (time.perf_counter() - t0) / reps
    img = rgb.cpu().numpy()
    e = (img.astype(np.float64) - egt)[emask]
    psnr = -10.0 * math.log10(float(np.mean(e * e)))
    # early termination: samples the marcher keeps vs samples composited
    md = O.march_desc_of(work, f)
    mk = O.march(md, eo_d, ed_d, fld.occ, capacity=eo.shape[0] * 48)
    marched = mk["n"]
    # sampled parity of the render (oracle on the same fp16 table, rounded weights)
    pick = np.sort(synth.rng_for(33).choice(np.nonzero(emask)[0], size=64, replace=False))
    st = ostep.StepState([ostep.FieldState(f, fld.table_half.float().cpu().numpy()
                                           .astype(np.float64), _f16(fld.params.cpu().numpy()),
                                           occ_words=occ)])
    rC, rD = ostep.render(work, st, eo[pick], ed_[pick], [(0, pick.size)],
                          t_stop=work.extra["t_stop"])
    wts = ostep.forward_all(work, st, eo[pick], ed_[pick], [(0, pick.size)],
                            t_stop=work.extra["t_stop"])["w"]
    kept = int(np.count_nonzero(wts))
    full = int(ostep.forward_all(work, st, eo[pick], ed_[pick], [(0, pick.size)])["w"].size)
    ec = float(np.abs(img[pick] - rC).max())
    tr.close()
    assert ec < 2e-2, f"key-frame render: sampled colour error {ec}"
    log(f"[bench] key frames: {dt * 1e3:.3f} ms/step ({n} samples); 1080p render "
        f"{dt_r * 1e3:.3f} ms, PSNR {psnr:.2f} dB after {warmup + steps + train_steps} steps")
    return {"workload": work.name, "rays_per_step": R, "samples_per_step": n,
            "ms_per_step": dt * 1e3, "rays_per_s": R / dt, "graph": True,
            "render": {"resolution": [W, H], "ms_per_frame": dt_r * 1e3,
                       "mpix_per_s": W * H / dt_r / 1e6, "t_stop": work.extra["t_stop"],
                       "trained_steps": warmup + steps + train_steps, "loss": loss,
                       "psnr_db_in_box": psnr, "marched_samples": marched,
                       "sampled_rays_composited_fraction": kept / max(full, 1),
                       "sampled_parity": {"rays": int(pick.size), "colour_max_abs": ec,
                                          "bar": 2e-2}}}


def cpu_baseline(n_rays):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    one training step (fwd + bwd + Adam) over n_rays rays of the same field."""
    import synth
    from oracle import grid as ogrid, step as ostep
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    w, f, rng, o, d, occ = make_inputs(n_rays, seed_offset=11)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    Ct = synth.smooth_colour_targets(o, d, rng)
    st = ostep.StepState([ostep.FieldState(f, table, params, occ_words=occ)])
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        t0 = time.perf_counter()
        ostep.train_step(w, st, o, d, Ct, None, [(0, n_rays)])
        dt = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    log(f"[bench] oracle step on {n_rays} rays: {dt:.2f} s")
    return {"value": n_rays / dt, "unit": "rays/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 training step (fwd+bwd+Adam) over {n_rays} rays of the same "
                      f"workload (full-size tables and networks), single thread, "
                      f"{dt:.1f} s",
            "host": {"cpu": host_cpu(), "nproc": os.cpu_count(), "blas_threads": 1}}


def host_cpu():
    """CPU model name of this host (from /proc/cpuinfo), or the platform string."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


if __name__ == "__main__":
    main()
