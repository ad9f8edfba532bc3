"""Whole-step parity of the HIP training step and renderer against the FP64 oracle."""
import copy

import numpy as np
import pytest

import synth
from oracle import march as omarch, composite as ocomp, grid as ogrid, network as onet, sh as osh
from oracle import step as ostep, warp as owarp

from helpers import bf16_round, decided_rays, dev, f16_round, field_inputs, host, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def lib():
    from paper_2304_03184_amd import _lib, field, ops
    return _lib, field, ops


def run_step(fields, n_rays, cap, o, d, Ct, Dt=None, precision=0, lam=0.0, apply=False,
             graph=False, deterministic=False):
    L, F, O = lib()
    tr = F.Trainer(fields, n_rays, cap, precision=precision, lambda_depth=lam, use_graph=graph,
                   deterministic=deterministic)
    tr.set_batch(dev(o), dev(d), dev(Ct), None if Dt is None else dev(Dt))
    Cg = torch.empty((n_rays, 3), device="cuda")
    Dg = torch.empty(n_rays, device="cuda")
    loss = tr.forward(C_out=Cg, D_out=Dg)
    tr.backward(apply_update=apply)
    torch.cuda.synchronize()
    return tr, float(loss.item()), host(Cg), host(Dg)


def test_cfg1_fp32_step_matches_oracle():
    I = field_inputs(1, 1024)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    fld = F.Field(w, f, I["table"], I["params"])
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 64, I["o"], I["d"], I["Ct"])
    st = ostep.StepState([ostep.FieldState(f, I["table"], I["params"])])
    ref = ostep.train_step(w, st, I["o"], I["d"], I["Ct"], None, [(0, w.n_rays)], apply=False)
    assert tr.sample_count() == w.n_rays * 64
    np.testing.assert_allclose(Cg, ref["C"], rtol=0, atol=1e-5)
    np.testing.assert_allclose(Dg, ref["D"], rtol=0, atol=1e-5)
    assert abs(loss - ref["loss"]) < 1e-5 * ref["loss"]
    g = ref["grads"][0]
    assert rel_err(host(fld.params_grad), g["params"]) < 1e-4
    assert rel_err(host(fld.table_grad), g["table"]) < 1e-4
    gt = host(fld.table_grad)
    assert np.max(np.abs(gt - g["table"])) <= 1e-4 * np.max(np.abs(g["table"]))
    tr.close()


def test_cfg1_fp32_update_matches_oracle_adam():
    I = field_inputs(1, 256, seed_offset=3)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    fld = F.Field(w, f, I["table"], I["params"])
    tr = F.Trainer([fld], w.n_rays, w.n_rays * 64, precision=L.NVR_F32)
    tr.set_batch(dev(I["o"]), dev(I["d"]), dev(I["Ct"]))
    st = ostep.StepState([ostep.FieldState(f, I["table"], I["params"])])
    losses_g, losses_r = [], []
    for _ in range(3):
        losses_g.append(float(tr.step().item()))
        losses_r.append(ostep.train_step(w, st, I["o"], I["d"], I["Ct"], None, [(0, w.n_rays)])["loss"])
    torch.cuda.synchronize()
    np.testing.assert_allclose(losses_g, losses_r, rtol=1e-4)
    np.testing.assert_allclose(host(fld.params), st.fields[0].params, rtol=0, atol=1e-4)
    assert O.state_values(tr.state)["step"] == 3
    tr.close()


def _cfg2_small(n_rays, seed_offset=0):
    return field_inputs(2, n_rays, seed_offset=seed_offset, occ_res=128)


def test_cfg2_fp32_step_matches_oracle():
    I = _cfg2_small(1500)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 128, I["o"], I["d"], I["Ct"])
    st = ostep.StepState([ostep.FieldState(f, I["table"], I["params"], occ_words=I["occ"])])
    ref = ostep.train_step(w, st, I["o"], I["d"], I["Ct"], None, [(0, w.n_rays)], apply=False)
    assert tr.sample_count() == ref["fwd"]["t"].size
    np.testing.assert_allclose(Cg, ref["C"], rtol=0, atol=1e-5)
    g = ref["grads"][0]
    assert rel_err(host(fld.params_grad), g["params"]) < 1e-4
    assert rel_err(host(fld.table_grad), g["table"]) < 1e-4
    tr.close()


@pytest.mark.parametrize("det", [False, True])
def test_cfg2_bf16_step_matches_oracle(det):
    I = _cfg2_small(1500, seed_offset=1)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 128, I["o"], I["d"], I["Ct"],
                                precision=L.NVR_BF16, deterministic=det)
    # the oracle sees the fp16 table copy and bf16 weights the fused path uses
    st = ostep.StepState([ostep.FieldState(f, f16_round(I["table"]), bf16_round(I["params"]),
                                           occ_words=I["occ"])])
    ref = ostep.train_step(w, st, I["o"], I["d"], I["Ct"], None, [(0, w.n_rays)], apply=False)
    err = np.abs(Cg - ref["C"]).max()
    print(f"bf16 step: colour max abs err {err:.3e}")
    assert err < 2e-2
    assert abs(loss - ref["loss"]) < 2e-2 * ref["loss"]
    g = ref["grads"][0]
    assert rel_err(host(fld.params_grad), g["params"]) < 5e-2
    assert rel_err(host(fld.table_grad), g["table"]) < 5e-2
    tr.close()


def test_graph_replay_matches_eager():
    I = _cfg2_small(800, seed_offset=2)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    outs = []
    for graph in (False, True):
        fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
        tr = F.Trainer([fld], w.n_rays, w.n_rays * 128, precision=L.NVR_BF16, use_graph=graph)
        tr.set_batch(dev(I["o"]), dev(I["d"]), dev(I["Ct"]))
        ls = []
        for _ in range(4):
            ls.append(float(tr.step().item()))       # eager sync between replays
        torch.cuda.synchronize()
        outs.append((ls, host(fld.params), host(fld.table)))
        tr.close()
    (l0, p0, t0), (l1, p1, t1) = outs
    # the table-gradient sums run in a non-deterministic order (LDS atomics), so
    # two runs differ by rounding; Adam's normalisation can scale that up for an
    # entry whose gradient is nearly zero, hence the per-entry bound of 4 lr
    np.testing.assert_allclose(l1, l0, rtol=1e-5)
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-4)
    diff = np.abs(t1 - t0)
    assert np.mean(diff > 1e-5) < 1e-4 and diff.max() < 4e-2


def test_deterministic_step_is_bitwise_reproducible():
    # NVR_DETERMINISTIC: four BF16 steps eagerly, again eagerly in a new
    # context, and as four replays of a captured graph give bit-identical
    # losses, parameters, tables and Adam moments
    I = _cfg2_small(800, seed_offset=2)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    outs = []
    for graph in (False, False, True):
        fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
        tr = F.Trainer([fld], w.n_rays, w.n_rays * 128, precision=L.NVR_BF16, use_graph=graph,
                       deterministic=True)
        tr.set_batch(dev(I["o"]), dev(I["d"]), dev(I["Ct"]))
        ls = []
        for _ in range(4):
            ls.append(host(tr.step()).copy())        # eager sync between replays
        torch.cuda.synchronize()
        outs.append([np.concatenate(ls), host(fld.params), host(fld.table), host(fld.table_m),
                     host(fld.table_v), host(fld.params_m), host(fld.params_v)])
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(np.ascontiguousarray(a).view(np.uint32),
                                  np.ascontiguousarray(b).view(np.uint32))


def test_autotuned_step_matches_default_shapes():
    # the autotuner only changes launch shapes: four graph steps with tuned
    # shapes agree with four eager steps at the default shapes (up to the
    # summation order of the gradients, as in the replay test above)
    I = _cfg2_small(900, seed_offset=5)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    outs, shapes = [], None
    for tune in (False, True):
        fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
        tr = F.Trainer([fld], w.n_rays, w.n_rays * 128, precision=L.NVR_BF16, use_graph=tune,
                       autotune=tune)
        tr.set_batch(dev(I["o"]), dev(I["d"]), dev(I["Ct"]))
        ls = [float(tr.step().item()) for _ in range(4)]
        torch.cuda.synchronize()
        if tune:
            shapes = tr.launch_shape(0)
        else:
            assert tr.launch_shape(0) == [0, 0, 0, 0, 0, 0, 0]
        outs.append((ls, host(fld.params), host(fld.table)))
        tr.close()
    assert shapes[0] in (256, 512, 1024, 2048) and shapes[1] in (256, 512, 1024, 2048)
    assert shapes[2] in (128, 256, 512) and shapes[3] in (32, 64, 128, 256, 512, 1024, 2048)
    assert shapes[4] in (4096, 16384, 65536) and shapes[5] == 1 and shapes[6] in (256, 512, 1024)
    (l0, p0, t0), (l1, p1, t1) = outs
    np.testing.assert_allclose(l1, l0, rtol=1e-5)
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-4)
    diff = np.abs(t1 - t0)
    assert np.mean(diff > 1e-5) < 1e-4 and diff.max() < 4e-2


def test_full_size_sampled_parity():
    # the object workload at its full size (2^18 rays, 16 levels, 2^19-entry
    # tables) in the launch configuration the benchmark times (captured graph,
    # autotuned shapes): after one training step, the forward of the trained
    # field is compared on sampled rays with the oracle computed ray by ray on
    # the same fp16 table and fp16-rounded weights
    L, F, O = lib()
    w = synth.config(2)
    f = w.fields[0]
    rng = synth.rng_for(w.seed)
    o, d = synth.sphere_rays(w.n_rays, rng)
    _, occ = synth.noise_occupancy(f.occ_res, rng)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    Ct = synth.smooth_colour_targets(o, d, rng)
    fld = F.Field(w, f, table, params, occ_words=occ)
    R = w.n_rays
    tr = F.Trainer([fld], R, R * 48, precision=L.NVR_BF16, use_graph=True, autotune=True)
    tr.set_batch(dev(o), dev(d), dev(Ct))
    loss = float(tr.step().item())
    assert np.isfinite(loss) and tr.launch_shape(0)[5] == 1
    Cg = torch.empty((R, 3), device="cuda")
    Dg = torch.empty(R, device="cuda")
    tr.forward(C_out=Cg, D_out=Dg)
    torch.cuda.synchronize()
    n_total = tr.sample_count()
    table16 = host(fld.table_half.float()).astype(np.float64)
    params16 = f16_round(host(fld.params))
    tr.close()
    pick = np.sort(synth.rng_for(99).choice(R, size=96, replace=False))
    st = ostep.StepState([ostep.FieldState(f, table16, params16, occ_words=occ)])
    ref = ostep.forward_all(w, st, o[pick], d[pick], [(0, pick.size)])
    # per-ray sample counts are exact (the marcher is bit-exact)
    full = omarch.march(o, d, f.aabb_min, f.aabb_max, w.near, w.far, omarch.step_size(w, f),
                        w.max_steps, occ, f.occ_res)
    assert n_total == full["t"].size
    np.testing.assert_array_equal(np.diff(ref["off"]), full["count"][pick])
    err = np.abs(host(Cg)[pick] - ref["C"]).max()
    print(f"full size: {n_total} samples, sampled colour max abs err {err:.3e}")
    assert err < 2e-2
    np.testing.assert_allclose(host(Dg)[pick], ref["D"], rtol=0, atol=2e-2)


def test_full_size_table_gradient_on_a_subset():
    # the binned table-gradient scatter over every sample of the object
    # workload's step (6.7 M marched samples, 16 levels, 2^19-entry tables;
    # the six launches the benchmark's roofline line times), with feature
    # gradients non-zero on a 10 000-sample subset: every table entry and the
    # position gradients against the oracle's backward of that subset
    L, F, O = lib()
    w = synth.config(2)
    f = w.fields[0]
    rng = synth.rng_for(w.seed)
    o, d = synth.sphere_rays(w.n_rays, rng)
    _, occ = synth.noise_occupancy(f.occ_res, rng)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, 2, rng)
    full = omarch.march(o, d, f.aabb_min, f.aabb_max, w.near, w.far, omarch.step_size(w, f),
                        w.max_steps, occ, f.occ_res)
    x = full["x"]
    n = x.shape[0]
    sub = np.sort(synth.rng_for(98).choice(n, size=10000, replace=False))
    g_sub = synth.rng_for(97).normal(size=(sub.size, 2 * f.n_levels)).astype(np.float32)
    grouped = np.zeros((8, n, 4), np.float32)
    for l in range(f.n_levels):
        grouped[l % 8, sub, 2 * (l // 8):2 * (l // 8) + 2] = g_sub[:, 2 * l:2 * l + 2]
    t16 = table.astype(np.float16)
    g = O.grid_desc_of(f)
    dtab = torch.zeros((lay.n_entries, 2), device="cuda")
    dx = torch.zeros((n, 3), device="cuda")
    O.encode_bwd_binned_grouped(g, dev(x), dev(t16), dev(grouped), dtab, dx)
    torch.cuda.synchronize()
    del grouped
    rt, rdx = ogrid.encode_backward(x[sub], t16.astype(np.float64), g_sub, lay)
    got = host(dtab)
    print(f"full-size subset scatter: {n} samples, table rel err {rel_err(got, rt):.3e}")
    assert rel_err(got, rt) < 1e-5
    np.testing.assert_allclose(got, rt, rtol=0, atol=1e-5 * np.abs(rt).max())
    gx = host(dx)
    assert rel_err(gx[sub], rdx) < 1e-4
    rest = np.ones(n, bool)
    rest[sub] = False
    assert not gx[rest].any()


def _human(n_rays, knn_res=32, n_nodes=512, seed=0, res_max=2048):
    f = synth.FieldCfg(occ_res=64, res_max=res_max)
    w = synth.WorkCfg("h", n_rays, (f,), warp=True)
    rng = synth.rng_for(500 + seed)
    rig = synth.human_rig(rng, n_nodes=n_nodes, knn_res=knn_res)
    o, d = synth.sphere_rays(n_rays, rng, aim_lo=(-0.3, -0.8, -0.2), aim_hi=(0.3, 0.8, 0.2))
    _, occ = synth.occupancy_from_points(rig["node_live"][0], 0.12, 64, f.aabb_min, f.aabb_max)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, 2, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    Ct = synth.uniform_targets(n_rays, rng)
    return w, f, rig, o, d, occ, table, params, Ct


def _decided_human(n_rays, seed=0, margin=5e-6):
    # candidate rays, then those whose warped samples keep 5e-6 m (about 50x
    # the float32 warp error) from every cell face of every level
    w, f, rig, o, d, occ, table, params, Ct = _human(8 * n_rays, seed=seed)
    box = ((-1.0,) * 3, (1.0,) * 3)
    pick = decided_rays(w, f, rig, o, d, occ, box, margin, n_rays)
    w = synth.WorkCfg(w.name, n_rays, w.fields, warp=True)
    return w, f, rig, o[pick], d[pick], occ, table, params, Ct[pick], box


def _position_sensitivity(run_oracle, eps=2.5e-7, seed=5):
    """The oracle's step with every warped (canonical) position moved by
    U[-eps, eps] per coordinate, eps the size of the float32 warp's rounding
    (2.5e-7 m measured at most): how far the gradients move when the positions
    carry float32-sized errors.  Only oracle arithmetic and seeded noise."""
    rng = np.random.default_rng(seed)
    orig = owarp.warp

    def noisy(x, *a, **k):
        out = orig(x, *a, **k)
        if k.get("want_cache"):
            return out
        return out + rng.uniform(-eps, eps, size=out.shape)

    owarp.warp = noisy
    try:
        return run_oracle()
    finally:
        owarp.warp = orig


def test_cfg3_warp_fp32_step():
    L, F, O = lib()
    w, f, rig, o, d, occ, table, params, Ct, box = _decided_human(600)
    R = O.Rig.from_numpy(rig)
    wd = O.warp_desc(n_nodes=512, lut_res=32)
    fld = F.Field(w, f, table, params, occ_words=occ, rig=R, warp_desc=wd)
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 128, o, d, Ct)
    def oracle():
        st = ostep.StepState([ostep.FieldState(f, table, params, occ_words=occ, rig=rig)])
        return ostep.train_step(w, st, o, d, Ct, None, [(0, w.n_rays)], box, apply=False)

    ref = oracle()
    pert = _position_sensitivity(oracle)
    g, gp = ref["grads"][0], pert["grads"][0]
    err = np.abs(Cg - ref["C"]).max()
    got = dict(params=host(fld.params_grad), table=host(fld.table_grad),
               node_dq=host(fld.node_dq_grad), bones=host(fld.bones_grad))
    errs = {k: rel_err(v, g[k].reshape(v.shape)) for k, v in got.items()}
    sens = {k: rel_err(gp[k], g[k]) for k in got}
    print(f"warp step: colour max abs err {err:.3e}, gradients {errs}, "
          f"oracle sensitivity to float32-sized position errors {sens}")
    assert err < 1e-5
    assert abs(loss - ref["loss"]) < 1e-5 * ref["loss"]
    # the FP32 bar, or what the oracle itself moves by when its canonical
    # positions carry float32-sized errors (at 2048 cells per axis the finest
    # weights change by ~2.5e-4 of a cell), whichever is larger
    for k, e in errs.items():
        assert e < max(1e-4, 4 * sens[k]), k
    tr.close()


def test_cfg4_two_fields_merged_fp32():
    L, F, O = lib()
    w, fh, rig, o, d, occ_h, table_h, params_h, Ct, box = _decided_human(600, seed=1)
    fo_ = synth.FieldCfg(log2_table=18, occ_res=64)
    rng = synth.rng_for(777)
    _, occ_o = synth.occupancy_from_points(synth.object_points(rng), 0.1, 64, fo_.aabb_min,
                                           fo_.aabb_max)
    lay_o = ogrid.Layout.from_field(fo_)
    table_o = synth.uniform_table(lay_o.n_entries, 2, rng)
    params_o = synth.xavier_params(fo_.layer_shapes(), rng)
    Dt = rng.uniform(1.0, 3.0, size=600).astype(np.float32)
    w = synth.WorkCfg("ho", 600, (fh, fo_), warp=True, lambda_depth=1.0)
    ranges = [(0, 450), (350, 600)]          # rays 350..449 shared
    R = O.Rig.from_numpy(rig)
    wd = O.warp_desc(n_nodes=512, lut_res=32)
    fld_h = F.Field(w, fh, table_h, params_h, occ_words=occ_h, rig=R, warp_desc=wd,
                    ray_range=ranges[0])
    fld_o = F.Field(w, fo_, table_o, params_o, occ_words=occ_o, ray_range=ranges[1])
    tr, loss, Cg, Dg = run_step([fld_h, fld_o], 600, 600 * 128, o, d, Ct, Dt, lam=1.0)
    def oracle():
        st = ostep.StepState([ostep.FieldState(fh, table_h, params_h, occ_words=occ_h, rig=rig),
                              ostep.FieldState(fo_, table_o, params_o, occ_words=occ_o)])
        return ostep.train_step(w, st, o, d, Ct, Dt, ranges, box, apply=False)

    ref = oracle()
    pert = _position_sensitivity(oracle)
    shared = (ref["fwd"]["src"] == 1).sum()
    assert shared > 0
    got = dict(params_h=(host(fld_h.params_grad), 0, "params"),
               table_h=(host(fld_h.table_grad), 0, "table"),
               node_dq=(host(fld_h.node_dq_grad), 0, "node_dq"),
               bones=(host(fld_h.bones_grad), 0, "bones"),
               params_o=(host(fld_o.params_grad), 1, "params"),
               table_o=(host(fld_o.table_grad), 1, "table"))
    errs = {k: rel_err(v, ref["grads"][i][n].reshape(v.shape)) for k, (v, i, n) in got.items()}
    sens = {k: rel_err(pert["grads"][i][n], ref["grads"][i][n]) for k, (_, i, n) in got.items()}
    ec, ed = np.abs(Cg - ref["C"]).max(), np.abs(Dg - ref["D"]).max()
    print(f"two fields: colour {ec:.3e}, depth {ed:.3e}, gradients {errs}, "
          f"oracle sensitivity {sens}")
    assert ec < 1e-5 and ed < 1e-5
    assert abs(loss - ref["loss"]) < 1e-5 * ref["loss"]
    # the object field has no warp: the FP32 bar as it stands
    for k in ("params_o", "table_o"):
        assert errs[k] < 1e-4, k
    for k in ("params_h", "table_h", "node_dq", "bones"):
        assert errs[k] < max(1e-4, 4 * sens[k]), k
    tr.close()


def test_render_bf16_matches_oracle_on_rounded_inputs():
    # the BF16 renderer (fp16 table copy, fp16 forward network with the SH
    # coefficients read from its per-ray table) against the oracle given the
    # same fp16 table and fp16-rounded weights.  What remains is the rounding
    # of the network's activations to fp16 (measured ~1e-5); the bound is 1e-3,
    # well inside the 2e-2 colour bar of the BF16 path
    I = _cfg2_small(700, seed_offset=5)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    fld = F.Field(w, f, I["table"], I["params"], occ_words=I["occ"])
    # a small sample capacity forces several ray chunks
    tr = F.Trainer([fld], w.n_rays, 200 * 128, precision=L.NVR_BF16)
    rgb, depth = tr.render(dev(I["o"]), dev(I["d"]), t_stop=1e-4)
    torch.cuda.synchronize()
    table16 = host(fld.table_half.float()).astype(np.float64)
    params16 = f16_round(host(fld.params))
    st = ostep.StepState([ostep.FieldState(f, table16, params16, occ_words=I["occ"])])
    rC, rD = ostep.render(w, st, I["o"], I["d"], [(0, w.n_rays)], t_stop=1e-4)
    err = np.abs(host(rgb) - rC).max()
    print(f"bf16 render: colour max abs err {err:.3e}")
    assert err < 1e-3
    np.testing.assert_allclose(host(depth), rD, rtol=0, atol=1e-3)
    tr.close()


def test_render_fp32_early_termination():
    I = _cfg2_small(700, seed_offset=4)
    L, F, O = lib()
    w, f = I["work"], I["fcfg"]
    # denser field so that early termination triggers
    params = I["params"].copy()
    fld = F.Field(w, f, I["table"], params, occ_words=I["occ"])
    tr = F.Trainer([fld], w.n_rays, 700 * 128, precision=L.NVR_F32)
    rgb, depth = tr.render(dev(I["o"]), dev(I["d"]), t_stop=1e-4)
    torch.cuda.synchronize()
    st = ostep.StepState([ostep.FieldState(f, I["table"], params, occ_words=I["occ"])])
    rC, rD = ostep.render(w, st, I["o"], I["d"], [(0, w.n_rays)], t_stop=1e-4)
    np.testing.assert_allclose(host(rgb), rC, rtol=0, atol=1e-4)
    tr.close()


# ----------------------------------------------------- deformation network
_DEFORM_GRID = (16, 2, 14, 16, 512, (-1.0,) * 3, (1.0,) * 3)   # levels, F, log2 T, res, box


def _deform_inputs(seed):
    lay = ogrid.Layout(*_DEFORM_GRID)
    theta, table, params = synth.deform_inputs(lay.n_entries, synth.rng_for(900 + seed))
    return lay, theta, table, params


def _decided_human_deform(n_rays, seed=0, margin=5e-6):
    # the human field on a 16 -> 512 ladder, its deformation network on its
    # own 16 -> 512 grid; rays decided on both encodings
    w, f, rig, o, d, occ, table, params, Ct = _human(16 * n_rays, seed=seed, res_max=512)
    box = ((-1.0,) * 3, (1.0,) * 3)
    dfm = _deform_inputs(seed)
    pick = decided_rays(w, f, rig, o, d, occ, box, margin, n_rays, deform=dfm)
    w = synth.WorkCfg(w.name, n_rays, w.fields, warp=True)
    return w, f, rig, o[pick], d[pick], occ, table, params, Ct[pick], box, dfm


def _deform_field(F, O, w, f, table, params, occ, rig, dfm):
    lay, theta, dtab, dpar = dfm
    D = F.Deform(O.grid_desc(*_DEFORM_GRID), theta, dtab, dpar)
    R = O.Rig.from_numpy(rig)
    wd = O.warp_desc(n_nodes=512, lut_res=32)
    return F.Field(w, f, table, params, occ_words=occ, rig=R, warp_desc=wd, deform=D)


def _deform_grads(fld):
    D = fld.deform
    return dict(params=host(fld.params_grad), table=host(fld.table_grad),
                node_dq=host(fld.node_dq_grad), bones=host(fld.bones_grad),
                deform_params=host(D.params_grad), deform_table=host(D.table_grad),
                theta=host(D.theta_grad))


def test_cfg3_warp_deform_fp32_step():
    # warp -> deformation network -> field (Sec. 4.2), float32 kernels, every
    # gradient of the step against the FP64 oracle
    L, F, O = lib()
    w, f, rig, o, d, occ, table, params, Ct, box, dfm = _decided_human_deform(300)
    fld = _deform_field(F, O, w, f, table, params, occ, rig, dfm)
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 128, o, d, Ct)

    def oracle():
        lay, theta, dtab, dpar = dfm
        st = ostep.StepState([ostep.FieldState(f, table, params, occ_words=occ, rig=rig,
                                               deform=ostep.DeformState(lay, theta, dtab,
                                                                        dpar))])
        return ostep.train_step(w, st, o, d, Ct, None, [(0, w.n_rays)], box, apply=False)

    ref = oracle()
    pert = _position_sensitivity(oracle)
    g, gp = ref["grads"][0], pert["grads"][0]
    got = _deform_grads(fld)
    errs = {k: rel_err(v, g[k].reshape(v.shape)) for k, v in got.items()}
    sens = {k: rel_err(gp[k], g[k]) for k in got}
    err = np.abs(Cg - ref["C"]).max()
    print(f"warp + deformation step: colour max abs err {err:.3e}, gradients {errs}, "
          f"oracle sensitivity {sens}")
    assert err < 1e-5
    assert abs(loss - ref["loss"]) < 1e-5 * ref["loss"]
    for k, e in errs.items():
        assert e < max(1e-4, 4 * sens[k]), k
    tr.close()


def test_cfg3_warp_deform_bf16_step():
    # the matrix-core deformation kernels inside the fused BF16 step against the
    # oracle on the fp16 / bf16 copies of the field and the fp16 copy of the
    # network's table: colour 2e-2 absolute, the
    # field's and the warp's gradients 5e-2 relative.  The network's own
    # gradients (weights, table, pose) sit behind two low-precision stages in
    # series -- their input, the encoding's position gradient, carries the
    # BF16 step's 5e-2, and the network's bf16 backward alone carries up to
    # 5e-2 (its large-batch test) -- so their bar is the sum, 1e-1.
    L, F, O = lib()
    w, f, rig, o, d, occ, table, params, Ct, box, dfm = _decided_human_deform(300, seed=1)
    fld = _deform_field(F, O, w, f, table, params, occ, rig, dfm)
    tr, loss, Cg, Dg = run_step([fld], w.n_rays, w.n_rays * 128, o, d, Ct, precision=L.NVR_BF16)
    lay, theta, dtab, dpar = dfm
    st = ostep.StepState([ostep.FieldState(f, f16_round(table), bf16_round(params),
                                           occ_words=occ, rig=rig,
                                           deform=ostep.DeformState(lay, theta, f16_round(dtab),
                                                                    dpar))])
    ref = ostep.train_step(w, st, o, d, Ct, None, [(0, w.n_rays)], box, apply=False)
    g = ref["grads"][0]
    got = _deform_grads(fld)
    errs = {k: rel_err(v, g[k].reshape(v.shape)) for k, v in got.items()}
    err = np.abs(Cg - ref["C"]).max()
    print(f"bf16 warp + deformation step: colour max abs err {err:.3e}, gradients {errs}")
    assert err < 2e-2
    assert abs(loss - ref["loss"]) < 2e-2 * ref["loss"]
    for k, e in errs.items():
        assert e < (1e-1 if k in ("deform_params", "deform_table", "theta") else 5e-2), k
    tr.close()


def test_deform_step_deterministic_and_graph():
    # NVR_DETERMINISTIC with the deformation network: three BF16 steps eagerly,
    # again in a new context, and as replays of a captured graph give
    # bit-identical losses and trained state (field and network)
    L, F, O = lib()
    w, f, rig, o, d, occ, table, params, Ct = _human(400, seed=2, res_max=512)
    dfm = _deform_inputs(2)
    outs = []
    for graph in (False, False, True):
        fld = _deform_field(F, O, w, f, table, params, occ, rig, dfm)
        tr = F.Trainer([fld], w.n_rays, w.n_rays * 128, precision=L.NVR_BF16, use_graph=graph,
                       deterministic=True)
        tr.set_batch(dev(o), dev(d), dev(Ct))
        ls = []
        for _ in range(3):
            ls.append(host(tr.step()).copy())        # eager sync between replays
        torch.cuda.synchronize()
        D = fld.deform
        outs.append([np.concatenate(ls), host(fld.params), host(fld.table), host(D.params),
                     host(D.table), host(D.params_m), host(D.table_v)])
        tr.close()
    assert np.abs(outs[0][3] - dfm[3]).max() > 0       # the network was trained
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(np.ascontiguousarray(a).view(np.uint32),
                                  np.ascontiguousarray(b).view(np.uint32))


def test_deform_field_rejections_leave_state_untouched():
    # every check of a field's deformation network runs before the step
    # launches anything: a network without the warp, a BF16 step without the
    # fp16 table copy, an encoding other than 16 levels x 2 features (8 levels)
    L, F, O = lib()
    w, f, rig, o, d, occ, table, params, Ct = _human(64, seed=3, res_max=512)
    dfm = _deform_inputs(3)
    lay, theta, dtab, dpar = dfm

    def attempt(fld, precision, expect):
        tr = F.Trainer([fld], w.n_rays, w.n_rays * 128, precision=precision)
        tr.set_batch(dev(o), dev(d), dev(Ct))
        before = [host(t).copy() for t in (fld.params, fld.table, fld.params_grad)]
        with pytest.raises(L.NvrError) as e:
            tr.forward()
        assert e.value.code == expect, str(e.value)
        torch.cuda.synchronize()
        after = [host(t) for t in (fld.params, fld.table, fld.params_grad)]
        assert all(np.array_equal(a, b) for a, b in zip(before, after))
        tr.close()

    # no warp
    D = F.Deform(O.grid_desc(*_DEFORM_GRID), theta, dtab, dpar)
    fld = F.Field(w, f, table, params, occ_words=occ)
    fld.rig = None
    fld.deform = D
    attempt(fld, L.NVR_F32, L.NVR_EINVAL)
    # BF16 without the fp16 copy of the network's table
    fld = _deform_field(F, O, w, f, table, params, occ, rig, dfm)
    fld.deform.table_half = None
    D2 = fld.deform
    D2.c = lambda: _c_without_half(L, D2)
    attempt(fld, L.NVR_BF16, L.NVR_EINVAL)
    # an 8-level encoding (16 wide)
    g8 = O.grid_desc(8, 2, 14, 16, 512, (-1.0,) * 3, (1.0,) * 3)
    n8 = ogrid.Layout(8, 2, 14, 16, 512, (-1.0,) * 3, (1.0,) * 3).n_entries
    D3 = F.Deform(g8, theta, np.zeros((n8, 2), np.float32), dpar)
    fld = _deform_field(F, O, w, f, table, params, occ, rig, dfm)
    fld.deform = D3
    attempt(fld, L.NVR_F32, L.NVR_EUNSUPPORTED)


def _c_without_half(L, D):
    d = L.DeformState()
    d.grid = D.grid
    for k in ("theta", "table", "params", "table_grad", "params_grad", "table_m", "table_v",
              "params_m", "params_v", "theta_grad"):
        setattr(d, k, getattr(D, k).data_ptr())
    D._c = d
    return d
