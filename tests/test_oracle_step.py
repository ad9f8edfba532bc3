"""Whole-step pins of the FP64 oracle: end-to-end gradients by finite
differences, the two-field merge, loss scaling and the non-finite skip."""
import copy

import numpy as np
import pytest

import synth
from oracle import grid, march, step


def tiny_field(k=1, **over):
    w = synth.config(k)
    f = w.fields[0]
    f = synth.FieldCfg(**{**f.__dict__, **over})
    return w, f


def make_state(fields, rng, occ=None, rig=None):
    sts = []
    for i, f in enumerate(fields):
        lay = grid.Layout.from_field(f)
        st = step.FieldState(f, synth.uniform_table(lay.n_entries, f.n_features, rng),
                             synth.xavier_params(f.layer_shapes(), rng),
                             occ_words=None if occ is None else occ[i],
                             rig=rig if (rig is not None and i == 0) else None)
        sts.append(st)
    return step.StepState(sts)


def loss_only(work, state, o, d, Ct, Dt, ranges, box=None):
    s = copy.deepcopy(state)
    return step.train_step(work, s, o, d, Ct, Dt, ranges, box, apply=False)["loss"]


def test_cfg1_tiny_end_to_end_fd():
    w, f = tiny_field(1, n_levels=4, log2_table=10, res_max=64)
    w = synth.WorkCfg(**{**w.__dict__, "n_rays": 6, "fields": (f,)})
    rng = synth.rng_for(40)
    o, d = synth.sphere_rays(6, rng)
    Ct = synth.uniform_targets(6, rng)
    state = make_state([f], rng)
    ranges = [(0, 6)]
    out = step.train_step(w, copy.deepcopy(state), o, d, Ct, None, ranges, apply=False)
    g = out["grads"][0]
    h = 1e-6
    for j in rng.choice(f.n_params, 10, replace=False):
        sp, sm = copy.deepcopy(state), copy.deepcopy(state)
        sp.fields[0].params[j] += h
        sm.fields[0].params[j] -= h
        fd = (loss_only(w, sp, o, d, Ct, None, ranges) - loss_only(w, sm, o, d, Ct, None, ranges)) / (2 * h)
        assert abs(fd - g["params"][j]) < 1e-8 + 1e-6 * abs(fd)
    nz = np.flatnonzero(np.abs(g["table"]).sum(1) > 0)
    for e in rng.choice(nz, 8, replace=False):
        sp, sm = copy.deepcopy(state), copy.deepcopy(state)
        sp.fields[0].table[e, 0] += h
        sm.fields[0].table[e, 0] -= h
        fd = (loss_only(w, sp, o, d, Ct, None, ranges) - loss_only(w, sm, o, d, Ct, None, ranges)) / (2 * h)
        assert abs(fd - g["table"][e, 0]) < 1e-8 + 1e-6 * abs(fd)


def test_human_warp_node_gradient_fd():
    rng = synth.rng_for(41)
    rig = synth.human_rig(rng, n_nodes=64, knn_res=8)
    f = synth.FieldCfg(n_levels=4, log2_table=10, res_max=64, occ_res=0, colour_hidden=(16,),
                       density_hidden=(16,), sh_degree=2)
    w = synth.WorkCfg("t", 8, (f,), warp=True, max_steps=24)
    o, d = synth.sphere_rays(8, rng, aim_lo=(-0.2, -0.5, -0.1), aim_hi=(0.2, 0.5, 0.1))
    Ct = synth.uniform_targets(8, rng)
    state = make_state([f], rng, rig=rig)
    box = ((-1.0,) * 3, (1.0,) * 3)
    out = step.train_step(w, copy.deepcopy(state), o, d, Ct, None, [(0, 8)], box, apply=False)
    g = out["grads"][0]["node_dq"][0]
    nodes = np.flatnonzero(np.abs(g).sum(1) > 0)
    assert nodes.size > 4
    h = 1e-6
    for nd in rng.choice(nodes, 4, replace=False):
        for c in (0, 2, 5, 7):
            sp, sm = copy.deepcopy(state), copy.deepcopy(state)
            for s_, sg in ((sp, 1), (sm, -1)):
                r = dict(rig)
                r["node_dq"] = rig["node_dq"].astype(np.float64).copy()
                r["node_dq"][0, nd, c] += sg * h
                s_.fields[0].rig = r
            fd = (loss_only(w, sp, o, d, Ct, None, [(0, 8)], box)
                  - loss_only(w, sm, o, d, Ct, None, [(0, 8)], box)) / (2 * h)
            # position steps may cross hash cells: allow FD noise of that size
            assert abs(fd - g[nd, c]) < 1e-6 + 2e-3 * abs(fd), (nd, c, fd, g[nd, c])


def test_two_field_merge_gradient_fd():
    rng = synth.rng_for(42)
    fa = synth.FieldCfg(n_levels=3, log2_table=10, res_max=32, occ_res=0, density_hidden=(8,),
                        colour_hidden=(8,), sh_degree=1)
    fb = synth.FieldCfg(n_levels=3, log2_table=9, res_max=32, occ_res=0, density_hidden=(8,),
                        colour_hidden=(8,), sh_degree=1, aabb_min=(-0.5,) * 3, aabb_max=(1.0,) * 3)
    w = synth.WorkCfg("t2", 6, (fa, fb), lambda_depth=1.0, max_steps=16)
    o, d = synth.sphere_rays(6, rng)
    Ct = synth.uniform_targets(6, rng)
    Dt = rng.uniform(1, 3, size=6).astype(np.float32)
    state = make_state([fa, fb], rng)
    ranges = [(0, 4), (2, 6)]               # rays 2,3 shared
    out = step.train_step(w, copy.deepcopy(state), o, d, Ct, Dt, ranges, apply=False)
    fw = out["fwd"]
    # shared rays composite samples of both fields, sorted by t
    for r in (2, 3):
        a, b = fw["off"][r], fw["off"][r + 1]
        assert set(fw["src"][a:b].tolist()) == {0, 1}
        assert np.all(np.diff(fw["t"][a:b]) >= 0)
    h = 1e-6
    for fi in (0, 1):
        gp = out["grads"][fi]["params"]
        for j in rng.choice(gp.size, 6, replace=False):
            sp, sm = copy.deepcopy(state), copy.deepcopy(state)
            sp.fields[fi].params[j] += h
            sm.fields[fi].params[j] -= h
            fd = (loss_only(w, sp, o, d, Ct, Dt, ranges) - loss_only(w, sm, o, d, Ct, Dt, ranges)) / (2 * h)
            assert abs(fd - gp[j]) < 1e-8 + 1e-6 * abs(fd)


def test_loss_scale_is_exact_and_nonfinite_skips():
    w, f = tiny_field(1, n_levels=4, log2_table=10, res_max=64)
    w = synth.WorkCfg(**{**w.__dict__, "n_rays": 4, "fields": (f,)})
    rng = synth.rng_for(43)
    o, d = synth.sphere_rays(4, rng)
    Ct = synth.uniform_targets(4, rng)
    s1 = make_state([f], rng)
    s2 = copy.deepcopy(s1)
    s2.loss_scale = 1024.0
    g1 = step.train_step(w, s1, o, d, Ct, None, [(0, 4)])["grads"][0]
    g2 = step.train_step(w, s2, o, d, Ct, None, [(0, 4)])["grads"][0]
    np.testing.assert_allclose(g1["params"], g2["params"], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(s1.fields[0].params, s2.fields[0].params, rtol=1e-13)
    # an infinite target makes every gradient non-finite: skip + halve
    s3 = copy.deepcopy(s1)
    before = s3.fields[0].params.copy()
    Cbad = Ct.copy()
    Cbad[0, 0] = np.inf
    out = step.train_step(w, s3, o, d, Cbad, None, [(0, 4)])
    assert not out["finite"]
    assert s3.loss_scale == 0.5 * s1.loss_scale
    np.testing.assert_array_equal(s3.fields[0].params, before)


def test_training_decreases_loss():
    w, f = tiny_field(1, n_levels=4, log2_table=10, res_max=64)
    w = synth.WorkCfg(**{**w.__dict__, "n_rays": 32, "fields": (f,)})
    rng = synth.rng_for(44)
    o, d = synth.sphere_rays(32, rng)
    Ct = synth.uniform_targets(32, rng)
    s = make_state([f], rng)
    losses = [step.train_step(w, s, o, d, Ct, None, [(0, 32)])["loss"] for _ in range(15)]
    assert losses[-1] < 0.7 * losses[0]


def _human_deform_case(seed, out_scale=0.05):
    rng = synth.rng_for(seed)
    rig = synth.human_rig(rng, n_nodes=64, knn_res=8)
    f = synth.FieldCfg(n_levels=4, log2_table=10, res_max=64, occ_res=0, colour_hidden=(16,),
                       density_hidden=(16,), sh_degree=2)
    w = synth.WorkCfg("t", 8, (f,), warp=True, max_steps=24)
    o, d = synth.sphere_rays(8, rng, aim_lo=(-0.2, -0.5, -0.1), aim_hi=(0.2, 0.5, 0.1))
    Ct = synth.uniform_targets(8, rng)
    state = make_state([f], rng, rig=rig)
    dlay = grid.Layout(16, 2, 10, 4, 64, (-1.0,) * 3, (1.0,) * 3)
    theta, table, params = synth.deform_inputs(dlay.n_entries, rng, out_scale=out_scale)
    state.fields[0].deform = step.DeformState(dlay, theta, table, params)
    return w, rig, o, d, Ct, state


def test_human_deform_zero_output_layer_reduces_to_the_warp():
    # with the output layer at zero the residual vanishes exactly: every loss
    # and field / node gradient equals the warp-only step's, the network's only
    # nonzero gradient is the output layer's (Sec. 4.2, x_c = x_t + residual)
    w, rig, o, d, Ct, state = _human_deform_case(43)
    D = state.fields[0].deform
    n_out = 3 * 128
    D.params[-n_out:] = 0.0
    box = ((-1.0,) * 3, (1.0,) * 3)
    plain = copy.deepcopy(state)
    plain.fields[0].deform = None
    a = step.train_step(w, copy.deepcopy(state), o, d, Ct, None, [(0, 8)], box, apply=False)
    b = step.train_step(w, plain, o, d, Ct, None, [(0, 8)], box, apply=False)
    assert a["loss"] == b["loss"]
    ga, gb = a["grads"][0], b["grads"][0]
    for k in ("table", "params", "node_dq", "bones"):
        np.testing.assert_array_equal(ga[k], gb[k])
    assert np.all(ga["deform_params"][:-n_out] == 0.0)
    assert np.abs(ga["deform_params"][-n_out:]).max() > 0.0
    assert np.all(ga["deform_table"] == 0.0) and np.all(ga["theta"] == 0.0)


def test_human_deform_gradients_fd():
    # central differences of the whole step's loss through the deformation
    # network: its parameters (first and last layer, pose columns included),
    # its table, the pose and the node motions behind it
    w, rig, o, d, Ct, state = _human_deform_case(44)
    box = ((-1.0,) * 3, (1.0,) * 3)
    rng = synth.rng_for(45)
    out = step.train_step(w, copy.deepcopy(state), o, d, Ct, None, [(0, 8)], box, apply=False)
    g = out["grads"][0]
    h = 1e-6

    def fd_of(mutate):
        sp, sm = copy.deepcopy(state), copy.deepcopy(state)
        mutate(sp, h)
        mutate(sm, -h)
        return (loss_only(w, sp, o, d, Ct, None, [(0, 8)], box)
                - loss_only(w, sm, o, d, Ct, None, [(0, 8)], box)) / (2 * h)

    def close(fd, an):
        # position steps may cross hash cells: allow FD noise of that size
        return abs(fd - an) < 1e-7 + 2e-3 * abs(fd)

    gp = g["deform_params"]
    first = 128 * 104
    picks = list(rng.choice(first, 3, replace=False)) + [5 * 104 + 40, 77 * 104 + 100]
    picks += list(gp.size - 3 * 128 + rng.choice(3 * 128, 3, replace=False))
    checked = 0
    for j in picks:
        def mut(s_, e, j=j):
            s_.fields[0].deform.params[j] += e
        fd = fd_of(mut)
        assert close(fd, gp[j]), (j, fd, gp[j])
        checked += abs(fd) > 1e-9
    assert checked >= 4
    gt = g["deform_table"]
    nz = np.flatnonzero(np.abs(gt).sum(1) > 0)
    assert nz.size > 10
    for e in rng.choice(nz, 4, replace=False):
        def mut(s_, dd, e=e):
            s_.fields[0].deform.table[e, 1] += dd
        fd = fd_of(mut)
        assert close(fd, gt[e, 1]), (e, fd, gt[e, 1])
    for c in (0, 31, 71):
        def mut(s_, dd, c=c):
            s_.fields[0].deform.theta[c] += dd
        fd = fd_of(mut)
        assert close(fd, g["theta"][c]), (c, fd, g["theta"][c])
    gn = g["node_dq"][0]
    for nd in rng.choice(np.flatnonzero(np.abs(gn).sum(1) > 0), 2, replace=False):
        def mut(s_, dd, nd=nd):
            r = dict(rig)
            r["node_dq"] = rig["node_dq"].astype(np.float64).copy()
            r["node_dq"][0, nd, 5] += dd
            s_.fields[0].rig = r
        fd = fd_of(mut)
        assert close(fd, gn[nd, 5]), (nd, fd, gn[nd, 5])


def test_human_deform_adam_trains_the_network():
    # one applied step moves the deformation network's parameters and the
    # table entries its encoding touched, and leaves untouched entries alone
    w, rig, o, d, Ct, state = _human_deform_case(46)
    box = ((-1.0,) * 3, (1.0,) * 3)
    D0 = copy.deepcopy(state.fields[0].deform)
    out = step.train_step(w, state, o, d, Ct, None, [(0, 8)], box, apply=True)
    D = state.fields[0].deform
    touched = np.abs(out["grads"][0]["deform_table"]).sum(1) > 0
    assert np.all(D.table[~touched] == D0.table[~touched])
    assert np.all(D.table[touched] != D0.table[touched])
    assert np.abs(D.params - D0.params).max() > 0
    np.testing.assert_array_equal(D.theta, D0.theta)
