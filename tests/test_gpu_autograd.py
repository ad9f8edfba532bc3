"""The torch.autograd.Function layer (ops.EncodeFn, WarpFn, FieldNetFn,
CompositeFn): gradients that torch's backward pass collects through the
hand-written backward entry points, against the FP64 oracle's gradients and
against central differences of the GPU forward (float32, so the difference
quotients carry ~1e-4 relative rounding)."""
import numpy as np
import pytest

import synth
from oracle import composite as ocomp, grid as ogrid, network as onet, sh as osh
from oracle import warp as owarp

from helpers import dev, host, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def ops():
    from paper_2304_03184_amd import ops as O
    return O


def _fd(f, t, idx, h):
    """Central difference of the scalar f() in element idx of tensor t."""
    with torch.no_grad():
        old = t[idx].item()
        t[idx] = old + h
        fp = f().item()
        t[idx] = old - h
        fm = f().item()
        t[idx] = old
    return (fp - fm) / (2 * h)


def test_encode_fn():
    # 8-level ladder (16 -> 512 over a 3 m box): cells of >= 6 mm, so a 1e-4 m
    # step stays inside its cell and the trilinear blend is exactly linear in it
    O = ops()
    f = synth.config(1).fields[0]
    lay = ogrid.Layout.from_field(f)
    g = O.grid_desc_of(f)
    rng = synth.rng_for(300)
    n = 257
    x_np = rng.uniform(-1.2, 1.2, size=(n, 3)).astype(np.float32)
    t_np = synth.uniform_table(lay.n_entries, 2, rng).astype(np.float32)
    W_np = rng.normal(size=(n, 2 * f.n_levels)).astype(np.float32)
    x = dev(x_np).requires_grad_(True)
    table = dev(t_np).requires_grad_(True)
    W = dev(W_np)

    def loss():
        return (O.EncodeFn.apply(x, table, g) * W).sum()

    loss().backward()
    rt, rdx = ogrid.encode_backward(x_np, t_np.astype(np.float64), W_np, lay)
    assert rel_err(host(table.grad), rt) < 1e-5
    assert rel_err(host(x.grad), rdx) < 1e-4
    # central differences of the GPU forward: linear in the table (exact up to
    # rounding), trilinear inside a cell in the position
    hit = np.argwhere(np.abs(rt).sum(1) > 0)[:, 0]
    for e in rng.choice(hit, 4, replace=False):
        fd = _fd(loss, table, (int(e), 0), 1e-2)
        assert abs(fd - table.grad[e, 0].item()) < 1e-3 * max(1.0, abs(fd))
    h = 1e-4
    u = np.clip((x_np[:, None, :] - lay.lo) / lay.side, 0, 1) * np.asarray(lay.res)[None, :, None]
    margin = (np.abs(u - np.round(u)) * (lay.side / np.asarray(lay.res)[:, None])).min((1, 2))
    for s in np.nonzero(margin > 3 * h)[0][:3]:      # steps that stay inside every cell
        for a in range(3):
            fd = _fd(loss, x, (int(s), a), h)
            assert abs(fd - x.grad[s, a].item()) < 2e-2 * max(1.0, abs(fd))


def test_warp_fn():
    O = ops()
    rig = synth.human_rig(synth.rng_for(301), n_nodes=256, knn_res=16)
    wd = O.warp_desc(n_nodes=256, lut_res=16)
    R = O.Rig.from_numpy(rig)
    rng = synth.rng_for(302)
    p = rig["node_live"][0][rng.integers(0, 256, 500)]
    x_np = (p + rng.normal(scale=0.03, size=p.shape)).astype(np.float32)
    G_np = rng.normal(size=(500, 3)).astype(np.float32)
    x = dev(x_np).requires_grad_(True)
    node_dq = R.node_dq.clone().requires_grad_(True)
    bones = R.bones.clone().requires_grad_(True)
    G = dev(G_np)

    def loss():
        return (O.WarpFn.apply(x, node_dq, bones, wd, R) * G).sum()

    loss().backward()
    r_dq, r_b, r_dx = owarp.warp_backward(x_np, rig, (-1.0,) * 3, (1.0,) * 3, G_np, want_dx=True)
    assert rel_err(host(node_dq.grad), r_dq) < 1e-4
    assert rel_err(host(bones.grad), r_b.reshape(host(bones.grad).shape)) < 1e-4
    assert rel_err(host(x.grad), r_dx) < 1e-4
    # the forward reads the node motions and bones passed in, not the rig's
    with torch.no_grad():
        moved = node_dq.clone()
        moved[..., 4:] = 0.0                         # no translation on any node
        z0 = O.WarpFn.apply(x, node_dq, bones, wd, R)
        z1 = O.WarpFn.apply(x, moved, bones, wd, R)
    assert (z0 - z1).abs().max().item() > 1e-3
    # central differences of the GPU forward (small steps keep every float32
    # joint, voxel and sign choice)
    touched = np.argwhere(np.abs(r_dq[0]).sum(1) > 0)[:, 0]
    for node in rng.choice(touched, 3, replace=False):
        for c in (0, 5):
            fd = _fd(loss, node_dq, (0, int(node), c), 1e-3)
            assert abs(fd - node_dq.grad[0, node, c].item()) < 2e-2 * max(1.0, abs(fd))
    h = 1e-4
    checked = 0
    for s in range(50):
        if checked == 3:
            break
        # only where the step keeps the float32 voxel and joint choices
        xs = np.repeat(x_np[s:s + 1].astype(np.float64), 7, 0)
        for a in range(3):
            xs[1 + 2 * a, a] += h
            xs[2 + 2 * a, a] -= h
        vox = owarp.lut_voxel(xs.astype(np.float32), (-1.0,) * 3, (1.0,) * 3, 16)
        js = np.sort(owarp.nearest_joints(xs.astype(np.float32), rig["joints"], 4), 1)
        if np.any(vox != vox[0]) or np.any(js != js[0]):
            continue
        checked += 1
        for a in range(3):
            fd = _fd(loss, x, (s, a), h)
            assert abs(fd - x.grad[s, a].item()) < 2e-2 * max(1.0, abs(fd))
    assert checked == 3


def test_field_net_fn():
    O = ops()
    f = synth.config(2).fields[0]
    rng = synth.rng_for(303)
    n = 1000
    params_np = synth.xavier_params(f.layer_shapes(), rng).astype(np.float32)
    feat_np = rng.uniform(-0.2, 0.2, size=(n, f.enc_width)).astype(np.float32)
    d = rng.normal(size=(n // 4 + 1, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    ray = rng.integers(0, d.shape[0], size=n).astype(np.int32)
    a_np = rng.normal(size=n).astype(np.float32)
    B_np = rng.normal(size=(n, 3)).astype(np.float32)
    feat = dev(feat_np).requires_grad_(True)
    params = dev(params_np).requires_grad_(True)
    md = O.mlp_desc_of(f)
    dd, rr, a, B = dev(d), dev(ray), dev(a_np), dev(B_np)

    def loss():
        sigma, rgb = O.FieldNetFn.apply(feat, params, dd, rr, md, O.F32)
        return (sigma * a).sum() + (rgb * B).sum()

    loss().backward()
    shv = osh.sh_encode(d[ray], f.sh_degree)
    _, _, cache = onet.forward(f, params_np, feat_np, shv)
    rp, rf = onet.backward(f, cache, a_np, B_np)
    assert rel_err(host(params.grad), rp) < 1e-5
    assert rel_err(host(feat.grad), rf) < 1e-5
    for i in rng.choice(params_np.size, 4, replace=False):
        fd = _fd(loss, params, (int(i),), 1e-3)
        assert abs(fd - params.grad[i].item()) < 2e-2 * max(1.0, abs(fd))


def test_composite_fn():
    O = ops()
    rng = synth.rng_for(304)
    R, n_max = 200, 60
    counts = rng.integers(0, n_max, size=R)
    counts[:3] = (0, 1, n_max)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(off[-1])
    sig_np = rng.uniform(0.0, 30.0, size=n).astype(np.float32)
    rgb_np = rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
    dt_np = np.full(n, 0.02, np.float32)
    t_np = np.concatenate([0.5 + 0.02 * (np.arange(c) + 0.5) for c in counts]).astype(np.float32)
    gC_np = rng.normal(size=(R, 3)).astype(np.float32)
    gD_np = rng.normal(size=R).astype(np.float32)
    sigma = dev(sig_np).requires_grad_(True)
    rgb = dev(rgb_np).requires_grad_(True)
    t, dt, offd, gC, gD = dev(t_np), dev(dt_np), dev(off), dev(gC_np), dev(gD_np)

    def loss():
        C, D = O.CompositeFn.apply(sigma, rgb, t, dt, offd)
        return (C * gC).sum() + (D * gD).sum()

    loss().backward()
    rs, rr = ocomp.backward(off, sig_np, rgb_np, t_np, dt_np, gC_np, gD_np)
    assert rel_err(host(sigma.grad), rs) < 1e-4
    assert rel_err(host(rgb.grad), rr) < 1e-5
    for i in rng.choice(n, 4, replace=False):
        fd = _fd(loss, sigma, (int(i),), 1e-2)
        assert abs(fd - sigma.grad[i].item()) < 2e-2 * max(1.0, abs(fd))


def test_chained_functions_match_the_oracle_step_gradients():
    # encode -> networks -> compositing chained by torch autograd over the
    # samples of a marched batch (the 4096-ray workload's field at 300 rays);
    # each backward recomputes its forward, nothing per sample is stored
    # between the Functions but their inputs
    from oracle import step as ostep
    from helpers import field_inputs
    O = ops()
    I = field_inputs(1, 300)
    w, f = I["work"], I["fcfg"]
    md = O.march_desc_of(w, f)
    m = O.march(md, dev(I["o"]), dev(I["d"]))
    g = O.grid_desc_of(f)
    table = dev(I["table"].astype(np.float32)).requires_grad_(True)
    params = dev(I["params"].astype(np.float32)).requires_grad_(True)
    feat = O.EncodeFn.apply(m["x"], table, g)
    sigma, rgb = O.FieldNetFn.apply(feat, params, dev(I["d"]), m["ray_id"], O.mlp_desc_of(f),
                                    O.F32)
    C, D = O.CompositeFn.apply(sigma, rgb, m["t"], m["dt"], m["off"])
    loss = ((C - dev(I["Ct"])) ** 2).sum(1).mean()
    loss.backward()
    st = ostep.StepState([ostep.FieldState(f, I["table"], I["params"])])
    ref = ostep.train_step(w, st, I["o"], I["d"], I["Ct"], None, [(0, w.n_rays)], apply=False)
    assert abs(loss.item() - ref["loss"]) < 1e-5 * ref["loss"]
    assert rel_err(host(params.grad), ref["grads"][0]["params"]) < 1e-4
    assert rel_err(host(table.grad), ref["grads"][0]["table"]) < 1e-4
