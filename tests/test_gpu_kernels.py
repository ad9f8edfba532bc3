"""Kernel-level parity of the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import composite as ocomp, grid as ogrid, march as omarch, network as onet
from oracle import optim as ooptim, sh as osh, warp as owarp

from helpers import bf16_round, dev, f16_round, field_inputs, host, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_03184_amd import _lib
    _lib.lib()


def ops():
    from paper_2304_03184_amd import ops as o
    return o


# ------------------------------------------------------------------ march
@pytest.mark.parametrize("k,n_rays,occ_res", [(1, 300, None), (2, 3000, 128), (2, 777, 32)])
def test_march_bit_exact(k, n_rays, occ_res):
    I = field_inputs(k, n_rays, occ_res=occ_res)
    w, f = I["work"], I["fcfg"]
    O = ops()
    md = O.march_desc_of(w, f)
    occ = dev(I["occ"].view(np.int32)) if I["occ"] is not None else None
    g = O.march(md, dev(I["o"]), dev(I["d"]), occ)
    ref = omarch.march(I["o"], I["d"], f.aabb_min, f.aabb_max, w.near, w.far,
                       omarch.step_size(w, f), w.max_steps, I["occ"], f.occ_res)
    assert g["n"] == ref["t"].size and g["n"] > 0
    np.testing.assert_array_equal(host(g["off"]), ref["off"])
    np.testing.assert_array_equal(host(g["ray_id"]), ref["ray"])
    np.testing.assert_array_equal(host(g["t"]), ref["t"])
    np.testing.assert_array_equal(host(g["x"]), ref["x"])
    np.testing.assert_array_equal(host(g["dt"]), ref["dt"])


def test_march_ray_range_capacity_and_empty():
    I = field_inputs(2, 500, occ_res=64)
    w, f = I["work"], I["fcfg"]
    O = ops()
    md = O.march_desc_of(w, f)
    occ = dev(I["occ"].view(np.int32))
    g = O.march(md, dev(I["o"]), dev(I["d"]), occ, ray_begin=100, ray_end=300)
    off = host(g["off"])
    assert np.all(off[:101] == 0) and np.all(off[300:] == off[300])
    ref = omarch.march(I["o"][100:300], I["d"][100:300], f.aabb_min, f.aabb_max, w.near, w.far,
                       omarch.step_size(w, f), w.max_steps, I["occ"], f.occ_res)
    np.testing.assert_array_equal(host(g["t"]), ref["t"])
    # capacity smaller than the total: reported, offsets clamped, nothing written past it
    g2 = O.march(md, dev(I["o"]), dev(I["d"]), occ, capacity=50, sync=False)
    torch.cuda.synchronize()
    assert int(g2["n_dev"].item()) > 50
    assert int(host(g2["off"]).max()) == 50
    # rays that miss the box entirely
    o = np.array([[5.0, 5.0, 5.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    g3 = O.march(md, dev(o), dev(d), occ)
    assert g3["n"] == 0


# ------------------------------------------------------------------ encode
def _positions(rng, n, lo, hi):
    x = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    x[:4] = np.array([[lo] * 3, [hi] * 3, [lo, hi, lo], [hi, lo, hi]], np.float32)  # corners
    return x


@pytest.mark.parametrize("k", [1, 2])
def test_encode_fp32_fwd_bwd(k):
    I = field_inputs(k, 8)
    f, lay = I["fcfg"], I["lay"]
    O = ops()
    g = O.grid_desc_of(f)
    assert g.n_entries == lay.n_entries and list(g.res)[:f.n_levels] == lay.res
    rng = synth.rng_for(7)
    x = _positions(rng, 5000, f.aabb_min[0], f.aabb_max[0])
    feat = O.encode_fwd(g, dev(x), dev(I["table"]))
    ref = ogrid.encode(x, I["table"], lay)
    np.testing.assert_allclose(host(feat), ref, rtol=0, atol=2e-7)
    dfeat = rng.normal(size=ref.shape).astype(np.float32)
    dtab = torch.zeros((lay.n_entries, 2), device="cuda")
    dx = torch.zeros((5000, 3), device="cuda")
    O.encode_bwd(g, dev(x), dev(I["table"]), dev(dfeat), dtab, dx)
    rt, rdx = ogrid.encode_backward(x, I["table"], dfeat, lay)
    assert rel_err(host(dtab), rt) < 1e-5
    np.testing.assert_allclose(host(dtab), rt, rtol=0, atol=1e-5 * np.abs(rt).max())
    assert rel_err(host(dx), rdx) < 1e-4


def test_encode_split_fp16_table():
    I = field_inputs(2, 8)
    f, lay = I["fcfg"], I["lay"]
    O = ops()
    g = O.grid_desc_of(f)
    rng = synth.rng_for(8)
    x = _positions(rng, 20000, -1.0, 1.0)
    t16 = I["table"].astype(np.float16)
    feat = O.encode_fwd(g, dev(x), dev(t16), torch.float32)
    ref = ogrid.encode(x, t16.astype(np.float64), lay)
    np.testing.assert_allclose(host(feat), ref, rtol=0, atol=2e-7)
    featb = O.encode_fwd(g, dev(x), dev(t16), torch.bfloat16)
    np.testing.assert_allclose(host(featb.float()), ref, rtol=8e-3, atol=1e-6)
    dfeat = rng.normal(size=ref.shape).astype(np.float32)
    dtab = torch.zeros((lay.n_entries, 2), device="cuda")
    dx = torch.zeros((20000, 3), device="cuda")
    O.encode_bwd(g, dev(x), dev(t16), dev(dfeat), dtab, dx)
    rt, rdx = ogrid.encode_backward(x, t16.astype(np.float64), dfeat, lay)
    assert rel_err(host(dtab), rt) < 1e-5
    assert rel_err(host(dx), rdx) < 1e-4
    # binned scatter (count / scan / append / per-tile LDS sum): same gradients
    dtab2 = torch.zeros((lay.n_entries, 2), device="cuda")
    dx2 = torch.zeros((20000, 3), device="cuda")
    O.encode_bwd_binned(g, dev(x), dev(t16), dev(dfeat), dtab2, dx2)
    assert rel_err(host(dtab2), rt) < 1e-5
    np.testing.assert_allclose(host(dtab2), rt, rtol=0, atol=1e-5 * np.abs(rt).max())
    assert rel_err(host(dx2), rdx) < 1e-4
    # a second call accumulates
    O.encode_bwd_binned(g, dev(x), dev(t16), dev(dfeat), dtab2)
    assert rel_err(host(dtab2), 2 * rt) < 1e-5


def _to_grouped(a, L):
    """[n][2L] -> level-group layout [8][n][2 ceil(L/8)] (level g + 8m at 2m, 2m+1)."""
    lpg = (L + 7) // 8
    out = np.zeros((8, a.shape[0], 2 * lpg), a.dtype)
    for l in range(L):
        g, m = l % 8, l // 8
        out[g, :, 2 * m:2 * m + 2] = a[:, 2 * l:2 * l + 2]
    return out


@pytest.mark.parametrize("k,n", [(1, 3001), (2, 20000)])
def test_encode_grouped_layout(k, n):
    I = field_inputs(k, 8)
    f, lay = I["fcfg"], I["lay"]
    O = ops()
    g = O.grid_desc_of(f)
    rng = synth.rng_for(18)
    lo, hi = (-1.5, 1.5) if k == 1 else (-1.0, 1.0)
    x = _positions(rng, n, lo, hi)
    t16 = I["table"].astype(np.float16)
    ref = ogrid.encode(x, t16.astype(np.float64), lay)
    L = f.n_levels
    feat = O.encode_fwd_grouped(g, dev(x), dev(t16))
    assert tuple(feat.shape) == (8, n, 2 * ((L + 7) // 8))
    np.testing.assert_allclose(host(feat.float()), _to_grouped(ref, L), rtol=1e-3, atol=1e-7)
    dfeat = rng.normal(size=ref.shape).astype(np.float32)
    rt, rdx = ogrid.encode_backward(x, t16.astype(np.float64), dfeat, lay)
    dtab = torch.zeros((lay.n_entries, 2), device="cuda")
    dx = torch.zeros((n, 3), device="cuda")
    O.encode_bwd_binned_grouped(g, dev(x), dev(t16), dev(_to_grouped(dfeat, L)), dtab, dx)
    assert rel_err(host(dtab), rt) < 1e-5
    np.testing.assert_allclose(host(dtab), rt, rtol=0, atol=1e-5 * np.abs(rt).max())
    assert rel_err(host(dx), rdx) < 1e-4


def test_encode_binned_heavy_tiles_and_empty():
    # 300k samples in a small region: the coarse tiles are split over many work
    # items (partial slabs summed by a last pass), the rest owned by single items
    I = field_inputs(2, 8)
    f, lay = I["fcfg"], I["lay"]
    O = ops()
    g = O.grid_desc_of(f)
    rng = synth.rng_for(9)
    x = rng.uniform(-0.2, 0.2, size=(300000, 3)).astype(np.float32)
    t16 = I["table"].astype(np.float16)
    dfeat = rng.normal(size=(300000, 32)).astype(np.float32)
    dtab = torch.zeros((lay.n_entries, 2), device="cuda")
    O.encode_bwd_binned(g, dev(x), dev(t16), dev(dfeat), dtab)
    rt, _ = ogrid.encode_backward(x, t16.astype(np.float64), dfeat, lay, want_dx=False)
    assert rel_err(host(dtab), rt) < 1e-5
    empty = torch.zeros((0, 3), device="cuda")
    O.encode_bwd_binned(g, empty, dev(t16), torch.zeros((0, 32), device="cuda"), dtab)


# ------------------------------------------------------------------ warp
@pytest.fixture(scope="module")
def small_rig():
    return synth.human_rig(synth.rng_for(60), n_nodes=512, knn_res=32)


def _live(rig, rng, n):
    p = rig["node_live"][0][rng.integers(0, rig["node_live"].shape[1], n)]
    return (p + rng.normal(scale=0.03, size=p.shape)).astype(np.float32)


def test_warp_fwd_bwd(small_rig):
    O = ops()
    rig = small_rig
    R = O.Rig.from_numpy(rig)
    wd = O.warp_desc(n_nodes=512, lut_res=32)
    rng = synth.rng_for(61)
    x = _live(rig, rng, 4000)
    z = O.warp_fwd(wd, R, dev(x))
    ref = owarp.warp(x, rig, (-1.0,) * 3, (1.0,) * 3)
    np.testing.assert_allclose(host(z), ref, rtol=0, atol=5e-6)
    gz = rng.normal(size=(4000, 3)).astype(np.float32)
    d_dq = torch.zeros_like(R.node_dq)
    d_b = torch.zeros_like(R.bones)
    dx = torch.full((4000, 3), 0.5, device="cuda")      # accumulated into
    O.warp_bwd(wd, R, dev(x), dev(gz), d_dq, d_b, dx_live=dx)
    r_dq, r_b, r_dx = owarp.warp_backward(x, rig, (-1.0,) * 3, (1.0,) * 3, gz, want_dx=True)
    assert rel_err(host(d_dq), r_dq) < 1e-4
    assert rel_err(host(d_b), r_b.reshape(host(d_b).shape)) < 1e-4
    assert rel_err(host(dx) - 0.5, r_dx) < 1e-4
    np.testing.assert_allclose(host(dx) - 0.5, r_dx, rtol=0, atol=1e-4 * np.abs(r_dx).max())


def test_warp_identity_rig(small_rig):
    O = ops()
    rig = dict(small_rig)
    b = np.zeros_like(rig["bones"])
    b[..., 0, 0] = b[..., 1, 1] = b[..., 2, 2] = 1
    dq = np.zeros_like(rig["node_dq"])
    dq[..., 0] = 1
    rig["bones"], rig["node_dq"] = b, dq
    x = _live(rig, synth.rng_for(62), 1000)
    z = O.warp_fwd(O.warp_desc(n_nodes=512, lut_res=32), O.Rig.from_numpy(rig), dev(x))
    np.testing.assert_allclose(host(z), x, rtol=0, atol=1e-6)


# ------------------------------------------------------------------ networks
def _net_inputs(k, n, seed):
    f = synth.config(k).fields[0]
    rng = synth.rng_for(seed)
    params = synth.xavier_params(f.layer_shapes(), rng)
    feat = rng.uniform(-0.2, 0.2, size=(n, f.enc_width)).astype(np.float32)
    d = rng.normal(size=(n // 4 + 1, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    ray = rng.integers(0, d.shape[0], size=n).astype(np.int32)
    dsig = rng.normal(size=n).astype(np.float32)
    drgb = rng.normal(size=(n, 3)).astype(np.float32)
    return f, params, feat, d, ray, dsig, drgb


@pytest.mark.parametrize("k", [1, 2])
def test_mlp_fp32(k):
    O = ops()
    n = 3000
    f, params, feat, d, ray, dsig, drgb = _net_inputs(k, n, 70 + k)
    md = O.mlp_desc_of(f)
    sig, rgb = O.mlp_fwd(md, dev(feat), dev(d), dev(params), dev(ray))
    shv = osh.sh_encode(d[ray], f.sh_degree)
    rs, rr, cache = onet.forward(f, params, feat, shv)
    np.testing.assert_allclose(host(sig), rs, rtol=2e-6)
    np.testing.assert_allclose(host(rgb), rr, rtol=0, atol=1e-6)
    dparams = torch.zeros(params.size, device="cuda")
    dfeat = O.mlp_bwd(md, dev(feat), dev(d), dev(params), dev(dsig), dev(drgb), dparams, dev(ray))
    rp, rf = onet.backward(f, cache, dsig, drgb)
    assert rel_err(host(dparams), rp) < 1e-5
    assert rel_err(host(dfeat), rf) < 1e-5


@pytest.mark.parametrize("k", [2])
def test_mlp_bf16_mfma(k):
    O = ops()
    n = 5000       # several tiles and a ragged tail (5000 = 312*16 + 8)
    f, params, feat, d, ray, dsig, drgb = _net_inputs(k, n, 80 + k)
    md = O.mlp_desc_of(f)
    pb = dev(params).to(torch.bfloat16)
    fb = dev(feat).to(torch.bfloat16)
    sig, rgb = O.mlp_fwd(md, fb, dev(d), pb, dev(ray), O.BF16)
    # oracle on the same bf16-rounded inputs, in float64
    shv = osh.sh_encode(d[ray], f.sh_degree)
    rs, rr, cache = onet.forward(f, bf16_round(params), bf16_round(feat), shv)
    np.testing.assert_allclose(host(rgb), rr, rtol=0, atol=2e-2)
    assert rel_err(host(sig), rs) < 3e-2
    dparams = torch.zeros(params.size, device="cuda")
    dfeat = O.mlp_bwd(md, fb, dev(d), pb, dev(dsig), dev(drgb), dparams, dev(ray), O.BF16)
    rp, rf = onet.backward(f, cache, dsig, drgb)
    assert rel_err(host(dparams), rp) < 3e-2
    assert rel_err(host(dfeat), rf) < 3e-2


@pytest.mark.parametrize("k", [2])
def test_mlp_f16_forward_mfma(k):
    # fp16 forward (fp16 features, fp32 parameters converted to fp16 fragments,
    # fp16 activations), bf16 backward products
    O = ops()
    n = 5000
    f, params, feat, d, ray, dsig, drgb = _net_inputs(k, n, 90 + k)
    md = O.mlp_desc_of(f)
    pf = dev(params)
    fh = dev(feat).to(torch.float16)
    sig, rgb = O.mlp_fwd(md, fh, dev(d), pf, dev(ray), O.F16)
    shv = osh.sh_encode(d[ray], f.sh_degree)
    rs, rr, cache = onet.forward(f, f16_round(params), f16_round(feat), shv)
    # fp16 activations: relative rounding 2^-11 per layer
    np.testing.assert_allclose(host(rgb), rr, rtol=0, atol=4e-3)
    assert rel_err(host(sig), rs) < 1e-2
    dparams = torch.zeros(params.size, device="cuda")
    dfeat = O.mlp_bwd(md, fh, dev(d), pf, dev(dsig), dev(drgb), dparams, dev(ray), O.F16)
    rp, rf = onet.backward(f, cache, dsig, drgb)
    assert rel_err(host(dparams), rp) < 3e-2
    assert rel_err(host(dfeat), rf) < 3e-2


# ------------------------------------------------------------------ compositing
def _ragged(rng, R, maxs, sig_scale=30.0):
    counts = rng.integers(0, maxs, size=R)
    counts[:3] = [0, 1, maxs]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(off[-1])
    sigma = rng.uniform(0, sig_scale, size=n).astype(np.float32)
    rgb = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    dt = np.full(n, 0.02, np.float32)
    t = np.concatenate([1.0 + np.arange(c) * 0.02 for c in counts]).astype(np.float32) \
        if n else np.zeros(0, np.float32)
    return off, sigma, rgb, t, dt


def test_composite_fwd_bwd():
    O = ops()
    rng = synth.rng_for(90)
    off, sigma, rgb, t, dt = _ragged(rng, 700, 130)
    keep = [dev(v) for v in (off, sigma, rgb, t, dt)]
    a = O.samples(*keep)
    C, D, TN = O.composite_fwd(a, n_rays=700)
    rC, rD, rTN, _ = ocomp.forward(off, sigma, rgb, t, dt)
    np.testing.assert_allclose(host(C), rC, rtol=0, atol=2e-6)
    np.testing.assert_allclose(host(D), rD, rtol=0, atol=1e-5)
    np.testing.assert_allclose(host(TN), rTN, rtol=0, atol=2e-6)
    gC = rng.normal(size=(700, 3)).astype(np.float32)
    gD = rng.normal(size=700).astype(np.float32)
    ds, dr, _, _ = O.composite_bwd(a, sigma.size, C, D, dev(gC), dev(gD))
    rs, rr = ocomp.backward(off, sigma, rgb, t, dt, gC, gD)
    np.testing.assert_allclose(host(dr), rr, rtol=0, atol=2e-6)
    assert rel_err(host(ds), rs) < 1e-4
    np.testing.assert_allclose(host(ds), rs, rtol=0, atol=2e-5 * np.abs(rs).max())


def test_composite_merged_and_early_stop():
    O = ops()
    rng = synth.rng_for(91)
    offa, sa, ca, ta, dta = _ragged(rng, 300, 40)
    offb, sb, cb, tb, dtb = _ragged(rng, 300, 40)
    tb = (tb + 0.01).astype(np.float32)          # interleave with list a
    ka = [dev(v) for v in (offa, sa, ca, ta, dta)]
    kb = [dev(v) for v in (offb, sb, cb, tb, dtb)]
    a, b = O.samples(*ka), O.samples(*kb)
    C, D, _ = O.composite_fwd(a, b, n_rays=300)
    moff, src, idx = ocomp.merge_two(offa, ta, offb, tb)
    pick = lambda va, vb: np.where((src == 0)[:, None] if va.ndim == 2 else src == 0,  # noqa: E731
                                   va[np.where(src == 0, idx, 0)], vb[np.where(src == 1, idx, 0)])
    ms, mc, mt, mdt = pick(sa, sb), pick(ca, cb), pick(ta, tb), pick(dta, dtb)
    rC, rD, _, _ = ocomp.forward(moff, ms, mc, mt, mdt)
    np.testing.assert_allclose(host(C), rC, rtol=0, atol=2e-6)
    np.testing.assert_allclose(host(D), rD, rtol=0, atol=1e-5)
    gC = rng.normal(size=(300, 3)).astype(np.float32)
    gD = rng.normal(size=300).astype(np.float32)
    dsa, dra, dsb, drb = O.composite_bwd(a, sa.size, C, D, dev(gC), dev(gD), b, sb.size)
    rs, rr = ocomp.backward(moff, ms, mc, mt, mdt, gC, gD)
    ds_m = np.where(src == 0, host(dsa)[np.where(src == 0, idx, 0)], host(dsb)[np.where(src == 1, idx, 0)])
    assert rel_err(ds_m, rs) < 1e-4
    # early termination (forward only)
    Cs, Ds, _ = O.composite_fwd(a, n_rays=300, t_stop=1e-4)
    rCs, rDs, _, _ = ocomp.forward(offa, sa, ca, ta, dta, t_stop=1e-4)
    np.testing.assert_allclose(host(Cs), rCs, rtol=0, atol=1e-4)


def test_loss_and_adam():
    O = ops()
    rng = synth.rng_for(92)
    C = rng.uniform(size=(1000, 3)).astype(np.float32)
    Ct = rng.uniform(size=(1000, 3)).astype(np.float32)
    D = rng.uniform(1, 3, size=1000).astype(np.float32)
    Dt = rng.uniform(1, 3, size=1000).astype(np.float32)
    scale = torch.tensor([8.0], device="cuda")
    l, dC, dD = O.loss(dev(C), dev(D), dev(Ct), dev(Dt), None, 0.5, scale)
    rl, rdC, rdD = ooptim.loss(C, D, Ct, Dt, 0.5)
    assert abs(l.item() - rl) < 1e-5 * rl
    np.testing.assert_allclose(host(dC) / 8.0, rdC, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(host(dD) / 8.0, rdD, rtol=1e-5, atol=1e-9)
    # Adam: three steps with a loss scale of 4, zero-gradient entries skipped
    p = rng.normal(size=4096).astype(np.float32)
    pg, mg, vg = dev(p), torch.zeros(4096, device="cuda"), torch.zeros(4096, device="cuda")
    copy = dev(p).to(torch.float16)        # the copy starts equal to the master
    st = O.new_state(4.0)
    pr, mr, vr = p.astype(np.float64), np.zeros(4096), np.zeros(4096)
    ad = ooptim.Adam()
    for s in range(1, 4):
        g = rng.normal(size=4096).astype(np.float32)
        g[::7] = 0
        gg = dev(g * 4.0)
        O.state_begin(st)
        O.check_finite(gg, st)
        O.adam(O.adam_desc(), pg, mg, vg, gg, st, skip_zero=True, copy=copy)
        O.state_end(st)
        ad.update(pr, g.astype(np.float64), mr, vr, s, skip_zero=True)
        assert float(host(gg).max()) == 0.0
    np.testing.assert_allclose(host(pg), pr, rtol=0, atol=2e-6)
    np.testing.assert_allclose(host(copy).astype(np.float64), pr, rtol=1e-3, atol=1e-4)
    assert O.state_values(st)["step"] == 3
    # a non-finite gradient skips the update and halves the scale
    bad = torch.full((4096,), float("inf"), device="cuda")
    before = host(pg).copy()
    O.state_begin(st)
    O.check_finite(bad, st)
    O.adam(O.adam_desc(), pg, mg, vg, bad, st)
    O.state_end(st)
    sv = O.state_values(st)
    assert sv["step"] == 3 and sv["loss_scale"] == 2.0
    np.testing.assert_array_equal(host(pg), before)
    # exponential rate decay: update k uses lr * 0.5^(k-1), k from the device step
    st2 = O.new_state(1.0)
    pg2, mg2, vg2 = dev(p), torch.zeros(4096, device="cuda"), torch.zeros(4096, device="cuda")
    pr2, mr2, vr2 = p.astype(np.float64), np.zeros(4096), np.zeros(4096)
    ad2 = ooptim.Adam(lr_decay=0.5)
    for s in range(1, 5):
        g = rng.normal(size=4096).astype(np.float32)
        O.state_begin(st2)
        O.adam(O.adam_desc(lr_decay=0.5), pg2, mg2, vg2, dev(g), st2)
        O.state_end(st2)
        ad2.update(pr2, g.astype(np.float64), mr2, vr2, s)
    np.testing.assert_allclose(host(pg2), pr2, rtol=0, atol=2e-6)


@pytest.mark.parametrize("k,n,spread", [(1, 3001, 1.5), (2, 20000, 1.0), (2, 300000, 0.2)])
def test_encode_deterministic_scatter(k, n, spread):
    # the deterministic binned scatter: oracle gradients to the binned bar, and
    # bit-identical tables and position gradients over repeated calls (the
    # 300k clustered case splits the coarse tiles over many work items)
    I = field_inputs(k, 8)
    f, lay = I["fcfg"], I["lay"]
    O = ops()
    g = O.grid_desc_of(f)
    rng = synth.rng_for(19)
    x = rng.uniform(-spread, spread, size=(n, 3)).astype(np.float32)
    t16 = I["table"].astype(np.float16)
    dfeat = rng.normal(size=(n, 2 * f.n_levels)).astype(np.float32)
    rt, rdx = ogrid.encode_backward(x, t16.astype(np.float64), dfeat, lay)
    xd, td, dfd = dev(x), dev(t16), dev(dfeat)
    outs = []
    for rep in range(3):
        print(f"deterministic scatter: k={k} n={n} call {rep}", flush=True)
        dtab = torch.zeros((lay.n_entries, 2), device="cuda")
        dx = torch.zeros((n, 3), device="cuda")
        O.encode_bwd_deterministic(g, xd, td, dfd, dtab, dx)
        outs.append((host(dtab), host(dx)))
    assert rel_err(outs[0][0], rt) < 1e-5
    np.testing.assert_allclose(outs[0][0], rt, rtol=0, atol=1e-5 * np.abs(rt).max())
    assert rel_err(outs[0][1], rdx) < 1e-4
    for dtab, dx in outs[1:]:
        assert np.array_equal(dtab.view(np.uint32), outs[0][0].view(np.uint32))
        assert np.array_equal(dx.view(np.uint32), outs[0][1].view(np.uint32))
    # accumulation into a non-zero table
    dtab = torch.from_numpy(outs[0][0].copy()).cuda()
    O.encode_bwd_deterministic(g, xd, td, dfd, dtab)
    assert rel_err(host(dtab), 2 * rt) < 1e-5
