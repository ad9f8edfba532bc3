"""Pins of the FP64 compositing, marching, loss and Adam oracles."""
import math

import numpy as np
import pytest

import synth
from oracle import composite, march, optim


def ragged(rng, R=12, maxs=9):
    counts = rng.integers(0, maxs, size=R)
    counts[0] = 0
    off = np.concatenate([[0], np.cumsum(counts)])
    n = off[-1]
    sigma = rng.uniform(0, 30, size=n)
    rgb = rng.uniform(0, 1, size=(n, 3))
    dt = rng.uniform(0.01, 0.05, size=n)
    t = np.concatenate([np.cumsum(dt[a:b]) for a, b in zip(off[:-1], off[1:])] or [[]])
    return off, sigma, rgb, t, dt


def test_weights_telescope_and_transmittance_monotone():
    off, sigma, rgb, t, dt = ragged(synth.rng_for(20))
    C, D, TN, w = composite.forward(off, sigma, rgb, t, dt)
    for r in range(off.size - 1):
        a, b = off[r], off[r + 1]
        assert abs(w[a:b].sum() - (1 - TN[r])) < 1e-15
        assert w[a:b].sum() <= 1.0
    T = composite.product_form(off, sigma, dt)
    for r in range(off.size - 1):
        a, b = off[r], off[r + 1]
        assert np.all(np.diff(T[a:b]) <= 0)
    assert C[0].tolist() == [0, 0, 0] and D[0] == 0 and TN[0] == 1


def test_product_form_equals_exp_of_sum():
    off, sigma, rgb, t, dt = ragged(synth.rng_for(21))
    T = composite.product_form(off, sigma, dt)
    C, D, TN, w = composite.forward(off, sigma, rgb, t, dt)
    alpha = 1 - np.exp(-sigma * dt)
    np.testing.assert_allclose(w, T * alpha, rtol=1e-13, atol=1e-15)


def test_zero_density_and_closed_forms():
    off = np.array([0, 5])
    dt = np.full(5, 0.1)
    t = np.arange(5) * 0.1 + 0.05
    rgb = np.tile([0.2, 0.5, 0.9], (5, 1))
    C, D, TN, _ = composite.forward(off, np.zeros(5), rgb, t, dt)
    assert np.all(C == 0) and D[0] == 0 and TN[0] == 1
    s = 3.0
    C, D, TN, w = composite.forward(off, np.full(5, s), rgb, t, dt)
    np.testing.assert_allclose(C[0], rgb[0] * (1 - math.exp(-s * 0.5)), rtol=1e-15)
    np.testing.assert_allclose(TN[0], math.exp(-s * 0.5), rtol=1e-15)
    # depth of a constant-density ray: sum_i e^{-s dt i} (1-e^{-s dt}) t_i
    a = 1 - math.exp(-s * 0.1)
    want = sum(math.exp(-s * 0.1 * i) * a * t[i] for i in range(5))
    np.testing.assert_allclose(D[0], want, rtol=1e-14)
    C1, _, _, _ = composite.forward(np.array([0, 1]), np.array([s]), rgb[:1], t[:1], dt[:1])
    np.testing.assert_allclose(C1[0], rgb[0] * (1 - math.exp(-s * 0.1)), rtol=1e-15)


def test_early_termination_bounded():
    off, sigma, rgb, t, dt = ragged(synth.rng_for(22), R=30, maxs=40)
    sigma = sigma * 5
    C, D, _, _ = composite.forward(off, sigma, rgb, t, dt)
    Cs, Ds, _, w = composite.forward(off, sigma, rgb, t, dt, t_stop=1e-4)
    assert np.any(Cs != C)
    # the dropped weight is at most the transmittance at the cut, < 1e-4
    assert np.max(np.abs(Cs - C)) <= 1e-4 * rgb.max()


def test_backward_vs_fd_and_torch():
    import torch
    rng = synth.rng_for(23)
    off, sigma, rgb, t, dt = ragged(rng, R=10, maxs=8)
    R = off.size - 1
    gC = rng.normal(size=(R, 3))
    gD = rng.normal(size=R)
    dsig, drgb = composite.backward(off, sigma, rgb, t, dt, gC, gD)

    def L(s, c):
        C, D, _, _ = composite.forward(off, s, c, t, dt)
        return np.sum(C * gC) + np.sum(D * gD)
    h = 1e-6
    for i in range(sigma.size):
        sp, sm = sigma.copy(), sigma.copy()
        sp[i] += h
        sm[i] -= h
        assert abs((L(sp, rgb) - L(sm, rgb)) / (2 * h) - dsig[i]) < 1e-7
    # torch autograd of the exp-of-sum form, ray by ray
    ts = torch.tensor(sigma, requires_grad=True)
    tc = torch.tensor(rgb, requires_grad=True)
    tot = 0
    for r in range(R):
        a, b = off[r], off[r + 1]
        if a == b:
            continue
        tau = ts[a:b] * torch.tensor(dt[a:b])
        cs = torch.cumsum(tau, 0)
        Ti = torch.exp(-(cs - tau))
        w = Ti * (1 - torch.exp(-tau))
        tot = tot + (w @ tc[a:b] * torch.tensor(gC[r])).sum() + (w @ torch.tensor(t[a:b])) * gD[r]
    tot.backward()
    np.testing.assert_allclose(dsig, ts.grad.numpy(), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(drgb, tc.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_merge_two_sorted_and_ties():
    off_a = np.array([0, 2, 2, 4])
    t_a = np.array([0.1, 0.5, 0.2, 0.3])
    off_b = np.array([0, 1, 3, 4])
    t_b = np.array([0.3, 0.0, 0.9, 0.3])
    off, src, idx = composite.merge_two(off_a, t_a, off_b, t_b)
    assert off.tolist() == [0, 3, 5, 8]
    assert list(zip(src.tolist(), idx.tolist())) == [(0, 0), (1, 0), (0, 1), (1, 1), (1, 2),
                                                      (0, 2), (0, 3), (1, 3)]


# ------------------------------------------------------------------ march
def test_march_cfg1_fixed_samples():
    w = synth.config(1)
    f = w.fields[0]
    o, d = synth.sphere_rays(64, synth.rng_for(24))
    m = march.march(o, d, f.aabb_min, f.aabb_max, w.near, w.far, march.step_size(w, f),
                    w.max_steps)
    assert np.all(m["count"] == 64)
    t = m["t"].reshape(64, 64)
    np.testing.assert_array_equal(t[0], 1.0 + (np.arange(64) + 0.5) / 32.0)


def test_march_clip_matches_float64_box_intersection():
    rng = synth.rng_for(25)
    o, d = synth.sphere_rays(400, rng)
    lo, hi = np.array([-1.0] * 3), np.array([1.0] * 3)
    tn, tf = march.clip(o, d, lo, hi, 0.0, 1e30)
    od, dd = o.astype(np.float64), d.astype(np.float64)
    for r in range(400):
        # brute force: bisection on the inside test along the ray
        ts = np.linspace(0, 5, 50001)
        pts = od[r] + ts[:, None] * dd[r]
        ins = np.all((pts >= lo) & (pts <= hi), 1)
        if not ins.any():
            assert tf[r] <= tn[r]
            continue
        assert abs(ts[ins][0] - tn[r]) < 2e-4 and abs(ts[ins][-1] - tf[r]) < 2e-4


def test_march_occupancy_skip_equals_masked_dense():
    w = synth.config(2, scale=1 / 1024)
    f = w.fields[0]
    rng = synth.rng_for(26)
    o, d = synth.sphere_rays(w.n_rays, rng)
    occ, words = synth.noise_occupancy(32, rng)
    delta = march.step_size(w, f)
    m = march.march(o, d, f.aabb_min, f.aabb_max, w.near, w.far, delta, w.max_steps,
                    words, 32)
    full, bit = march.march_dense(o, d, f.aabb_min, f.aabb_max, w.near, w.far, delta,
                                  w.max_steps, words, 32)
    assert 0 < m["t"].size < full["t"].size
    np.testing.assert_array_equal(m["t"], full["t"][bit])
    np.testing.assert_array_equal(m["x"], full["x"][bit])
    # compositing the kept samples == compositing all with sigma forced to 0
    rngv = synth.rng_for(27)
    sig_full = rngv.uniform(0, 20, size=full["t"].size)
    rgb_full = rngv.uniform(0, 1, size=(full["t"].size, 3))
    C1, D1, _, _ = composite.forward(m["off"], sig_full[bit], rgb_full[bit], m["t"], m["dt"])
    C2, D2, _, _ = composite.forward(full["off"], np.where(bit, sig_full, 0), rgb_full,
                                     full["t"], full["dt"])
    np.testing.assert_allclose(C1, C2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(D1, D2, rtol=0, atol=1e-15)
    # positions stay in the box, spacing is delta, at most max_steps per ray
    assert np.all(np.abs(m["x"]) <= 1.0 + 1e-6)
    assert m["count"].max() <= w.max_steps
    ft = full["t"]
    for r in range(20):
        a, b = full["off"][r], full["off"][r + 1]
        if b - a > 1:
            np.testing.assert_allclose(np.diff(ft[a:b]), delta, rtol=0, atol=1e-6)


def test_march_diagonal_has_max_steps():
    w = synth.config(2)
    f = w.fields[0]
    o = np.array([[-1.5, -1.5, -1.5]], np.float32)
    d = np.array([[1, 1, 1]], np.float32) / np.float32(math.sqrt(3))
    m = march.march(o, d, f.aabb_min, f.aabb_max, 0.0, 1e30, march.step_size(w, f), 128)
    assert m["count"][0] in (127, 128)


# ------------------------------------------------------------------ loss / Adam
def test_loss_grad_fd_and_eq8_relation():
    rng = synth.rng_for(28)
    C, Ct = rng.uniform(size=(7, 3)), rng.uniform(size=(7, 3))
    D, Dt = rng.uniform(1, 3, size=7), rng.uniform(1, 3, size=7)
    L, dC, dD = optim.loss(C, D, Ct, Dt, lambda_d=0.5)
    h = 1e-6
    Cp = C.copy()
    Cp[2, 1] += h
    Cm = C.copy()
    Cm[2, 1] -= h
    fd = (optim.loss(Cp, D, Ct, Dt, 0.5)[0] - optim.loss(Cm, D, Ct, Dt, 0.5)[0]) / (2 * h)
    assert abs(fd - dC[2, 1]) < 1e-9
    Dp = D.copy()
    Dp[3] += h
    Dm = D.copy()
    Dm[3] -= h
    fd = (optim.loss(C, Dp, Ct, Dt, 0.5)[0] - optim.loss(C, Dm, Ct, Dt, 0.5)[0]) / (2 * h)
    assert abs(fd - dD[3]) < 1e-9
    # a single ray: the squared colour term is the square of the printed norm
    lc, ld = optim.eq8_loss(C[:1], D[:1], Ct[:1], Dt[:1])
    L1, _, _ = optim.loss(C[:1], D[:1], Ct[:1], Dt[:1], 1.0)
    np.testing.assert_allclose(L1, lc ** 2 + ld ** 2, rtol=1e-14)


def test_adam_matches_torch_float64():
    import torch
    rng = synth.rng_for(29)
    p0 = rng.normal(size=50)
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    ad = optim.Adam()
    for s in range(1, 6):
        g = rng.normal(size=50)
        ad.update(p, g, m, v, s)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_decay_matches_torch_exponential_schedule():
    # update k uses lr * decay^(k-1): torch's ExponentialLR multiplies the rate
    # by gamma after every step
    import torch
    rng = synth.rng_for(30)
    p0 = rng.normal(size=40)
    p = p0.copy()
    m = np.zeros(40)
    v = np.zeros(40)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    sched = torch.optim.lr_scheduler.ExponentialLR(opt, gamma=0.5)
    ad = optim.Adam(lr_decay=0.5)
    for s in range(1, 7):
        g = rng.normal(size=40)
        ad.update(p, g, m, v, s)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        sched.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)
    # a single update of a unit gradient moves by the decayed rate exactly
    q = np.zeros(1)
    mm, vv = np.zeros(1), np.zeros(1)
    for k in range(1, 4):
        before = q.copy()
        optim.Adam(lr_decay=0.5).update(q, np.ones(1), mm, vv, k)
        assert abs((before - q)[0] - 1e-2 * 0.5 ** (k - 1)) < 1e-15


def test_adam_skips_zero_gradient_entries():
    p = np.ones(4)
    m = np.zeros(4)
    v = np.zeros(4)
    optim.Adam().update(p, np.array([0.0, 1.0, 0.0, -2.0]), m, v, 1, skip_zero=True)
    assert p[0] == 1 and p[2] == 1 and m[0] == 0 and v[2] == 0
    np.testing.assert_allclose(p[[1, 3]], [1 - 1e-2, 1 + 1e-2], rtol=1e-12)


def test_unscale_detects_non_finite():
    g, ok = optim.unscale_and_check([np.array([2.0, 4.0])], 2.0)
    assert ok and g[0].tolist() == [1.0, 2.0]
    _, ok = optim.unscale_and_check([np.array([np.inf, 1.0])], 2.0)
    assert not ok
