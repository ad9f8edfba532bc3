"""Pins of the FP64 SH and network oracles."""
import math

import numpy as np
import pytest

import synth
from oracle import network, sh


def unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_sh_constant_band():
    d = unit(synth.rng_for(10), 20)
    np.testing.assert_allclose(sh.sh_encode(d, 1)[:, 0], 1.0 / (2.0 * math.sqrt(math.pi)),
                               rtol=0, atol=0)


def test_sh_addition_theorem():
    # sum_m Y_lm(d)^2 = (2l+1)/(4 pi) for every unit d
    d = unit(synth.rng_for(11), 200)
    Y = sh.sh_encode(d, 4)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) * (l + 1)] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi integrates degree <= 6
    # polynomial products exactly.
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * math.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y = sh.sh_encode(d, 4)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_sh_matches_scipy_real_form():
    from scipy.special import sph_harm_y
    d = unit(synth.rng_for(12), 64)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = sh.sh_encode(d, 4)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            elif m == 0:
                ref = c.real
            else:
                ref = math.sqrt(2) * (-1) ** m * c.real
            np.testing.assert_allclose(Y[:, k], ref, atol=1e-13)
            k += 1


def _torch_net(fcfg, params, feat, shv):
    import torch
    Ws, p = [], 0
    for o, i in fcfg.layer_shapes():
        Ws.append(params[p:p + o * i].reshape(o, i))
        p += o * i
    nd = len(fcfg.density_hidden) + 1
    h = feat
    for k in range(nd):
        h = torch.nn.functional.linear(h, Ws[k])
        if k < nd - 1:
            h = torch.relu(h)
    sigma = torch.exp(torch.clamp(h[:, 0], -15, 15))
    g = torch.cat([h, shv], 1)
    for k in range(nd, len(Ws)):
        g = torch.nn.functional.linear(g, Ws[k])
        if k < len(Ws) - 1:
            g = torch.relu(g)
    return sigma, torch.sigmoid(g)


@pytest.mark.parametrize("k", [1, 2])
def test_network_forward_backward_vs_torch_autograd(k):
    import torch
    fcfg = synth.config(k).fields[0]
    rng = synth.rng_for(13)
    n = 64
    params = synth.xavier_params(fcfg.layer_shapes(), rng).astype(np.float64)
    feat = rng.uniform(-0.2, 0.2, size=(n, fcfg.enc_width))
    shv = sh.sh_encode(unit(rng, n), fcfg.sh_degree)
    dsig = rng.normal(size=n)
    drgb = rng.normal(size=(n, 3))
    sigma, rgb, cache = network.forward(fcfg, params, feat, shv)
    dparams, dfeat = network.backward(fcfg, cache, dsig, drgb)
    tp = torch.tensor(params, requires_grad=True)
    tf = torch.tensor(feat, requires_grad=True)
    ts, tr = _torch_net(fcfg, tp, tf, torch.tensor(shv))
    np.testing.assert_allclose(sigma, ts.detach().numpy(), rtol=1e-14)
    np.testing.assert_allclose(rgb, tr.detach().numpy(), rtol=1e-14)
    (ts * torch.tensor(dsig)).sum().add((tr * torch.tensor(drgb)).sum()).backward()
    np.testing.assert_allclose(dparams, tp.grad.numpy(), rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(dfeat, tf.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_network_param_fd():
    fcfg = synth.config(1).fields[0]
    rng = synth.rng_for(14)
    n = 16
    params = synth.xavier_params(fcfg.layer_shapes(), rng).astype(np.float64)
    feat = rng.uniform(-0.2, 0.2, size=(n, fcfg.enc_width))
    shv = sh.sh_encode(unit(rng, n), fcfg.sh_degree)
    dsig, drgb = rng.normal(size=n), rng.normal(size=(n, 3))
    _, _, cache = network.forward(fcfg, params, feat, shv)
    dparams, _ = network.backward(fcfg, cache, dsig, drgb)

    def f(p):
        s, c, _ = network.forward(fcfg, p, feat, shv)
        return np.sum(s * dsig) + np.sum(c * drgb)
    for j in rng.choice(params.size, 25, replace=False):
        h = 1e-6
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        assert abs((f(pp) - f(pm)) / (2 * h) - dparams[j]) < 1e-7 * max(1, abs(dparams[j]))


def test_density_clamp_has_zero_gradient_outside():
    fcfg = synth.config(1).fields[0]
    rng = synth.rng_for(15)
    params = synth.xavier_params(fcfg.layer_shapes(), rng).astype(np.float64) * 40.0
    feat = rng.uniform(-1, 1, size=(256, fcfg.enc_width))
    shv = sh.sh_encode(unit(rng, 256), fcfg.sh_degree)
    sigma, _, cache = network.forward(fcfg, params, feat, shv)
    out = np.abs(cache["o0"]) > 15
    assert out.any()
    np.testing.assert_allclose(sigma[out], np.exp(np.sign(cache["o0"][out]) * 15))


def test_xavier_bounds():
    rng = synth.rng_for(16)
    shapes = [(64, 32), (16, 64)]
    p = synth.xavier_params(shapes, rng)
    a0 = math.sqrt(6 / 96)
    w0 = p[:2048]
    assert np.abs(w0).max() <= a0
    # variance of U[-a,a] is a^2/3
    assert abs(w0.var() - a0 * a0 / 3) < 0.1 * a0 * a0 / 3
