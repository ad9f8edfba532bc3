"""Pins of the deformation-network oracle (oracle/deform.py)."""
import numpy as np
import torch

from oracle import deform, grid


def _setup(seed, n=64, log2_table=14):
    rng = np.random.default_rng(seed)
    lay = grid.Layout(16, 2, log2_table, 16, 512, (-1.0,) * 3, (1.0,) * 3)
    table = rng.uniform(-0.5, 0.5, size=(lay.n_entries, 2))
    shapes = deform.layer_shapes()
    params = np.concatenate([rng.uniform(-1, 1, size=r * c) * np.sqrt(6.0 / (r + c))
                             for r, c in shapes])
    x = rng.uniform(-0.9, 0.9, size=(n, 3))
    theta = rng.normal(scale=0.3, size=72)
    return rng, lay, table, shapes, params, x, theta


def test_shapes_and_parameter_count():
    shapes = deform.layer_shapes()
    assert shapes == [(128, 104), (128, 128), (128, 128), (128, 128), (3, 128)]
    assert sum(r * c for r, c in shapes) == 104 * 128 + 3 * 128 * 128 + 3 * 128


def test_network_matches_torch_autograd():
    rng, lay, table, shapes, params, x, theta = _setup(0)
    vc, cache = deform.forward(params, x, theta, table, lay)
    dvc = rng.normal(size=vc.shape)
    dparams, dtable, dx, dtheta = deform.backward(cache, dvc)
    # an independent formulation: torch.nn.functional.linear / relu, autograd
    feat = torch.tensor(grid.encode(x, table, lay), dtype=torch.float64, requires_grad=True)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    Ws, o = [], 0
    for r, c in shapes:
        Ws.append(torch.tensor(params[o:o + r * c].reshape(r, c), dtype=torch.float64,
                               requires_grad=True))
        o += r * c
    h = torch.cat([feat, th.expand(len(x), 72)], 1)
    for W in Ws[:-1]:
        h = torch.nn.functional.relu(torch.nn.functional.linear(h, W))
    out = torch.tensor(x) + torch.nn.functional.linear(h, Ws[-1])
    np.testing.assert_allclose(out.detach().numpy(), vc, rtol=1e-12, atol=1e-12)
    (out * torch.tensor(dvc)).sum().backward()
    ref = np.concatenate([W.grad.numpy().reshape(-1) for W in Ws])
    np.testing.assert_allclose(dparams, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dtheta, th.grad.numpy(), rtol=1e-10, atol=1e-12)
    ref_dtable, _ = grid.encode_backward(x, table, feat.grad.numpy(), lay, want_dx=False)
    np.testing.assert_allclose(dtable, ref_dtable, rtol=1e-10, atol=1e-12)


def test_position_gradient_by_finite_differences():
    rng, lay, table, shapes, params, x, theta = _setup(1, n=8)
    vc, cache = deform.forward(params, x, theta, table, lay)
    dvc = rng.normal(size=vc.shape)
    _, _, dx, _ = deform.backward(cache, dvc)
    h = 1e-7
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h
        xm[:, a] -= h
        fp = np.sum(deform.forward(params, xp, theta, table, lay)[0] * dvc, 1)
        fm = np.sum(deform.forward(params, xm, theta, table, lay)[0] * dvc, 1)
        np.testing.assert_allclose(dx[:, a], (fp - fm) / (2 * h), rtol=1e-4, atol=1e-6)


def test_zero_output_layer_is_the_identity():
    rng, lay, table, shapes, params, x, theta = _setup(2)
    params[-3 * 128:] = 0.0
    vc, cache = deform.forward(params, x, theta, table, lay)
    np.testing.assert_array_equal(vc, x)
    dvc = rng.normal(size=vc.shape)
    dparams, dtable, dx, dtheta = deform.backward(cache, dvc)
    np.testing.assert_array_equal(dx, dvc)
    assert not dtable.any() and not dtheta.any()
    assert dparams[-3 * 128:].any() and not dparams[:-3 * 128].any()
