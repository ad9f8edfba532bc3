"""Pins of the occupancy-grid maintenance oracle (oracle/occupancy.py)."""
import math

import numpy as np

import synth
from oracle import grid, march, network, occupancy, sh


def _rng(k):
    return np.random.default_rng(7100 + k)


def test_decay_and_max_matches_brute_force():
    rng = _rng(0)
    g = rng.uniform(0, 3, size=4096)
    cells = rng.integers(0, 4096, size=3000)          # many repeated cells
    sigma = rng.uniform(0, 5, size=3000)
    got = occupancy.decay_and_max(g, cells, sigma, decay=0.9)
    want = 0.9 * g.copy()
    for c, s in zip(cells.tolist(), sigma.tolist()):
        if s > want[c]:
            want[c] = s
    np.testing.assert_array_equal(got, want)


def test_repeated_decay_closed_form():
    g = _rng(1).uniform(0, 10, size=1000)
    out = g.copy()
    for _ in range(7):
        out = occupancy.decay_and_max(out, [], [], decay=occupancy.DECAY)
    np.testing.assert_allclose(out, g * occupancy.DECAY ** 7, rtol=1e-14, atol=0)


def test_threshold_is_min_of_cap_and_mean():
    assert math.isclose(occupancy.TAU_MAX, 5.9120668, rel_tol=1e-7)   # 10.24 / 1.7320508
    small = np.array([0.0, 1.0, 2.0, 5.0])
    assert occupancy.threshold(small) == 2.0
    big = np.full(10, 100.0)
    assert occupancy.threshold(big) == occupancy.TAU_MAX
    assert occupancy.threshold(big, tau_max=1e9) == 100.0


def test_bitfield_is_the_marchers_layout():
    # a marcher reading the packed bits keeps exactly the dense samples whose
    # voxel is occupied in the boolean grid the bits were packed from
    rng = _rng(3)
    res = 32
    occ = rng.random(res ** 3) < 0.3
    words = occupancy.pack_bits(occ)
    assert words.dtype == np.uint32 and words.size == res ** 3 // 32
    o, d = synth.sphere_rays(300, rng)
    lo, hi = np.full(3, -1.0), np.full(3, 1.0)
    delta = math.sqrt(3) * 2 / 128
    kept = march.march(o, d, lo, hi, 0.0, 1e9, delta, 128, occ_words=words, occ_res=res)
    full = march.march(o, d, lo, hi, 0.0, 1e9, delta, 128)
    sc = march.occ_scale(res, lo, hi)
    u = (full["x"] - np.asarray(lo, np.float32)[None, :]) * sc[None, :]
    v = np.clip(np.floor(u), 0, res - 1).astype(np.int64)
    keep = occ[v[:, 0] + res * (v[:, 1] + res * v[:, 2])]
    np.testing.assert_array_equal(kept["t"], full["t"][keep])
    np.testing.assert_array_equal(kept["ray"], full["ray"][keep])


def test_density_closed_form_and_direction_independence():
    w = synth.config(1)
    f = w.fields[0]
    lay = grid.Layout.from_field(f)
    rng = _rng(4)
    table = synth.uniform_table(lay.n_entries, f.n_features, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    x = rng.uniform(-1.4, 1.4, size=(200, 3))
    # all-zero weights: o_0 = 0 everywhere, so sigma = exp(0) = 1
    np.testing.assert_array_equal(occupancy.density(f, table, np.zeros_like(params), x), 1.0)
    # the direction does not enter the density
    dirs = rng.normal(size=(200, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    s_any, _, _ = network.forward(f, params, grid.encode(x, table, lay),
                                  sh.sh_encode(dirs, f.sh_degree))
    np.testing.assert_allclose(occupancy.density(f, table, params, x), s_any, rtol=1e-15)


def test_update_is_consistent():
    w = synth.config(1)
    f = w.fields[0]
    lay = grid.Layout.from_field(f)
    rng = _rng(5)
    table = synth.uniform_table(lay.n_entries, f.n_features, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    res = 16
    g = rng.uniform(0, 2, size=res ** 3)
    cells = rng.integers(0, res ** 3, size=500)
    points = rng.uniform(-1.4, 1.4, size=(500, 3))
    g2, tau, words, sigma = occupancy.update(f, table, params, g, cells, points)
    probed = np.zeros(res ** 3, bool)
    probed[cells] = True
    np.testing.assert_array_equal(g2[~probed], occupancy.DECAY * g[~probed])
    assert np.all(g2[probed] >= occupancy.DECAY * g[probed])
    assert np.all(g2[cells] >= sigma)
    assert tau == min(occupancy.TAU_MAX, g2.mean())
    bits = (words[np.arange(res ** 3) >> 5] >> (np.arange(res ** 3) & 31).astype(np.uint32)) & 1
    np.testing.assert_array_equal(bits.astype(bool), g2 > tau)
