"""Pins of the FP64 hash-encoding oracle against facts fixed outside it."""
import os

import numpy as np
import pytest

import synth
from oracle import grid


def small_layout(log2T=14, L=4, nmin=4, nmax=32, lo=(-1.5,) * 3, hi=(1.5,) * 3):
    return grid.Layout(L, 2, log2T, nmin, nmax, lo, hi)


def test_level_resolutions_endpoints_and_totals():
    # N_0 = N_min and N_{L-1} = N_max hold exactly for the geometric ladder
    # N_min * b^l with b = (N_max/N_min)^(1/(L-1)); float32 evaluation misses
    # the top level (511 / 2047), float64 does not.
    for L, nmin, nmax in [(8, 16, 512), (16, 16, 2048), (4, 4, 32)]:
        res = grid.level_resolutions(L, nmin, nmax)
        assert res[0] == nmin and res[-1] == nmax
        assert all(b > a for a, b in zip(res, res[1:]))
    # table sizes: dense level l holds (N_l+1)^3 entries iff that fits in T
    lay = grid.Layout.from_field(synth.config(2).fields[0])
    assert lay.dense == [True] * 5 + [False] * 11
    assert lay.size[:5] == [17 ** 3, 23 ** 3, 31 ** 3, 43 ** 3, 59 ** 3]
    # slices are padded to multiples of 8 entries: 4913 -> 4920, 12167 -> 12168,
    # 29791 -> 29792, 79507 -> 79512, 205379 -> 205384; 2^19 is already aligned
    assert lay.offset[:6] == [0, 4920, 17088, 46880, 126392, 331776]
    assert all(o % 8 == 0 for o in lay.offset)
    assert all(b - a >= s for a, b, s in zip(lay.offset, lay.offset[1:], lay.size))
    assert lay.n_entries == 331776 + 11 * 2 ** 19


def test_hash_spot_values(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "hash_spot_values.txt"), dtype=np.int64)
    for cx, cy, cz, log2T, want in rows:
        lay = grid.Layout(2, 2, int(log2T), 4096, 8192, (0,) * 3, (1,) * 3)
        assert not lay.dense[0]
        got = grid.corner_index(0, np.array([[cx, cy, cz]]), lay)[0]
        assert got == want


def test_dense_index_is_bijection():
    lay = small_layout(log2T=16)
    for l in range(lay.L):
        if not lay.dense[l]:
            continue
        n = lay.res[l] + 1
        c = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"),
                     -1).reshape(-1, 3)
        idx = grid.corner_index(l, c, lay)
        assert np.array_equal(np.sort(idx), np.arange(n ** 3))


def test_trilinear_weights_partition_of_unity():
    rng = synth.rng_for(1)
    lay = small_layout()
    x = rng.uniform(-1.5, 1.5, size=(500, 3))
    u = (x - lay.lo) / lay.side
    for l in range(lay.L):
        _, w, _ = grid._level_terms(u, l, lay)
        assert np.all(w >= 0)
        np.testing.assert_allclose(w.sum(1), 1.0, rtol=0, atol=4e-16)


def test_vertex_returns_table_entry():
    # At a grid vertex of level l the level-l feature is that vertex's entry.
    rng = synth.rng_for(2)
    lay = small_layout()
    table = rng.uniform(-0.1, 0.1, size=(lay.n_entries, 2))
    for l in range(lay.L):
        n = lay.res[l]
        c = rng.integers(0, n + 1, size=(50, 3))
        x = lay.lo + c / n * lay.side
        feat = grid.encode(x, table, lay)[:, 2 * l:2 * l + 2]
        want = table[grid.corner_index(l, c, lay) + lay.offset[l]]
        np.testing.assert_allclose(feat, want, rtol=0, atol=1e-15)


def test_dense_level_equals_scipy_trilinear():
    from scipy.interpolate import RegularGridInterpolator
    rng = synth.rng_for(3)
    lay = small_layout(log2T=16)
    table = rng.uniform(-0.1, 0.1, size=(lay.n_entries, 2))
    x = rng.uniform(-1.5, 1.5, size=(300, 3))
    feat = grid.encode(x, table, lay)
    for l in range(lay.L):
        assert lay.dense[l]
        n = lay.res[l] + 1
        vals = table[lay.offset[l]:lay.offset[l] + n ** 3].reshape(n, n, n, 2)  # [z,y,x,f]
        g = np.linspace(0.0, 1.0, n)
        u = (x - lay.lo) / lay.side
        for f in range(2):
            it = RegularGridInterpolator((g, g, g), vals[..., f], method="linear")
            want = it(u[:, ::-1])
            np.testing.assert_allclose(feat[:, 2 * l + f], want, rtol=0, atol=1e-14)


def test_table_gradient_is_the_weights_and_fd_exact():
    rng = synth.rng_for(4)
    lay = small_layout()
    table = rng.uniform(-0.1, 0.1, size=(lay.n_entries, 2))
    x = rng.uniform(-1.4, 1.4, size=(40, 3))
    dfeat = rng.normal(size=(40, lay.L * 2))
    dtab, _ = grid.encode_backward(x, table, dfeat, lay, want_dx=False)
    # finite differences in the table are exact up to rounding (linear map)
    for e in rng.choice(np.flatnonzero(np.abs(dtab).sum(1) > 0), 12, replace=False):
        for f in range(2):
            h = 1e-3
            tp = table.copy()
            tp[e, f] += h
            tm = table.copy()
            tm[e, f] -= h
            fd = (np.sum(grid.encode(x, tp, lay) * dfeat)
                  - np.sum(grid.encode(x, tm, lay) * dfeat)) / (2 * h)
            assert abs(fd - dtab[e, f]) < 1e-11


def test_position_gradient_matches_fd():
    rng = synth.rng_for(5)
    lay = small_layout()
    table = rng.uniform(-0.1, 0.1, size=(lay.n_entries, 2))
    x = rng.uniform(-1.4, 1.4, size=(30, 3))
    dfeat = rng.normal(size=(30, lay.L * 2))
    _, dx = grid.encode_backward(x, table, dfeat, lay)
    h = 1e-7
    for a in range(3):
        xp = x.copy()
        xp[:, a] += h
        xm = x.copy()
        xm[:, a] -= h
        fd = (np.sum(grid.encode(xp, table, lay) * dfeat, 1)
              - np.sum(grid.encode(xm, table, lay) * dfeat, 1)) / (2 * h)
        # rows whose +-h step crosses a cell face on some level are skipped
        ok = np.ones(30, bool)
        for l in range(lay.L):
            n = lay.res[l]
            up = (xp - lay.lo) / lay.side * n
            um = (xm - lay.lo) / lay.side * n
            ok &= np.all(np.floor(up) == np.floor(um), axis=1)
        assert ok.sum() > 20
        np.testing.assert_allclose(dx[ok, a], fd[ok], rtol=1e-6, atol=1e-8)


def test_outside_box_is_clamped_with_zero_gradient():
    rng = synth.rng_for(6)
    lay = small_layout()
    table = rng.uniform(-0.1, 0.1, size=(lay.n_entries, 2))
    x = np.array([[2.0, 0.1, 0.2], [-3.0, 0.3, -0.1]])
    xin = np.array([[1.5, 0.1, 0.2], [-1.5, 0.3, -0.1]])
    np.testing.assert_array_equal(grid.encode(x, table, lay), grid.encode(xin, table, lay))
    _, dx = grid.encode_backward(x, table, np.ones((2, lay.L * 2)), lay)
    assert dx[0, 0] == 0 and dx[1, 0] == 0
