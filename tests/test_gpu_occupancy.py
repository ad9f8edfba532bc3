"""Occupancy-grid upkeep (nvr_occupancy_update) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import grid as ogrid, occupancy as oocc

from helpers import dev, f16_round, host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_03184_amd import _lib as L, field as F
    L.lib()
    return L, F


def _setup(seed, m):
    """Object field (16 levels, 128^3 occupancy grid), a random grid and m probes,
    each a cell and a position inside it."""
    w = synth.config(2)
    f = w.fields[0]
    rng = synth.rng_for(w.seed + 90 + seed)
    lay = ogrid.Layout.from_field(f)
    table = synth.uniform_table(lay.n_entries, f.n_features, rng)
    params = synth.xavier_params(f.layer_shapes(), rng)
    res = f.occ_res
    g = rng.uniform(0.0, 2.0, size=res ** 3).astype(np.float32)
    return w, f, rng, table, params, g


def _probes(f, rng, m):
    res = f.occ_res
    cells = rng.integers(0, res ** 3, size=m).astype(np.int32)
    v = np.stack([cells % res, (cells // res) % res, cells // (res * res)], 1)
    lo, hi = np.asarray(f.aabb_min, np.float64), np.asarray(f.aabb_max, np.float64)
    pts = lo + (v + rng.uniform(0.05, 0.95, size=(m, 3))) * (hi - lo) / res
    return cells, pts.astype(np.float32)


def _bits_of(words, n):
    c = np.arange(n)
    return ((words.view(np.uint32)[c >> 5] >> (c & 31).astype(np.uint32)) & 1).astype(bool)


def _check(f, got_g, got_tau, got_bits, ref_g, ref_tau, g_rtol, tau_rtol, band):
    n = f.occ_res ** 3
    np.testing.assert_allclose(got_g, ref_g, rtol=g_rtol, atol=1e-30)
    assert abs(got_tau - ref_tau) <= tau_rtol * ref_tau
    # the bits are the grid against the threshold: equal except where the
    # two grids sit within the comparison band of the threshold
    far = np.abs(ref_g - ref_tau) > band * ref_tau
    np.testing.assert_array_equal(_bits_of(got_bits, n)[far], (ref_g > ref_tau)[far])
    assert far.mean() > 0.95


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_occupancy_update_matches_oracle(precision):
    L, F = _lib()
    w, f, rng, table, params, g = _setup(0, 20000)
    res = f.occ_res
    fld = F.Field(w, f, table, params)
    prec = L.NVR_F32 if precision == "f32" else L.NVR_BF16
    if precision == "f32":
        o_table, o_params, g_rtol = table, params, 1e-5
    else:   # the oracle on the same fp16 table and fp16-rounded weights
        o_table = host(fld.table_half.float()).astype(np.float64)
        o_params = f16_round(params)
        g_rtol = 5e-3
    grid = dev(g)
    bits = torch.zeros((res ** 3 + 31) // 32, dtype=torch.int32, device="cuda")
    ref_g = g.astype(np.float64)
    # two updates in a row, the second with fewer probes, then one without any;
    # the first probe list also names cells outside the grid (ignored)
    for m, bad in ((20000, True), (7000, False), (0, False)):
        cells, pts = _probes(f, rng, m) if m else (np.zeros(0, np.int32), np.zeros((0, 3), np.float32))
        if bad:
            cells[:3] = [-1, res ** 3, 2 ** 31 - 1]
        tau = F.occupancy_update(fld, prec, dev(cells), dev(pts), grid, bits)
        torch.cuda.synchronize()
        ok = (cells >= 0) & (cells < res ** 3)
        if m:
            ref_g, ref_tau, _, _ = oocc.update(f, o_table, o_params, ref_g, cells[ok], pts[ok])
        else:
            ref_g = oocc.decay_and_max(ref_g, [], [])
            ref_tau = oocc.threshold(ref_g)
        _check(f, host(grid), float(host(tau)[0]), host(bits), ref_g, ref_tau,
               g_rtol, 1e-5 if precision == "f32" else 1e-4, 1e-4 if precision == "f32" else 1e-2)


def test_occupancy_update_rejects_bad_arguments():
    L, F = _lib()
    w, f, rng, table, params, g = _setup(1, 10)
    fld = F.Field(w, f, table, params)
    res = f.occ_res
    grid = dev(g)
    bits = torch.zeros((res ** 3 + 31) // 32, dtype=torch.int32, device="cuda")
    cells, pts = _probes(f, rng, 10)
    with pytest.raises(L.NvrError):
        F.occupancy_update(fld, L.NVR_F32, dev(cells), dev(pts), grid, bits, decay=1.5)
    with pytest.raises(L.NvrError):
        F.occupancy_update(fld, L.NVR_F32, dev(cells), dev(pts), grid, bits, tau_max=0.0)
