"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every declared symbol, its structures match the header's layout, and bad
descriptors are rejected before anything is launched."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from oracle import grid as ogrid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2304_03184_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libnvr.so not built")
    _lib.lib()
    return _lib


def header_functions():
    src = open(os.path.join(ROOT, "include", "nvr.h")).read()
    return sorted(set(re.findall(r"\b(nvr_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (nvr_[a-z0-9_]+)", out))
    declared = header_functions()
    assert declared, "no declarations found"
    missing = [s for s in declared if s not in exported]
    assert not missing, f"declared but not exported: {missing}"
    assert sorted(L.declared_symbols()) == declared
    for s in declared:
        getattr(L.lib(), s)


def test_struct_layout_matches_header(L, tmp_path):
    names = ["nvr_grid_desc", "nvr_march_desc", "nvr_warp_desc", "nvr_warp_rig", "nvr_mlp_desc",
             "nvr_samples", "nvr_train_state", "nvr_adam_desc", "nvr_field", "nvr_step_desc",
             "nvr_batch"]
    py = [L.GridDesc, L.MarchDesc, L.WarpDesc, L.WarpRig, L.MlpDesc, L.Samples, L.TrainState,
          L.AdamDesc, L.Field, L.StepDesc, L.Batch]
    src = tmp_path / "sz.c"
    body = "\n".join(f'printf("%zu\\n", sizeof({n}));' for n in names)
    body += '\nprintf("%zu %zu %zu\\n", offsetof(nvr_field, ray_begin), offsetof(nvr_field, occ), offsetof(nvr_step_desc, adam));'
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"nvr.h\"\nint main(void){\n"
                   + body + "\nreturn 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in vals[:len(names)]]
    assert sizes == [C.sizeof(p) for p in py]
    offs = [int(v) for v in vals[len(names):]]
    assert offs == [L.Field.ray_begin.offset, L.Field.occ.offset, L.StepDesc.adam.offset]


def test_grid_init_matches_oracle_layout(L):
    for k in (1, 2, 4):
        for f in synth.config(k).fields:
            g = L.GridDesc()
            lo = (C.c_float * 3)(*f.aabb_min)
            hi = (C.c_float * 3)(*f.aabb_max)
            L.call("nvr_grid_init", C.byref(g), f.n_levels, f.n_features, f.log2_table,
                   f.res_min, f.res_max, lo, hi)
            lay = ogrid.Layout.from_field(f)
            assert list(g.res)[:f.n_levels] == lay.res
            assert [bool(v) for v in list(g.dense)[:f.n_levels]] == lay.dense
            assert list(g.offset)[:f.n_levels + 1] == lay.offset


def test_mlp_param_count_matches_layer_shapes(L):
    for k in (1, 2):
        f = synth.config(k).fields[0]
        m = L.MlpDesc(f.enc_width, len(f.density_hidden), (C.c_int32 * 4)(*f.density_hidden),
                      f.density_out, f.sh_degree, len(f.colour_hidden),
                      (C.c_int32 * 4)(*f.colour_hidden))
        n = C.c_int64()
        L.call("nvr_mlp_param_count", C.byref(m), C.byref(n))
        assert n.value == f.n_params


def test_invalid_arguments_rejected_before_launch(L):
    lib = L.lib()
    g = L.GridDesc()
    lo = (C.c_float * 3)(-1, -1, -1)
    hi = (C.c_float * 3)(1, 1, 1)
    assert lib.nvr_grid_init(C.byref(g), 16, 3, 19, 16, 2048, lo, hi) == L.NVR_EUNSUPPORTED
    assert b"n_features" in lib.nvr_last_error()
    assert lib.nvr_grid_init(C.byref(g), 40, 2, 19, 16, 2048, lo, hi) == L.NVR_EINVAL
    assert lib.nvr_grid_init(C.byref(g), 16, 2, 19, 16, 2048, hi, lo) == L.NVR_EINVAL
    L.call("nvr_grid_init", C.byref(g), 16, 2, 19, 16, 2048, lo, hi)
    bad = L.GridDesc.from_buffer_copy(g)
    bad.offset[3] += 1
    assert lib.nvr_encode_fwd(C.byref(bad), 10, None, None, 0, None, 0, None) == L.NVR_EINVAL
    assert lib.nvr_encode_fwd(C.byref(g), -1, None, None, 0, None, 0, None) == L.NVR_EINVAL
    assert lib.nvr_encode_fwd(C.byref(g), 10, None, None, 0, None, 0, None) == L.NVR_EINVAL
    assert lib.nvr_encode_fwd(C.byref(g), 0, None, None, 0, None, 0, None) == L.NVR_OK
    m = L.MarchDesc((C.c_float * 3)(-1, -1, -1), (C.c_float * 3)(1, 1, 1), 0, 1e30, 0, 0, 0)
    assert lib.nvr_march(C.byref(m), 10, 0, 10, None, None, None, 0, None, None, None, None,
                         None, None, None, None) == L.NVR_EINVAL       # max_steps == 0
    md = L.MlpDesc(32, 1, (C.c_int32 * 4)(64), 16, 4, 2, (C.c_int32 * 4)(64, 64))
    assert lib.nvr_mlp_fwd(C.byref(md), 5, None, None, L.NVR_BF16, None, None, None,
                           L.NVR_BF16, None, None, None) == L.NVR_EINVAL  # NULL arrays
    md2 = L.MlpDesc(32, 1, (C.c_int32 * 4)(48), 16, 4, 2, (C.c_int32 * 4)(64, 64))
    assert lib.nvr_mlp_fwd(C.byref(md2), 0, None, None, L.NVR_BF16, None, None, None,
                           L.NVR_BF16, None, None, None) == L.NVR_EUNSUPPORTED
    wd = L.WarpDesc(100, 4, 0.1, 1024, 8, 1, 0.1, 128, (C.c_float * 3)(-1, -1, -1),
                    (C.c_float * 3)(1, 1, 1))
    rig = L.WarpRig(1, 1, 1, 1, 1)
    assert lib.nvr_warp_fwd(C.byref(wd), C.byref(rig), 5, None, None, None, None, None) \
        == L.NVR_EINVAL                                                # n_joints > 64
    s = L.Samples(None, None, None, None, None)
    assert lib.nvr_composite_fwd(3, C.byref(s), None, 0.0, None, None, None, None) == L.NVR_EINVAL
    assert lib.nvr_composite_fwd(3, C.byref(s), None, 1.5, None, None, None, None) == L.NVR_EINVAL
    ad = L.AdamDesc(-1.0, 0.9, 0.99, 1e-15)
    assert lib.nvr_adam(C.byref(ad), 4, None, None, None, None, 0, C.c_void_p(8), None, 0,
                        None) == L.NVR_EINVAL


def test_new_entry_points_reject_before_launch(L):
    # host-side validation of the grouped-layout encode calls, the binned
    # scatter's size limits, the random-gather probe and the occupancy upkeep:
    # each returns its status before any device work (fake pointers are never
    # touched)
    lib = L.lib()
    fake = C.c_void_p(4096)
    lo = (C.c_float * 3)(-1, -1, -1)
    hi = (C.c_float * 3)(1, 1, 1)
    g = L.GridDesc()
    L.call("nvr_grid_init", C.byref(g), 16, 2, 19, 16, 2048, lo, hi)
    assert lib.nvr_encode_fwd_grouped(C.byref(g), 10, None, fake, fake, None) == L.NVR_EINVAL
    assert lib.nvr_encode_fwd_grouped(C.byref(g), -1, fake, fake, fake, None) == L.NVR_EINVAL
    assert lib.nvr_encode_fwd_grouped(C.byref(g), 0, None, None, None, None) == L.NVR_OK
    assert lib.nvr_encode_bwd_binned_grouped(C.byref(g), 10, fake, fake, None, fake, None, fake,
                                             None) == L.NVR_EINVAL
    assert lib.nvr_encode_bwd_binned(C.byref(g), 10, fake, fake, fake, fake, None,
                                     C.c_void_p(4096 + 8), None) == L.NVR_EINVAL   # workspace alignment
    # 32 levels of 2^24 entries: more table tiles than the binned scatter holds
    big = L.GridDesc()
    L.call("nvr_grid_init", C.byref(big), 32, 2, 24, 16, 65536, lo, hi)
    assert lib.nvr_encode_bwd_binned(C.byref(big), 10, fake, fake, fake, fake, None, fake,
                                     None) == L.NVR_EUNSUPPORTED
    assert b"8192 tiles" in lib.nvr_last_error()
    assert lib.nvr_encode_bwd_binned_grouped(C.byref(big), 10, fake, fake, fake, fake, None,
                                             fake, None) == L.NVR_EUNSUPPORTED
    assert lib.nvr_encode_bwd_workspace(C.byref(g), -1) == 0
    # random-gather probe: loads a multiple of 4, a table of at least 8 words
    assert lib.nvr_probe_gather(fake, 4096, 10, 6, 1, fake, None) == L.NVR_EINVAL
    assert lib.nvr_probe_gather(fake, 64, 10, 8, 1, fake, None) == L.NVR_EINVAL
    assert lib.nvr_probe_gather(None, 4096, 10, 8, 1, fake, None) == L.NVR_EINVAL
    assert lib.nvr_probe_gather(None, 4096, 0, 8, 1, None, None) == L.NVR_OK
    # occupancy upkeep: a warped field, no occupancy grid, bad decay / tau_max
    import synth
    from paper_2304_03184_amd import ops as O
    w = synth.config(2)
    fc = w.fields[0]
    f = L.Field()
    f.grid, f.mlp, f.march = O.grid_desc_of(fc), O.mlp_desc_of(fc), O.march_desc_of(w, fc)
    f.table, f.params, f.table_half = fake, fake, fake
    assert lib.nvr_occupancy_workspace(C.byref(f), L.NVR_F32, 100) > 0
    args = (10, fake, fake, 0.95, 5.9, fake, fake, fake, fake, None)
    assert lib.nvr_occupancy_update(C.byref(f), L.NVR_F32, 10, fake, fake, 1.5, 5.9, fake, fake,
                                    fake, fake, None) == L.NVR_EINVAL
    assert lib.nvr_occupancy_update(C.byref(f), L.NVR_F32, 10, fake, fake, 0.95, 0.0, fake, fake,
                                    fake, fake, None) == L.NVR_EINVAL
    assert lib.nvr_occupancy_update(C.byref(f), L.NVR_F32, 10, None, fake, 0.95, 5.9, fake, fake,
                                    fake, fake, None) == L.NVR_EINVAL
    f.has_warp = 1
    assert lib.nvr_occupancy_update(C.byref(f), L.NVR_F32, *args) == L.NVR_EUNSUPPORTED
    assert lib.nvr_occupancy_workspace(C.byref(f), L.NVR_F32, 100) == 0
    f.has_warp = 0
    f.march.occ_res = 0
    assert lib.nvr_occupancy_update(C.byref(f), L.NVR_F32, *args) == L.NVR_EINVAL
    # live look-up table: resolutions, node counts, radius, boxes, pointers
    d = L.LutDesc()
    d.canon_min[:], d.canon_max[:] = (-1, -1, -1), (1, 1, 1)
    d.live_min[:], d.live_max[:] = (-1, -1, -1), (1, 1, 1)
    d.canon_res, d.live_res, d.k_nodes, d.n_nodes, d.r_ed = 16, 16, 4, 64, 0.1
    for field, bad in (("canon_res", 0), ("live_res", 1025), ("k_nodes", 9), ("n_nodes", 0),
                       ("n_nodes", 65536), ("r_ed", 0.0)):
        old = getattr(d, field)
        setattr(d, field, bad)
        assert lib.nvr_live_lut(C.byref(d), fake, fake, fake, fake, None) == L.NVR_EINVAL
        setattr(d, field, old)
    d.live_max[1] = -1.0
    assert lib.nvr_live_lut(C.byref(d), fake, fake, fake, fake, None) == L.NVR_EINVAL
    d.live_max[1] = 1.0
    assert lib.nvr_live_lut(C.byref(d), None, fake, fake, fake, None) == L.NVR_EINVAL
    assert lib.nvr_live_lut(C.byref(d), fake, fake, fake, C.c_void_p(4098), None) == L.NVR_EINVAL
    assert lib.nvr_live_lut(None, fake, fake, fake, fake, None) == L.NVR_EINVAL


def test_deform_and_deterministic_entry_points_reject_before_launch(L):
    # the deformation network checks the binned scatter's limits and every
    # array before its first launch; the deterministic scatter and the
    # allocation-free march reject like their counterparts (fake pointers are
    # never touched)
    lib = L.lib()
    fake = C.c_void_p(4096)
    lo = (C.c_float * 3)(-1, -1, -1)
    hi = (C.c_float * 3)(1, 1, 1)
    # 16 levels x 2 features (32 wide) hashed at 2^24 entries: more table tiles
    # than the binned scatter holds
    big = L.GridDesc()
    L.call("nvr_grid_init", C.byref(big), 16, 2, 24, 16, 65536, lo, hi)
    F32, F16 = L.NVR_F32, L.NVR_F16
    args = (C.byref(big), 10, fake, fake, fake, fake, F16, fake, fake, fake, None, None, fake,
            None)
    assert lib.nvr_deform_bwd(*args) == L.NVR_EUNSUPPORTED
    assert b"8192 tiles" in lib.nvr_last_error()
    assert lib.nvr_deform_fwd(C.byref(big), 10, fake, fake, fake, fake, F32, fake, fake,
                              None) == L.NVR_EUNSUPPORTED
    g = L.GridDesc()
    L.call("nvr_grid_init", C.byref(g), 16, 2, 14, 16, 512, lo, hi)
    assert lib.nvr_deform_bwd(C.byref(g), 10, fake, fake, fake, fake, F32, fake, fake, fake,
                              None, None, None, None) == L.NVR_EINVAL    # NULL workspace
    assert lib.nvr_deform_bwd(C.byref(g), 10, fake, fake, fake, fake, F16, fake, fake,
                              C.c_void_p(4096 + 4), None, None, fake, None) == L.NVR_EINVAL
    assert lib.nvr_deform_bwd(C.byref(g), 10, fake, fake, fake, fake, F16, fake, fake, None,
                              None, None, fake, None) == L.NVR_EINVAL    # NULL dtable
    assert lib.nvr_deform_fwd(C.byref(g), 10, fake, fake, fake, fake, L.NVR_BF16, fake, fake,
                              None) == L.NVR_EINVAL                      # math type
    assert lib.nvr_encode_bwd_deterministic(C.byref(big), 10, fake, fake, fake, fake, None, fake,
                                            None) == L.NVR_EUNSUPPORTED
    assert lib.nvr_encode_bwd_deterministic(C.byref(g), 10, fake, fake, fake, fake, None,
                                            C.c_void_p(4096 + 8), None) == L.NVR_EINVAL
    assert lib.nvr_encode_bwd_deterministic_workspace(C.byref(g), 1000) > \
        lib.nvr_encode_bwd_workspace(C.byref(g), 1000)
    md = L.MarchDesc((C.c_float * 3)(-1, -1, -1), (C.c_float * 3)(1, 1, 1), 0.0, 1e30, 0.0,
                     128, 0)
    assert lib.nvr_march_noalloc(C.byref(md), 10, 5, 3, fake, fake, None, 100, fake, fake, fake,
                                 fake, fake, fake, None) == L.NVR_EINVAL    # empty range
    md.max_steps = 0
    assert lib.nvr_march_noalloc(C.byref(md), 10, 0, 10, fake, fake, None, 100, fake, fake, fake,
                                 fake, fake, fake, None) == L.NVR_EINVAL
