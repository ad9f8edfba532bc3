"""The host-side spatial-pool bookkeeping (nvr_pool_step, nvr_pool_select)
against the oracle's rules, and the key-frame entry points' argument checks
(no GPU needed: every check returns before any launch)."""
import ctypes as C

import numpy as np
import pytest

from oracle import keyframe as kf


@pytest.fixture(scope="module")
def O():
    from paper_2304_03184_amd import _lib as L, ops
    try:
        L.lib()
    except ImportError as e:  # the library is built by the build step
        pytest.skip(str(e))
    return ops


def test_pool_sequence_matches_oracle(O):
    rng = np.random.default_rng(3)
    for cap in (1, 5, 100):
        pool_o, pool_g = [], []
        for frame in range(400):
            # distances drawn around gamma, many exact ties in the replacement
            d = np.round(rng.uniform(0.0, 6.0, size=len(pool_o)), 1).astype(np.float32)
            pool_o, act, slot = kf.pool_step(pool_o, d, frame, cap=cap)
            a, s = O.pool_step(pool_g, d, frame, cap=cap)
            names = {0: "reject", 1: "first", 2: "append", 3: "replace"}
            assert (names[a], s) == (act, slot), (cap, frame)
            assert pool_g == pool_o


def test_pool_select_matches_oracle(O):
    rng = np.random.default_rng(4)
    for n in (0, 1, 7, 10, 11, 100):
        d = np.round(rng.uniform(0, 3, size=n), 1).astype(np.float32)
        pool = list(range(100, 100 + n))
        near, _ = kf.select(pool, d, [], m=10)
        assert [pool[j] for j in O.pool_select(d, m=10)] == near


def test_keyframe_entry_points_reject_bad_arguments(O):
    from paper_2304_03184_amd import _lib as L
    lib = L.lib()
    fake = C.c_void_p(4096)
    assert lib.nvr_visibility(-1, 10, fake, fake, fake, 4, 4, 0.01, fake, None) == L.NVR_EINVAL
    assert lib.nvr_visibility(1, 10, fake, fake, fake, 0, 4, 0.01, fake, None) == L.NVR_EINVAL
    assert lib.nvr_visibility(1, 10, fake, fake, fake, 4, 4, -1.0, fake, None) == L.NVR_EINVAL
    assert lib.nvr_visibility(1, 10, None, fake, fake, 4, 4, 0.01, fake, None) == L.NVR_EINVAL
    assert lib.nvr_visibility(1, 10, C.c_void_p(4098), fake, fake, 4, 4, 0.01, fake,
                              None) == L.NVR_EINVAL
    assert lib.nvr_visibility(0, 10, None, None, None, 4, 4, 0.01, None, None) == L.NVR_OK
    assert lib.nvr_human_distance(5, 72, 32, fake, None, fake, fake, fake, 0, fake, 0.01, 0.02,
                                  fake, None, None) == L.NVR_EINVAL
    assert lib.nvr_human_distance(5, 5000, 32, fake, fake, fake, fake, fake, 0, fake, 0.01, 0.02,
                                  fake, None, None) == L.NVR_EINVAL
    assert lib.nvr_object_distance(5, fake, None, fake, 0, 1.0, 0.02, fake, None) == L.NVR_EINVAL
    assert lib.nvr_depth_assemble(-1, fake, fake, fake, fake, fake, fake, fake, fake,
                                  None) == L.NVR_EINVAL
    assert lib.nvr_depth_assemble(5, fake, fake, None, fake, fake, fake, fake, fake,
                                  None) == L.NVR_EINVAL
    n = C.c_int32(3)
    pool = (C.c_int32 * 2)()
    act, slot = C.c_int32(), C.c_int32()
    assert lib.nvr_pool_step(pool, C.byref(n), 2, None, 0, 2.5, C.byref(act),
                             C.byref(slot)) == L.NVR_EINVAL          # n_pool > cap
