"""Pins of the key-frame selection and assembly oracle (oracle/keyframe.py)."""
import numpy as np

import synth
from oracle import keyframe as kf


def _camera(i=1, n=4, w=64, h=48, f=60.0):
    R, c = synth.look_at_cameras(n, radius=2.0)[i]
    K = np.array([[f, 0.0, w / 2], [0.0, -f, h / 2], [0.0, 0.0, 1.0]])
    P = K @ np.concatenate([R.T, (-R.T @ c)[:, None]], 1)
    return R, c, P, w, h, f


def test_visibility_matches_the_pixel_rays_camera():
    # nodes placed along the rays of chosen pixels (synth's own pinhole model)
    # project back into those pixels at their camera depth
    R, c, P, w, h, f = _camera()
    rng = np.random.default_rng(0)
    pix = rng.choice(w * h, size=200, replace=False)
    o, d = synth.pixel_rays(R, c, w, h, f, pix)
    s = rng.uniform(0.5, 3.0, size=len(pix))
    nodes = o.astype(np.float64) + s[:, None] * d.astype(np.float64)
    z = s * (d.astype(np.float64) @ R[:, 2])                 # camera depth
    depth = np.full((h, w), 9.0, np.float32)
    depth.reshape(-1)[pix] = z.astype(np.float32)
    assert kf.visibility(nodes, P, depth).all()
    # 2 eps behind or in front of the stored depth: hidden
    assert not kf.visibility(o + (s + 0.03)[:, None] * d, P, depth).any()
    assert not kf.visibility(o + (s - 0.03)[:, None] * d, P, depth).any()
    # behind the camera: never visible, whatever the map holds
    back = o - s[:, None] * d
    assert not kf.visibility(back, P, np.full((h, w), -1.0, np.float32)).any()


def test_visibility_outside_the_image():
    R, c, P, w, h, f = _camera()
    # a ray through the pixel column just right of the image
    u = np.array([w + 0.5, -0.5, 10.5, 10.5])
    v = np.array([10.5, 10.5, h + 0.5, -0.5])
    dc = np.stack([(u - w / 2) / f, -(v - h / 2) / f, np.ones(4)], 1)
    nodes = c + 1.5 * (dc @ R.T)
    assert not kf.visibility(nodes, P, np.full((h, w), 1.5, np.float32)).any()


def test_pack_bits_and_xor_count():
    rng = np.random.default_rng(1)
    for m in (1, 31, 32, 33, 1024, 1000):
        b = rng.uniform(size=m) < 0.4
        pad = np.zeros((m + 31) // 32 * 32, bool)
        pad[:m] = b
        ref = np.packbits(pad, bitorder="little").view("<u4")
        np.testing.assert_array_equal(kf.pack_bits(b), ref)
        b2 = rng.uniform(size=m) < 0.6
        assert kf.xor_count(kf.pack_bits(b), kf.pack_bits(b2)) == int(np.sum(b != b2))


def test_human_distance_terms():
    rng = np.random.default_rng(2)
    th = rng.normal(size=72)
    bits = kf.pack_bits(rng.uniform(size=1024) < 0.5)
    assert kf.human_distance(th, th, bits, bits, 7, 7) == 0.0
    b2 = bits.copy()
    b2[5] ^= np.uint32(1 << 7)
    assert abs(kf.human_distance(th, th, bits, b2, 7, 7) - 0.01) < 1e-15
    assert abs(kf.human_distance(th, th, bits, bits, 7, 10) - 9 * 0.02) < 1e-15
    th2 = th.copy()
    th2[3 * 9 + 1] += 0.5                       # spine3: torso
    assert abs(kf.human_distance(th, th2, bits, bits, 7, 7) - 0.1 * 0.25) < 1e-15
    th3 = th.copy()
    th3[3 * 18 + 2] -= 0.5                      # left elbow: limb
    assert abs(kf.human_distance(th, th3, bits, bits, 7, 7) - 0.02 * 0.25) < 1e-15
    b = kf.beta_pose()
    assert (b == 0.1).sum() == 24 and (b == 0.02).sum() == 48
    assert kf.human_distance(th, th2, bits, b2, 3, 9) == kf.human_distance(th2, th, b2, bits, 9, 3)


def test_object_distance_terms():
    assert abs(kf.object_distance([0, 0, 0], [0.3, 0.4, 0.0], 2, 2) - 0.25) < 1e-15
    assert abs(kf.object_distance([1, 2, 3], [1, 2, 3], 0, 5) - 0.5) < 1e-15


def test_pool_admission_and_replacement():
    pool, act, slot = kf.pool_step([], [], 0, cap=3)
    assert (pool, act, slot) == ([0], "first", 0)
    pool, act, _ = kf.pool_step(pool, [2.5], 1, cap=3)         # not above gamma
    assert (pool, act) == ([0], "reject")
    pool, act, slot = kf.pool_step(pool, [2.6], 2, cap=3)
    assert (pool, act, slot) == ([0, 2], "append", 1)
    pool, act, _ = kf.pool_step(pool, [9.0, 2.4], 3, cap=3)    # close to frame 2
    assert act == "reject"
    pool, act, slot = kf.pool_step(pool, [9.0, 3.0], 4, cap=3)
    assert (pool, act, slot) == ([0, 2, 4], "append", 2)
    # full: the new frame replaces the pooled frame nearest to it
    pool, act, slot = kf.pool_step(pool, [4.0, 3.0, 5.0], 5, cap=3)
    assert (pool, act, slot) == ([0, 5, 4], "replace", 1)
    pool, act, slot = kf.pool_step(pool, [3.0, 7.0, 3.0], 6, cap=3)   # tie: lower slot
    assert (pool, act, slot) == ([6, 5, 4], "replace", 0)


def test_select_smallest_distances_and_latest():
    pool = [10, 11, 12, 13, 14]
    near, latest = kf.select(pool, [0.5, 0.2, 0.9, 0.2, 3.0], list(range(20)), m=3)
    assert near == [11, 13, 10] and latest == [17, 18, 19]


def test_assembly_rules():
    ca = np.array([[1.0, 0, 0]] * 5)
    cb = np.array([[0, 0, 1.0]] * 5)
    # a nearer; b nearer; only b covers; neither covers; equal depth (first wins)
    da = np.array([0.9, 2.0, 0.1, 0.05, 1.0])
    aa = np.array([0.9, 1.0, 0.2, 0.1, 0.5])
    db = np.array([1.8, 0.8, 1.2, 0.06, 1.0])
    ab = np.array([0.9, 0.8, 0.6, 0.2, 0.5])
    rgb, z = kf.assemble(ca, da, aa, cb, db, ab)
    np.testing.assert_allclose(rgb, [[1, 0, 0], [0, 0, 1], [0, 0, 1], [1, 0, 1], [1, 0, 0]])
    np.testing.assert_allclose(z, [1.0, 1.0, 2.0, 0.3, 2.0])
    rgb, z = kf.assemble(ca[:1], [0.0], [0.0], cb[:1], [0.0], [0.0])
    np.testing.assert_allclose(z, [0.0])
