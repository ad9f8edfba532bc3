"""Pins of the FP64 hybrid-warp oracle."""
import numpy as np
import pytest

import synth
from oracle import warp

LO, HI = (-1.0,) * 3, (1.0,) * 3


@pytest.fixture(scope="module")
def rig():
    return synth.human_rig(synth.rng_for(30), n_nodes=256, knn_res=16)


def live_points(rig, rng, n):
    p = rig["node_live"][0][rng.integers(0, rig["node_live"].shape[1], n)]
    return (p + rng.normal(scale=0.03, size=p.shape)).astype(np.float32)


def identity_rig(rig):
    r = dict(rig)
    F, J = rig["bones"].shape[:2]
    b = np.zeros_like(rig["bones"])
    b[..., 0, 0] = b[..., 1, 1] = b[..., 2, 2] = 1.0
    r["bones"] = b
    dq = np.zeros_like(rig["node_dq"])
    dq[..., 0] = 1.0
    r["node_dq"] = dq
    return r


def test_identity_bones_and_nodes(rig):
    x = live_points(rig, synth.rng_for(31), 200)
    z = warp.warp(x, identity_rig(rig), LO, HI)
    np.testing.assert_allclose(z, x.astype(np.float64), rtol=0, atol=1e-15)


def test_equal_nodes_give_exact_inverse_rigid_motion(rig):
    # all nodes share one rigid motion: the blend is that motion whatever the
    # weights, and its conjugate is the inverse motion.
    rng = synth.rng_for(32)
    r = identity_rig(rig)
    ang = 0.3
    axis = np.array([0.2, -0.5, 0.8])
    axis /= np.linalg.norm(axis)
    qr = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * axis])
    T = np.array([0.03, -0.02, 0.05])
    qd = 0.5 * warp.qmul(np.concatenate([[0.0], T]), qr)
    r["node_dq"] = np.broadcast_to(np.concatenate([qr, qd]), rig["node_dq"].shape).copy()
    x = live_points(rig, rng, 100)
    z = warp.warp(x, r, LO, HI)
    # forward motion of z must give back x
    back = warp.dq_apply(np.concatenate([qr, qd])[None, :], z)
    np.testing.assert_allclose(back, x.astype(np.float64), atol=1e-14)
    # the inverse motion in matrix form: R^T (x - T)
    import scipy.spatial.transform as sst
    Rm = sst.Rotation.from_quat([*qr[1:], qr[0]]).as_matrix()
    np.testing.assert_allclose(z, (x.astype(np.float64) - T) @ Rm, atol=1e-14)


def test_identical_bones_are_a_rigid_map(rig):
    r = dict(identity_rig(rig))
    import scipy.spatial.transform as sst
    Rm = sst.Rotation.from_rotvec([0.1, 0.4, -0.2]).as_matrix()
    t = np.array([0.05, 0.0, -0.1])
    r["bones"] = np.broadcast_to(np.concatenate([Rm, t[:, None]], 1),
                                 rig["bones"].shape).copy()
    x = live_points(rig, synth.rng_for(33), 100)
    z = warp.warp(x, r, LO, HI)
    np.testing.assert_allclose(z, x.astype(np.float64) @ Rm.T + t, atol=1e-14)


def test_antipodal_node_quaternions_change_nothing(rig):
    # dq and -dq are the same rigid motion; the sign alignment must absorb it
    x = live_points(rig, synth.rng_for(34), 300)
    z0 = warp.warp(x, rig, LO, HI)
    r = dict(rig)
    dq = rig["node_dq"].copy()
    flip = synth.rng_for(35).uniform(size=dq.shape[1]) < 0.5
    dq[:, flip] *= -1
    r["node_dq"] = dq
    z1 = warp.warp(x, r, LO, HI)
    np.testing.assert_allclose(z1, z0, atol=1e-14)


def test_blend_is_rigid_and_weight_scale_invariant(rig):
    x = live_points(rig, synth.rng_for(36), 100)
    z, C = warp.warp(x, rig, LO, HI, want_cache=True)
    c = C["c"]
    assert np.allclose(np.linalg.norm(c[:, :4], axis=1), 1.0, atol=1e-15)
    # rotation part: R^T R = I, det R = 1
    e = np.eye(3)
    cols = np.stack([warp.qrot(c[:, :4], np.broadcast_to(e[k], (100, 3))) for k in range(3)], 2)
    np.testing.assert_allclose(np.einsum("nab,nac->nbc", cols, cols),
                               np.broadcast_to(e, (100, 3, 3)), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(cols), 1.0, atol=1e-14)
    # the unshifted weights exp(-|y-g|^2/r^2) give the same point
    w = np.exp(-((C["y"][:, None, :] - C["g"]) ** 2).sum(-1) / warp.R_ED ** 2)
    b = np.einsum("nk,nkc->nc", C["s"] * w, C["conj"])
    z2 = warp.dq_apply(b / np.linalg.norm(b[:, :4], axis=1, keepdims=True), C["y"])
    np.testing.assert_allclose(z2, z, atol=1e-13)


def test_forward_blend_then_inverse_round_trip_equal_nodes(rig):
    # Eq. 1 forward (canonical -> live) followed by the inverse warp returns
    # the canonical point when all nodes share a motion (identity bones).
    rng = synth.rng_for(37)
    r = identity_rig(rig)
    qr = np.array([np.cos(0.1), 0.0, np.sin(0.1), 0.0])
    qd = 0.5 * warp.qmul(np.array([0.0, 0.01, 0.02, -0.03]), qr)
    dq = np.concatenate([qr, qd])
    r["node_dq"] = np.broadcast_to(dq, rig["node_dq"].shape).copy()
    vc = rng.uniform(-0.3, 0.3, size=(50, 3))
    w = np.exp(-((vc[:, None, :] - rig["node_canon"][None, :8].astype(float)) ** 2).sum(-1)
               / 0.01)
    blend = np.einsum("nk,c->nc", w, dq)
    blend /= np.linalg.norm(blend[:, :4], axis=1, keepdims=True)
    v_live = warp.dq_apply(blend, vc).astype(np.float32)
    z = warp.warp(v_live, r, LO, HI)
    np.testing.assert_allclose(z, warp.dq_apply(np.broadcast_to(warp.qconj(qr).tolist() + warp.qconj(qd).tolist(), (50, 8)), v_live.astype(float)), atol=1e-14)
    np.testing.assert_allclose(z, vc, atol=1e-6)   # float32 rounding of v_live


def test_lut_voxel_and_joint_choice_are_float32_decisions():
    x = np.array([[0.0, 0.0, 0.0], [-1.0, 0.999999, 0.5]], np.float32)
    v = warp.lut_voxel(x, LO, HI, 16)
    assert v[0] == 8 + 16 * (8 + 16 * 8)
    assert v[1] == 0 + 16 * (15 + 16 * 12)
    J = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 2, 0], [0, 0, 3]], np.float32)
    sel = warp.nearest_joints(np.array([[0.0, 0.0, 0.0]], np.float32), J, 3)
    assert sel[0].tolist() == [0, 1, 2]      # tie between 1 and 2 -> lower first


def test_backward_vs_fd(rig):
    rng = synth.rng_for(38)
    x = live_points(rig, rng, 40)
    gz = rng.normal(size=(40, 3))
    d_dq, d_bones = warp.warp_backward(x, rig, LO, HI, gz)

    def L(r):
        return np.sum(warp.warp(x, r, LO, HI) * gz)
    touched = np.argwhere(np.abs(d_dq[0]).sum(1) > 0)[:, 0]
    assert touched.size > 8
    h = 1e-6
    for node in rng.choice(touched, 6, replace=False):
        for c in range(8):
            rp, rm = dict(rig), dict(rig)
            rp["node_dq"] = rig["node_dq"].astype(np.float64).copy()
            rm["node_dq"] = rig["node_dq"].astype(np.float64).copy()
            rp["node_dq"][0, node, c] += h
            rm["node_dq"][0, node, c] -= h
            fd = (L(rp) - L(rm)) / (2 * h)
            assert abs(fd - d_dq[0, node, c]) < 1e-6 * max(1, abs(fd)), (node, c)
    tj = np.argwhere(np.abs(d_bones[0]).sum((1, 2)) > 0)[:, 0]
    for j in tj[:4]:
        for a in range(3):
            for b in range(4):
                rp, rm = dict(rig), dict(rig)
                rp["bones"] = rig["bones"].astype(np.float64).copy()
                rm["bones"] = rig["bones"].astype(np.float64).copy()
                rp["bones"][0, j, a, b] += h
                rm["bones"][0, j, a, b] -= h
                fd = (L(rp) - L(rm)) / (2 * h)
                assert abs(fd - d_bones[0, j, a, b]) < 1e-6 * max(1, abs(fd)), (j, a, b)


def _tiny_rig(joints, bones, node_pos, node_dq, knn_ids):
    """A rig with a 1^3 look-up grid listing ``knn_ids`` for every live point."""
    return dict(joints=np.asarray(joints, np.float64),
                bones=np.asarray(bones, np.float64)[None],
                node_dq=np.asarray(node_dq, np.float64)[None],
                node_pos=np.asarray(node_pos, np.float64)[None],
                knn=np.asarray(knn_ids, np.uint16).reshape(1, 1, -1))


def _translation_bone(t):
    b = np.zeros((3, 4))
    b[0, 0] = b[1, 1] = b[2, 2] = 1.0
    b[:, 3] = t
    return b


def test_backward_position_gradient_vs_fd(rig):
    # dL/dx through the skinning blend (bones and skin weights) and the node
    # weights, against central differences in float64 (steps small enough that
    # no float32 joint or voxel choice changes)
    rng = synth.rng_for(39)
    x = live_points(rig, rng, 30).astype(np.float64)
    gz = rng.normal(size=(30, 3))
    _, _, gx = warp.warp_backward(x, rig, LO, HI, gz, want_dx=True)
    h = 1e-7
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h
        xm[:, a] -= h
        fd = np.sum((warp.warp(xp, rig, LO, HI) - warp.warp(xm, rig, LO, HI)) * gz, 1) / (2 * h)
        np.testing.assert_allclose(gx[:, a], fd, rtol=1e-6, atol=1e-6)
    # identity rig: z = x, so dx = gz exactly
    ident = dict(rig)
    ident["bones"] = np.tile(np.eye(3, 4), (1, rig["bones"].shape[1], 1, 1))
    dq = np.zeros_like(rig["node_dq"], dtype=np.float64)
    dq[..., 0] = 1.0
    ident["node_dq"] = dq
    _, _, gx0 = warp.warp_backward(x, ident, LO, HI, gz, want_dx=True)
    np.testing.assert_allclose(gx0, gz, rtol=0, atol=1e-12)


def test_skin_weights_hand_worked():
    # Inverse skinning with the Gaussian weights over the 4 nearest joints,
    # sigma_s = 0.1: the live point sits at the origin, joints at distances
    # 0.1, 0.2, 0.3, 0.4 and 0.5 (the last is not among the 4 nearest), every
    # bone a pure translation.  With d^2 = 0.01, 0.04, 0.09, 0.16 the exponents
    # -(d^2 - d_min^2) / (2 sigma_s^2) are 0, -1.5, -4, -7.5, so the normalised
    # weights are e^0, e^-1.5, e^-4, e^-7.5 over their sum (worked by hand):
    #   0.8051537029216888, 0.17965407467701772,
    #   0.014746904472640808, 0.0004453179286526382.
    # Translations (1,0,0), (0,1,0), (0,0,1), (1,1,1) and (5,5,5) then give
    # y = (w0 + w3, w1 + w3, w2 + w3); the single identity node leaves it.
    joints = [[0.1, 0, 0], [0, 0.2, 0], [0, 0, -0.3], [0.4, 0, 0], [0, 0.5, 0]]
    ts = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [5, 5, 5]]
    rig = _tiny_rig(joints, [_translation_bone(t) for t in ts], [[0.0, 0.0, 0.0]],
                    [[1, 0, 0, 0, 0, 0, 0, 0]], [0])
    z = warp.warp(np.zeros((1, 3), np.float32), rig, LO, HI)
    want = [0.8055990208503414, 0.18009939260567034, 0.015192222401293446]
    np.testing.assert_allclose(z[0], want, rtol=0, atol=1e-15)
    # a width of sigma_s^2 instead of 2 sigma_s^2 would give (0.950..., 0.0497..., ...)
    assert abs(z[0, 0] - 0.95) > 0.1


def test_inverse_node_blend_unequal_translations_hand_worked():
    # Eq. 4 with the node weight of Sec. 4.1 (r = 0.1) at the post-skinning
    # point y (identity bones, so y = x = (0.03, 0, 0)) against two deformed
    # nodes g_A = (0, 0, 0) and g_B = (0.1, 0, 0) moving by pure translations
    # t_A = (0.02, 0, 0) and t_B = (0, 0.04, 0).  The weights are
    # exp(-|y - g|^2 / r^2) = e^-0.09 and e^-0.49, normalised 0.598687660112452
    # and 0.401312339887548; the blend of the conjugated (inverse) motions is the
    # inverse translation by the weighted mean, so
    #   z = y - (w_A t_A + w_B t_B) / (w_A + w_B)
    #     = (0.01802624679775096, -0.016052493595501923, 0)   (worked by hand).
    eye = _translation_bone([0, 0, 0])
    dq_a = [1, 0, 0, 0, 0, 0.01, 0, 0]           # dual part t/2 for a pure translation
    dq_b = [1, 0, 0, 0, 0, 0, 0.02, 0]
    rig = _tiny_rig([[0.0, 0.0, 0.0]], [eye], [[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]],
                    [dq_a, dq_b], [0, 1])
    z = warp.warp(np.array([[0.03, 0.0, 0.0]], np.float32), rig, LO, HI, k_joints=1)
    x0 = float(np.float32(0.03))                 # the live point as float32
    want = [x0 - 0.03 + 0.01802624679775096, -0.016052493595501923, 0.0]
    np.testing.assert_allclose(z[0], want, rtol=0, atol=2e-9)
    # weights exp(-d^2 / r) (r instead of r^2) would move z[1] to about -0.0196
    assert abs(z[0, 1] + 0.0196) > 1e-3
