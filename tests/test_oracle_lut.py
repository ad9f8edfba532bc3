"""Pins of the live look-up-table oracle (oracle/lut.py)."""
import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

from oracle import lut, warp

LO, HI = np.full(3, -1.0), np.full(3, 1.0)


def _nodes(rng, m=64):
    return rng.uniform(-0.9, 0.9, size=(m, 3))


def _knn(node_canon, res, k=4):
    _, ids = cKDTree(node_canon).query(lut.voxel_centres(LO, HI, res), k=k)
    return ids.astype(np.int64)


def _identity_dq(m):
    dq = np.zeros((m, 8))
    dq[:, 0] = 1.0
    return dq


def _rigid_dq(q, t):
    """Unit dual quaternion of x -> R(q) x + t (q = w, x, y, z)."""
    qd = 0.5 * warp.qmul(np.concatenate([[0.0], t]), q)
    return np.concatenate([q, qd])


def test_identity_motion_maps_every_voxel_to_itself():
    rng = np.random.default_rng(1)
    nodes = _nodes(rng)
    res = 16
    table, _, carried, _ = lut.build(LO, HI, res, _knn(nodes, res), nodes,
                                     _identity_dq(len(nodes)), LO, HI, res)
    assert carried.all()
    np.testing.assert_array_equal(table, np.arange(res ** 3))


def test_common_rigid_motion_is_exact():
    # every node with the same motion: the blend is that motion (any weights)
    rng = np.random.default_rng(2)
    nodes = _nodes(rng)
    q = Rotation.from_rotvec([0.1, -0.2, 0.15]).as_quat()      # x, y, z, w
    q = np.array([q[3], q[0], q[1], q[2]])
    t = np.array([0.05, -0.02, 0.03])
    dq = np.tile(_rigid_dq(q, t), (len(nodes), 1))
    v = lut.voxel_centres(LO, HI, 8)
    live, carried = lut.forward_dqb(v, _knn(nodes, 8), nodes, dq)
    want = Rotation.from_rotvec([0.1, -0.2, 0.15]).apply(v) + t
    np.testing.assert_allclose(live, want, rtol=0, atol=1e-12)
    # the antipodal copy of the same motion changes nothing
    dq2 = dq.copy()
    dq2[::2] *= -1.0
    live2, _ = lut.forward_dqb(v, _knn(nodes, 8), nodes, dq2)
    np.testing.assert_allclose(live2, want, rtol=0, atol=1e-12)


def test_translation_by_one_voxel_shifts_the_table():
    rng = np.random.default_rng(3)
    nodes = _nodes(rng)
    res = 16
    step = (HI[0] - LO[0]) / res
    dq = np.tile(_rigid_dq(np.array([1.0, 0, 0, 0]), np.array([step, 0.0, 0.0])), (len(nodes), 1))
    table, _, _, _ = lut.build(LO, HI, res, _knn(nodes, res), nodes, dq, LO, HI, res)
    f = np.arange(res ** 3)
    ix = f % res
    np.testing.assert_array_equal(table[ix >= 1], f[ix >= 1] - 1)
    np.testing.assert_array_equal(table[ix == 0], -1)        # holes


def test_single_listed_node_applies_its_motion():
    rng = np.random.default_rng(4)
    nodes = _nodes(rng, 5)
    q = Rotation.from_rotvec([0.0, 0.3, 0.0]).as_quat()
    q = np.array([q[3], q[0], q[1], q[2]])
    dq = _identity_dq(5)
    dq[2] = _rigid_dq(q, np.array([0.1, 0.0, -0.1]))
    v = rng.uniform(-1, 1, size=(50, 3))
    ids = np.full((50, 4), -1)
    ids[:, 0] = 2
    live, carried = lut.forward_dqb(v, ids, nodes, dq)
    assert carried.all()
    want = Rotation.from_rotvec([0.0, 0.3, 0.0]).apply(v) + np.array([0.1, 0.0, -0.1])
    np.testing.assert_allclose(live, want, rtol=0, atol=1e-12)
    none = np.full((3, 4), -1)
    _, c2 = lut.forward_dqb(v[:3], none, nodes, dq)
    assert not c2.any()


def test_assembly_keeps_the_largest_index_and_drops_outsiders():
    u = np.array([[0.5, 0.5, 0.5],      # k = 0 -> live voxel 0
                  [1.2, 0.1, 0.9],      # k = 1 -> live voxel 1
                  [0.9, 0.2, 0.7],      # k = 2 -> live voxel 0 (collides with k = 0)
                  [-0.1, 0.5, 0.5],     # k = 3 -> outside
                  [1.5, 1.5, 1.5],      # k = 4 -> live voxel 7, but not carried
                  [1.999, 1.5, 1.0]])   # k = 5 -> live voxel 7
    carried = np.array([True, True, True, True, False, True])
    table = lut.assemble(u, carried, 2)
    np.testing.assert_array_equal(table, [2, 1, -1, -1, -1, -1, -1, 5])


def test_forward_blend_unequal_translations_hand_worked():
    # Eq. 1 with w(x_i, v) = exp(-|v - x_i|^2 / r^2), r = 0.1 (Sec. 4.1): the
    # point v = (0.03, 0, 0) between two canonical nodes x_A = (0, 0, 0) and
    # x_B = (0.1, 0, 0) that move by pure translations t_A = (0.02, 0, 0) and
    # t_B = (0, 0.04, 0).  Weights e^-0.09 and e^-0.49, normalised
    # 0.598687660112452 and 0.401312339887548; a blend of pure translations is
    # the translation by their weighted mean (the real parts add to a multiple of
    # the identity), so v~ = v + (w_A t_A + w_B t_B) / (w_A + w_B)
    #   = (0.04197375320224904, 0.016052493595501923, 0)   (worked by hand).
    dq = np.array([[1, 0, 0, 0, 0, 0.01, 0, 0], [1, 0, 0, 0, 0, 0, 0.02, 0]], np.float64)
    nodes = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]])
    live, carried = lut.forward_dqb(np.array([[0.03, 0.0, 0.0]]), np.array([[0, 1]]), nodes, dq)
    assert carried[0]
    np.testing.assert_allclose(live[0], [0.04197375320224904, 0.016052493595501923, 0.0],
                               rtol=0, atol=1e-15)
    # the listed order does not matter except for the sign reference
    live2, _ = lut.forward_dqb(np.array([[0.03, 0.0, 0.0]]), np.array([[1, 0]]), nodes, dq)
    np.testing.assert_allclose(live2, live, rtol=0, atol=1e-15)
    # with exp(-d^2 / r) the weights would be nearly equal and v~_y about 0.0196
    assert abs(live[0, 1] - 0.0196) > 1e-3
