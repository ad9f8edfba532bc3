"""Live look-up table of the fast neighbour search (nvr_live_lut) against the
FP64 oracle.

The kernel forms live positions in float32, so a canonical voxel whose live
position lies within rounding distance of a live-voxel face may land on either
side: the live voxels such a voxel could reach are compared by validity (their
entry is -1 or a canonical voxel that can land there), every other live voxel
exactly."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import lut as olut

from helpers import dev, host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-3          # live-voxel units; float32 positions are good to ~1e-5 here


def _ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_03184_amd import _lib as L, ops as O
    L.lib()
    return O


def _rig(seed):
    rig = synth.human_rig(synth.rng_for(seed), knn_res=8)
    return rig["node_canon"], rig["node_dq"][0]


def _knn(node_canon, lo, hi, res, k):
    _, ids = cKDTree(node_canon.astype(np.float64)).query(olut.voxel_centres(lo, hi, res), k=k)
    return ids.astype(np.int64)


def _reachable(u, carried, res, k_sel):
    """Live voxels each canonical voxel in k_sel could reach within TOL:
    (canonical index, live index) pairs."""
    ks, fs = [], []
    for dx in (-TOL, TOL):
        for dy in (-TOL, TOL):
            for dz in (-TOL, TOL):
                c = np.floor(u[k_sel] + np.array([dx, dy, dz])).astype(np.int64)
                ok = np.all((c >= 0) & (c < res), axis=1)
                ks.append(k_sel[ok])
                fs.append(c[ok, 0] + res * (c[ok, 1] + res * c[ok, 2]))
    return np.concatenate(ks), np.concatenate(fs)


def _run(O, knn, node_canon, node_dq, cbox, cres, lbox, lres):
    ids = np.where(knn < 0, 0xFFFF, knn).astype(np.uint16).view(np.int16)
    got = O.live_lut(dev(ids), dev(node_canon.astype(np.float32)),
                     dev(node_dq.astype(np.float32)), cbox, cres, lbox, lres)
    torch.cuda.synchronize()
    return host(got).astype(np.int64)


def _compare(got, knn, node_canon, node_dq, cbox, cres, lbox, lres):
    table, u, carried, margin = olut.build(cbox[0], cbox[1], cres, knn,
                                           node_canon.astype(np.float64),
                                           node_dq.astype(np.float64), lbox[0], lbox[1], lres)
    und = np.nonzero(carried & (margin < TOL))[0]
    k_und, f_und = _reachable(u, carried, lres, und)
    unsure = np.zeros(lres ** 3, bool)
    unsure[f_und] = True
    np.testing.assert_array_equal(got[~unsure], table[~unsure])
    # every entry of an unsure live voxel is -1 or a voxel that can land there,
    # and is at least the largest decided voxel landing there
    f = np.nonzero(unsure)[0]
    g = got[f]
    possible = set(zip(k_und.tolist(), f_und.tolist()))
    dec = np.ones(len(u), bool)
    dec[und] = False
    for fi, gi, ti in zip(f, g, table[f]):
        if gi < 0:
            assert ti < 0 or not dec[ti]
        elif not dec[gi]:
            assert (gi, fi) in possible
        else:
            assert ti == gi or (ti > gi and not dec[ti])
    assert (~unsure).mean() > 0.95, (~unsure).mean()
    return table


def test_live_lut_identity_is_exact():
    O = _ops()
    node_canon, _ = _rig(1)
    dq = np.zeros((len(node_canon), 8), np.float32)
    dq[:, 0] = 1.0
    box = ((-1.0,) * 3, (1.0,) * 3)
    knn = _knn(node_canon, *box, 40, 8)
    got = _run(O, knn, node_canon, dq, box, 40, box, 40)
    np.testing.assert_array_equal(got, np.arange(40 ** 3))


@pytest.mark.parametrize("cres,lres,k", [(48, 48, 8), (40, 56, 4), (33, 17, 8)])
def test_live_lut_matches_oracle(cres, lres, k):
    O = _ops()
    node_canon, node_dq = _rig(2 + cres)
    cbox = ((-1.0,) * 3, (1.0,) * 3)
    lbox = ((-0.7, -0.9, -0.8), (0.9, 0.8, 0.75)) if lres != cres else cbox
    knn = _knn(node_canon, *cbox, cres, k)
    table = _compare(_run(O, knn, node_canon, node_dq, cbox, cres, lbox, lres),
                     knn, node_canon, node_dq, cbox, cres, lbox, lres)
    assert (table >= 0).mean() > 0.15


def test_live_lut_missing_nodes():
    # trailing "none" ids drop out of the blend; a voxel whose first id is none
    # is not carried
    O = _ops()
    node_canon, node_dq = _rig(3)
    box = ((-1.0,) * 3, (1.0,) * 3)
    res = 24
    knn = _knn(node_canon, *box, res, 8)
    rng = np.random.default_rng(5)
    knn[rng.uniform(size=knn.shape) < 0.3] = -1
    knn[:, 0] = np.where(rng.uniform(size=res ** 3) < 0.1, -1, knn[:, 0])
    _compare(_run(O, knn, node_canon, node_dq, box, res, box, res),
             knn, node_canon, node_dq, box, res, box, res)
    knn[:] = -1
    got = _run(O, knn, node_canon, node_dq, box, res, box, res)
    assert (got == -1).all()


def test_live_lut_full_size_properties():
    # 128^3 canonical and live voxels, 8 of 1024 nodes: checked on a sample of
    # canonical voxels (the oracle one by one) -- a decided voxel's live voxel
    # holds it or a larger index, and every sampled live entry names a voxel
    # that lands there
    O = _ops()
    node_canon, node_dq = _rig(4)
    box = ((-1.0,) * 3, (1.0,) * 3)
    res = 128
    knn = _knn(node_canon, *box, res, 8)
    got = _run(O, knn, node_canon, node_dq, box, res, box, res)
    rng = np.random.default_rng(6)
    k = rng.choice(res ** 3, size=20000, replace=False)
    v = olut.voxel_centres(box[0], box[1], res)[k]
    live, carried = olut.forward_dqb(v, knn[k], node_canon.astype(np.float64),
                                     node_dq.astype(np.float64))
    u = olut.live_coords(live, box[0], box[1], res)
    frac = u - np.floor(u)
    dec = carried & (np.min(np.minimum(frac, 1 - frac), axis=1) >= TOL)
    c = np.floor(u).astype(np.int64)
    inside = dec & np.all((c >= 0) & (c < res), axis=1)
    f = c[:, 0] + res * (c[:, 1] + res * c[:, 2])
    assert inside.mean() > 0.9
    assert (got[f[inside]] >= k[inside]).all()
    # sampled live entries: the named canonical voxel lands there
    f2 = rng.choice(np.nonzero(got >= 0)[0], size=20000, replace=False)
    k2 = got[f2]
    v2 = olut.voxel_centres(box[0], box[1], res)[k2]
    live2, _ = olut.forward_dqb(v2, knn[k2], node_canon.astype(np.float64),
                                node_dq.astype(np.float64))
    u2 = olut.live_coords(live2, box[0], box[1], res)
    cell = np.stack([f2 % res, (f2 // res) % res, f2 // (res * res)], 1)
    assert (np.abs(u2 - (cell + 0.5)) <= 0.5 + TOL).all()


@pytest.mark.parametrize("k", [8, 4])
def test_live_lut_load_paths_agree(k):
    # eight (four) ids per voxel in 16-byte-aligned arrays take the vector-load
    # path; the same data 2 and 4 bytes off that alignment take the element-load
    # path: the tables are identical
    O = _ops()
    node_canon, node_dq = _rig(7)
    box = ((-1.0,) * 3, (1.0,) * 3)
    res = 32
    knn = _knn(node_canon, *box, res, k)
    ids = knn.astype(np.uint16).view(np.int16)
    a = O.live_lut(dev(ids), dev(node_canon), dev(node_dq), box, res, box, res)
    kbuf = torch.zeros(ids.size + 1, dtype=torch.int16, device="cuda")
    kbuf[1:] = dev(ids.reshape(-1))
    qbuf = torch.zeros(node_dq.size + 1, dtype=torch.float32, device="cuda")
    qbuf[1:] = dev(node_dq.reshape(-1))
    b = O.live_lut(kbuf[1:].view(-1, k), dev(node_canon), qbuf[1:].view(-1, 8), box, res, box,
                   res)
    torch.cuda.synchronize()
    assert kbuf[1:].data_ptr() % 16 != 0 and qbuf[1:].data_ptr() % 16 != 0
    np.testing.assert_array_equal(host(a), host(b))


def test_live_lut_large_node_set():
    # 4000 nodes with random small motions (a node table of 176 KB, larger
    # than one workgroup's local memory)
    O = _ops()
    from scipy.spatial.transform import Rotation
    from oracle import warp as owarp
    rng = np.random.default_rng(8)
    m = 4000
    node_canon = rng.uniform(-0.9, 0.9, size=(m, 3))
    rot = Rotation.from_rotvec(rng.normal(size=(m, 3)) * 0.05).as_quat()     # x, y, z, w
    q = np.concatenate([rot[:, 3:], rot[:, :3]], 1)
    t = rng.normal(size=(m, 3)) * 0.02
    dq = np.concatenate([q, 0.5 * owarp.qmul(np.concatenate([np.zeros((m, 1)), t], 1), q)], 1)
    dq[rng.uniform(size=m) < 0.5] *= -1.0                                    # antipodal copies
    box = ((-1.0,) * 3, (1.0,) * 3)
    res = 40
    knn = _knn(node_canon, *box, res, 8)
    node_canon, dq = node_canon.astype(np.float32), dq.astype(np.float32)
    table = _compare(_run(O, knn, node_canon, dq, box, res, box, res),
                     knn, node_canon, dq, box, res, box, res)
    assert (table >= 0).mean() > 0.5
