"""Pose-conditioned deformation network, FP64 (test infrastructure only).

Paper definitions followed (Sec. 4.2, hybrid deformation; widths in Sec. 4.3):

* a residual delta_v = MLP([hash(v_t), theta]) is added to the point,
  v_c = v_t + delta_v;
* the network input is the 32-wide hash encoding of v_t and the 72-wide pose
  theta; 4 hidden layers of 128 units.

Readings where the paper is silent:

* the encoding is a multiresolution hash grid of its own (16 levels x 2
  features, the field's ladder), delegated to Instant-NGP like the fields';
* the layers are bias-free, ReLU on the hidden layers, a linear 3-wide output
  (as the fields' networks); parameters are one flat vector, each layer's
  W[out][in] row-major, shapes 104 -> 128 -> 128 -> 128 -> 128 -> 3;
* the pose is one 72-vector per call (all points of a frame share it);
* gradients: to the parameters, to the deformation table (through the
  encoding), to the points (through the encoding, plus the identity of the
  residual) and to the pose (summed over the points).
"""
from __future__ import annotations

import numpy as np

from . import grid

N_FEAT, N_POSE, WIDTH, N_HIDDEN = 32, 72, 128, 4


def layer_shapes(n_in=N_FEAT + N_POSE, width=WIDTH, n_hidden=N_HIDDEN):
    shapes = [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(3, width)]
    return shapes


def split(params, shapes):
    out, o = [], 0
    for r, c in shapes:
        out.append(np.asarray(params[o:o + r * c], np.float64).reshape(r, c))
        o += r * c
    return out


def forward(params, x, theta, table, lay, shapes=None):
    """Returns (v_c [n][3], cache)."""
    shapes = shapes or layer_shapes()
    Ws = split(params, shapes)
    x = np.asarray(x, np.float64)
    feat = grid.encode(x, table, lay)
    h = np.concatenate([feat, np.broadcast_to(np.asarray(theta, np.float64),
                                              (len(x), len(theta)))], 1)
    acts = [h]
    for W in Ws[:-1]:
        h = np.maximum(h @ W.T, 0.0)
        acts.append(h)
    dv = h @ Ws[-1].T
    return x + dv, dict(x=x, acts=acts, Ws=Ws, table=table, lay=lay, shapes=shapes)


def backward(cache, dvc, want_dx=True):
    """Gradients of sum(dvc . v_c): (dparams flat, dtable, dx, dtheta)."""
    dvc = np.asarray(dvc, np.float64)
    acts, Ws = cache["acts"], cache["Ws"]
    dWs = [None] * len(Ws)
    dWs[-1] = dvc.T @ acts[-1]
    dh = dvc @ Ws[-1]
    for i in range(len(Ws) - 2, -1, -1):
        dz = dh * (acts[i + 1] > 0)
        dWs[i] = dz.T @ acts[i]
        dh = dz @ Ws[i]
    dfeat = dh[:, :N_FEAT]
    dtheta = dh[:, N_FEAT:].sum(0)
    dtable, dx_enc = grid.encode_backward(cache["x"], cache["table"], dfeat, cache["lay"],
                                          want_dx=want_dx)
    dx = dvc + dx_enc if want_dx else None
    return np.concatenate([d.reshape(-1) for d in dWs]), dtable, dx, dtheta
