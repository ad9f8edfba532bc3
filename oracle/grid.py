"""Multiresolution hash encoding in FP64 (test infrastructure only).

The paper extracts the features of a canonical point from a hash table H and
feeds them to the geometry and colour networks (Sec. 4.2, "Separated instant
neural representation"; the human field uses the same encoding after the warp),
delegating the encoding itself to Instant-NGP.  This module restates that
published encoding:

* level l has resolution N_l = floor(N_min * b**l), b = exp((ln N_max - ln
  N_min)/(L-1)), evaluated in float64 on the host;
* a point is normalised to x_hat in [0,1]^3 over the field's box (clamped);
  x_l = x_hat * N_l, cell c = min(floor(x_l), N_l - 1), fraction f = x_l - c;
* the 8 cell corners c + {0,1}^3 get trilinear weights prod(f or 1-f);
* a level whose (N_l+1)^3 vertices fit in T entries is indexed densely,
  idx = cx + (N_l+1)*(cy + (N_l+1)*cz); otherwise
  idx = (cx*1 xor cy*2654435761 xor cz*805459861) mod 2^32, masked to T-1;
* feat_l = sum_corners w * table_l[idx]; the output is level-major
  [level0 f0, level0 f1, level1 f0, ...].

Backward: d table_l[idx] += w * dfeat_l (the encoding is linear in the
table) and d x_hat = sum_l N_l sum_corners (dw/df) (table_l[idx] . dfeat_l);
d x = d x_hat / side where x_hat was not clamped, else 0.

Readings where the paper is silent: the level-resolution formula, no half-cell
offset, the clamp of the upper cell, the dense/hashed switch and the hash
primes above are the published Instant-NGP ones.
"""
from __future__ import annotations

import math

import numpy as np

PRIMES = (1, 2654435761, 805459861)


def level_resolutions(n_levels: int, res_min: int, res_max: int):
    """N_l = floor(N_min * b**l) in float64."""
    if n_levels == 1:
        return [int(res_min)]
    b = math.exp((math.log(res_max) - math.log(res_min)) / (n_levels - 1))
    return [int(math.floor(res_min * b ** l)) for l in range(n_levels)]


class Layout:
    """Per-level resolution, dense flag, size and offset into the table."""

    def __init__(self, n_levels, n_features, log2_table, res_min, res_max,
                 aabb_min, aabb_max):
        self.L = int(n_levels)
        self.F = int(n_features)
        self.T = 1 << int(log2_table)
        self.res = level_resolutions(n_levels, res_min, res_max)
        self.dense = [(n + 1) ** 3 <= self.T for n in self.res]
        self.size = [(n + 1) ** 3 if dn else self.T for n, dn in zip(self.res, self.dense)]
        # each level's slice starts at a multiple of 8 entries; the entries
        # between a level's last vertex and the next slice are never addressed
        self.offset = [0]
        for s in self.size:
            self.offset.append(self.offset[-1] + (s + 7) // 8 * 8)
        self.n_entries = self.offset[-1]
        self.lo = np.asarray(aabb_min, np.float64)
        self.hi = np.asarray(aabb_max, np.float64)
        self.side = self.hi - self.lo

    @classmethod
    def from_field(cls, f):
        return cls(f.n_levels, f.n_features, f.log2_table, f.res_min, f.res_max,
                   f.aabb_min, f.aabb_max)


def corner_index(level: int, c: np.ndarray, lay: Layout) -> np.ndarray:
    """Table index (within the level) of integer vertex coordinates c (...,3)."""
    n = lay.res[level]
    c = c.astype(np.uint64)
    if lay.dense[level]:
        s = np.uint64(n + 1)
        return (c[..., 0] + s * (c[..., 1] + s * c[..., 2])).astype(np.int64)
    h = (c[..., 0] * np.uint64(PRIMES[0])) ^ (c[..., 1] * np.uint64(PRIMES[1])) \
        ^ (c[..., 2] * np.uint64(PRIMES[2]))
    h = h & np.uint64(0xFFFFFFFF)
    return (h & np.uint64(lay.T - 1)).astype(np.int64)


_CORNERS = np.array([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)])


def _normalise(x, lay):
    """x - lo (float64) and whether x lies in the box (gradients flow)."""
    t = np.asarray(x, np.float64) - lay.lo
    inside = (t >= 0.0) & (t <= lay.side)
    return t, inside


def _level_terms(t, level, lay):
    # x_l = x_hat * N_l with x_hat = clamp((x - lo) / side, 0, 1), evaluated as
    # (x - lo) * N_l / side: the product is exact for float32 positions, so a
    # position exactly on a cell face gets the exact floor
    n = lay.res[level]
    xl = np.clip(t * n / lay.side, 0.0, n)
    c = np.minimum(np.floor(xl), n - 1).astype(np.int64)
    f = xl - c
    corners = c[:, None, :] + _CORNERS[None, :, :]                   # (n,8,3)
    pick = _CORNERS[None, :, :].astype(bool)
    fac = np.where(pick, f[:, None, :], 1.0 - f[:, None, :])          # (n,8,3)
    w = fac.prod(axis=2)                                              # (n,8)
    # d w / d f_a = (+1 or -1) * product of the other two factors
    sgn = np.where(pick, 1.0, -1.0)
    dw = np.empty(fac.shape)
    dw[..., 0] = sgn[..., 0] * fac[..., 1] * fac[..., 2]
    dw[..., 1] = sgn[..., 1] * fac[..., 0] * fac[..., 2]
    dw[..., 2] = sgn[..., 2] * fac[..., 0] * fac[..., 1]
    idx = corner_index(level, corners, lay) + lay.offset[level]
    return idx, w, dw


def encode(x, table, lay: Layout):
    """x (n,3) world positions, table (n_entries, F) -> feat (n, L*F)."""
    u, _ = _normalise(x, lay)
    table = np.asarray(table, np.float64)
    out = np.zeros((u.shape[0], lay.L * lay.F))
    for l in range(lay.L):
        idx, w, _ = _level_terms(u, l, lay)
        out[:, l * lay.F:(l + 1) * lay.F] = np.einsum("nk,nkf->nf", w, table[idx])
    return out


def encode_backward(x, table, dfeat, lay: Layout, want_dx=True):
    """Returns (dtable (n_entries,F), dx (n,3) or None)."""
    u, inside = _normalise(x, lay)
    table = np.asarray(table, np.float64)
    dfeat = np.asarray(dfeat, np.float64)
    dtable = np.zeros((lay.n_entries, lay.F))
    dxh = np.zeros_like(u)
    for l in range(lay.L):
        idx, w, dw = _level_terms(u, l, lay)
        g = dfeat[:, l * lay.F:(l + 1) * lay.F]                       # (n,F)
        np.add.at(dtable, idx.reshape(-1),
                  (w[:, :, None] * g[:, None, :]).reshape(-1, lay.F))
        if want_dx:
            tg = np.einsum("nkf,nf->nk", table[idx], g)               # (n,8)
            dxh += lay.res[l] * np.einsum("nka,nk->na", dw, tg)
    if not want_dx:
        return dtable, None
    dx = np.where(inside, dxh / lay.side, 0.0)
    return dtable, dx
