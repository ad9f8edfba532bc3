"""Occupancy-grid maintenance, FP64 (test infrastructure only).

The fields are trained on Instant-NGP's back-end (Sec. 4.3, Sec. 5), whose
occupancy bitfield lets the marcher skip empty space; the paper leaves its
upkeep to that back-end and states none of it.  The reading taken is the
published density grid of Instant-NGP at one scale:

* a density grid g of res^3 cells, indexed like the bitfield
  (vx + res * (vy + res * vz));
* an update first decays every cell, g <- lambda g (lambda = 0.95), then, for
  each probe i (a cell c_i and a position p_i inside it, both drawn by the
  caller), sets g[c_i] <- max(g[c_i], sigma(p_i)), sigma being the field's
  density at p_i (the density network of the training step,
  sigma = exp(clamp(o_0)); the view direction does not enter it);
* a cell is occupied iff g[c] > tau = min(tau_max, mean(g)), with
  tau_max = 0.01 * 1024 / sqrt(3): the density at which one step of
  sqrt(3)/1024 reaches optical thickness 0.01;
* the bitfield holds cell c at bit c & 31 of 32-bit word c >> 5, the layout the
  marcher reads.

Only fields without a warp are covered: a human field's occupancy lives in the
live space, where the density needs the warp of the frame.
"""
from __future__ import annotations

import numpy as np

from . import grid, network, sh

DECAY = 0.95
TAU_MAX = 0.01 * 1024.0 / np.sqrt(3.0)


def density(fcfg, table, params, x):
    """The field's density sigma at positions x [n][3] (world), float64."""
    lay = grid.Layout.from_field(fcfg)
    feat = grid.encode(np.asarray(x, np.float64), np.asarray(table, np.float64), lay)
    # any direction: sigma comes from the density network alone
    dirs = np.zeros((feat.shape[0], 3))
    dirs[:, 2] = 1.0
    sigma, _, _ = network.forward(fcfg, np.asarray(params, np.float64), feat,
                                  sh.sh_encode(dirs, fcfg.sh_degree))
    return sigma


def decay_and_max(g, cells, sigma, decay=DECAY):
    """lambda * g, then the running maximum of the probes' densities per cell."""
    out = np.asarray(g, np.float64) * decay
    np.maximum.at(out, np.asarray(cells, np.int64), np.asarray(sigma, np.float64))
    return out


def threshold(g, tau_max=TAU_MAX):
    """Occupancy threshold min(tau_max, mean(g))."""
    return min(float(tau_max), float(np.mean(np.asarray(g, np.float64))))


def pack_bits(occupied):
    """bool [n_cells] -> uint32 words, cell c at bit c & 31 of word c >> 5."""
    occupied = np.asarray(occupied, bool).ravel()
    words = np.zeros((occupied.size + 31) // 32, np.uint32)
    idx = np.nonzero(occupied)[0]
    np.bitwise_or.at(words, idx >> 5, np.left_shift(np.uint32(1), (idx & 31).astype(np.uint32)))
    return words


def update(fcfg, table, params, g, cells, points, decay=DECAY, tau_max=TAU_MAX):
    """One grid update.  Returns (new grid, tau, bitfield words, probe densities)."""
    sigma = density(fcfg, table, params, points)
    g2 = decay_and_max(g, cells, sigma, decay)
    tau = threshold(g2, tau_max)
    return g2, tau, pack_bits(g2 > tau), sigma
