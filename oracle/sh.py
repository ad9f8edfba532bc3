"""Real spherical harmonics of the view direction (test infrastructure only).

The colour network of each field takes the view direction (Sec. 4.2 delegates
the networks to Instant-NGP, whose colour network consumes a spherical-harmonics
encoding of the direction).  The paper does not state the encoding; the reading
taken: real, orthonormal SH on the unit sphere, ordered by band l = 0, 1, ...
and within a band by m = -l..l, with "degree d" meaning the d bands l < d
(d*d coefficients: 4 for d = 2, 16 for d = 4).  Sign convention: the standard
real basis Y_l^m = sqrt(2) (-1)^m Im / Re of the complex Y_l^|m| (which
carries the Condon-Shortley phase), so that Y_1 = sqrt(3/(4 pi)) (y, z, x).

The direction is used as given (unit length by construction).
"""
from __future__ import annotations

import math

import numpy as np


def sh_encode(d, degree: int):
    """d (n,3) -> (n, degree*degree) float64."""
    if not 1 <= degree <= 4:
        raise ValueError("degree must be in 1..4")
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [np.full_like(x, 0.5 * math.sqrt(1.0 / pi))]
    if degree > 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [c1 * y, c1 * z, c1 * x]
    if degree > 2:
        c2 = 0.5 * math.sqrt(15.0 / pi)
        out += [c2 * x * y,
                c2 * y * z,
                0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
                c2 * x * z,
                0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if degree > 3:
        a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        b = 0.5 * math.sqrt(105.0 / pi)
        c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        e = 0.25 * math.sqrt(7.0 / pi)
        g = 0.25 * math.sqrt(105.0 / pi)
        out += [a * y * (3.0 * x * x - y * y),
                b * x * y * z,
                c * y * (5.0 * z * z - 1.0),
                e * z * (5.0 * z * z - 3.0),
                c * x * (5.0 * z * z - 1.0),
                g * z * (x * x - y * y),
                a * x * (x * x - 3.0 * y * y)]
    return np.stack(out, axis=1)
