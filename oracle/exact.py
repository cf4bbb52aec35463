"""Exact rational ray-triangle arithmetic -- TEST INFRASTRUCTURE ONLY.

Pins the FP64 oracle on tiny inputs.  Every float32 input is converted to a
`fractions.Fraction` exactly, so the results below have no rounding at all.

The definition (the closest-hit outcome of section 1 of the paper, made
precise): a ray o + t d, t in the closed interval [tmin, tmax], hits the
triangle (a, b, c) when the point lies inside or on the boundary of the
triangle; the triangle is two-sided, and a ray parallel to its plane misses.
Barycentrics follow the Moller-Trumbore convention p = (1-u-v) a + u b + v c.
The closest hit is the least t; exact ties go to the lowest (instance,
primitive).

This module solves the 3x3 linear system o + t d = a + u (b-a) + v (c-a) by
Cramer's rule in exact arithmetic -- a different route from the oracle's
Moller-Trumbore code.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Optional, Sequence, Tuple

import numpy as np


def F(x) -> Fraction:
    """Exact value of a float (float32 inputs are first rounded to float32)."""
    return Fraction(float(np.float32(x)))


def _det3(c0, c1, c2):
    return (c0[0] * (c1[1] * c2[2] - c1[2] * c2[1])
            - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1])
            + c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]))


def intersect(o: Sequence, d: Sequence, a: Sequence, b: Sequence, c: Sequence,
              tmin=0, tmax=None) -> Optional[Tuple[Fraction, Fraction, Fraction]]:
    """Exact (t, u, v) of the hit, or None."""
    o, d, a, b, c = ([F(x) for x in v] for v in (o, d, a, b, c))
    e1 = [b[k] - a[k] for k in range(3)]
    e2 = [c[k] - a[k] for k in range(3)]
    s = [o[k] - a[k] for k in range(3)]
    # u e1 + v e2 - t d = s
    md = [-x for x in d]
    den = _det3(e1, e2, md)
    if den == 0:
        return None
    u = _det3(s, e2, md) / den
    v = _det3(e1, s, md) / den
    t = _det3(e1, e2, s) / den
    if u < 0 or v < 0 or u + v > 1:
        return None
    if t < F(tmin):
        return None
    if tmax is not None and np.isfinite(float(tmax)) and t > F(tmax):
        return None
    return t, u, v


def closest(o, d, tris, tmin=0, tmax=None):
    """Brute-force exact closest hit over a list of (inst, prim, a, b, c)
    already in world space.  Returns (t, inst, prim, u, v) or None."""
    best = None
    for inst, prim, a, b, c in tris:
        r = intersect(o, d, a, b, c, tmin, tmax)
        if r is None:
            continue
        key = (r[0], inst, prim)
        if best is None or key < (best[0], best[1], best[2]):
            best = (r[0], inst, prim, r[1], r[2])
    return best
