"""Steady frictionless flow on a radially symmetric surface (Sec. 3.2.1), test infrastructure.

The paper compares with an exact steady solution from a cited paper that is not here.  This
module writes out what mass and energy conservation alone fix for a steady radial flow
without friction or rain: the discharge per radian r h v is constant (K = r_in h0 v0 from
the inflow edge) and so is the head v^2/2 + g (h + f(r)) (E from the inflow state).  At each
r this leaves v^2/2 + g K / (r v) = E - g f(r), whose larger root is the supercritical branch
the inflow (Froude 1.43) starts on.  Only the tests use this module.
"""
from __future__ import annotations

import math

import numpy as np


def bed(meta, r):
    """f(r) of eq. eq_function_fr."""
    m = meta
    return m["A"] + m["s"] * m["A"] * np.cos(math.pi * (np.asarray(r) - m["r0"]) / (m["r1"] - m["r0"]))


def steady(meta, r):
    """(h, v) of the steady supercritical solution at radii r (v along the flow)."""
    g, h0, v0, rin = meta["g"], meta["h0"], meta["v0"], meta["r_in"]
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    K = rin * h0 * v0
    E = 0.5 * v0 * v0 + g * (h0 + float(bed(meta, rin)))
    rhs = E - g * bed(meta, r)

    def F(v):  # head at discharge K minus the available head; increasing for v > vc
        return 0.5 * v * v + g * K / (r * v) - rhs

    vc = (g * K / r) ** (1.0 / 3.0)  # the head's minimum over v: critical flow
    if np.any(F(vc) > 0):
        raise ValueError("no steady supercritical flow at some radius")
    lo = vc.copy()
    hi = np.maximum(2.0 * vc, np.sqrt(2.0 * np.maximum(rhs, 0.0)) + 1.0)
    while np.any(F(hi) < 0):
        hi = np.where(F(hi) < 0, 2.0 * hi, hi)
    for _ in range(200):  # bisection on [vc, hi]
        mid = 0.5 * (lo + hi)
        below = F(mid) < 0
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    v = 0.5 * (lo + hi)
    return K / (r * v), v
