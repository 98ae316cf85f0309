"""Exact solution of the non-oscillating Thacker problem (Appendix B), test infrastructure.

A planar free surface over the paraboloid z = A (x-x0)^2 + B (y-y0)^2 with theta = 1, no
rain and a linear soil resistance -tau h v: the velocity is uniform in space and each of its
components obeys a damped linear oscillator whose roots are real when
tau^2 - 8 g A > 0 and tau^2 - 8 g B > 0 (the non-oscillating case).  Only the tests and the
bench's checks use this module.
"""
from __future__ import annotations

import math

import numpy as np


class Axis:
    """One velocity component (Appendix B): V(t) = A1 e^{l1 t} + A2 e^{l2 t} with
    l1,2 = (-tau -+ sqrt(D)) / 2, D = tau^2 - 8 g c (c: the bed's curvature along the axis),
    A1 = (V0 l2 - V0') / sqrt(D), A2 = -(V0 l1 - V0') / sqrt(D)."""

    def __init__(self, g, tau, c, v0, dv0):
        D = tau * tau - 8.0 * g * c
        if not D > 0.0:
            raise ValueError("oscillating case: tau^2 - 8 g c must be > 0")
        sd = math.sqrt(D)
        self.g, self.tau = g, tau
        self.l1, self.l2 = (-tau - sd) / 2.0, (-tau + sd) / 2.0
        self.c1 = (v0 * self.l2 - dv0) / sd
        self.c2 = -(v0 * self.l1 - dv0) / sd

    def v(self, t):
        return self.c1 * math.exp(self.l1 * t) + self.c2 * math.exp(self.l2 * t)

    def dv(self, t):
        return self.c1 * self.l1 * math.exp(self.l1 * t) + self.c2 * self.l2 * math.exp(self.l2 * t)

    def W(self, t):
        """This axis's share of the surface level at the bowl's centre, W0(t) of Appendix B."""
        l1, l2, c1, c2, tau = self.l1, self.l2, self.c1, self.c2, self.tau
        return (c1 * c1 * (l2 / l1) * (1.0 - math.exp(2.0 * l1 * t))
                + c2 * c2 * (l1 / l2) * (1.0 - math.exp(2.0 * l2 * t))
                + 2.0 * c1 * c2 * (1.0 - math.exp(-tau * t))) / (2.0 * self.g)


class Thacker:
    """The exact state at time t from the problem's parameters (synth.thacker's meta)."""

    def __init__(self, meta):
        m = meta
        self.m = m
        self.ax = Axis(m["g"], m["tau"], m["A"], m["u0"], m["du0"])
        self.ay = Axis(m["g"], m["tau"], m["B"], m["v0"], m["dv0"])

    def level_at_centre(self, t):
        return self.m["w0"] + self.ax.W(t) + self.ay.W(t)

    def velocity(self, t):
        return self.ax.v(t), self.ay.v(t)

    def surface(self, t, x, y):
        """w(t, x, y): planar, tilted by the velocity and its rate of change."""
        m, g, tau = self.m, self.m["g"], self.m["tau"]
        u, du = self.ax.v(t), self.ax.dv(t)
        v, dv = self.ay.v(t), self.ay.dv(t)
        return (self.level_at_centre(t) - (x - m["x0"]) * (tau * u + du) / g
                - (y - m["y0"]) * (tau * v + dv) / g)

    def bed(self, x, y):
        m = self.m
        return m["A"] * (x - m["x0"]) ** 2 + m["B"] * (y - m["y0"]) ** 2

    def depth(self, t, x, y):
        return np.maximum(self.surface(t, x, y) - self.bed(x, y), 0.0)


def surface_error(h, z, h_exact):
    """The paper's error measure: max over cells of |(h+z)_app - (h+z)_ex| / (h+z)_ex."""
    ex = h_exact + z
    return float(np.max(np.abs((h + z) - ex) / ex))
