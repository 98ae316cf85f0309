"""Pins of the linear soil resistance and the Thacker test (Sec. 3.2.2, Appendix B).

The exact solution is checked against the shallow-water equations it must satisfy (not
against its own formulas): each velocity component is a damped oscillator, the level at the
bowl's centre moves as the mass balance of a planar surface demands, and the water volume
(closed form for a planar surface over a paraboloid) stays constant.  The oracle's linear
resistance is pinned by the implicit decay of a uniform flow, and the oracle's Thacker run
by the exact solution at the paper's resolution, against the paper's error figures.
No GPU needed.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.thacker import Thacker, surface_error
from tests._util import ref_run

# error ||((h+z)_app - (h+z)_ex) / (h+z)_ex||_inf the paper reports at these times on its
# 487 123-cell mesh of 0.888231 m cells (Sec. 3.2.2, figure of the four snapshots)
PAPER_ERR = {10.0: 0.0107, 30.0: 0.0102, 70.0: 0.0122, 330.0: 0.0045}
# The bound is the paper's figure, except at t = 10 s: the front still moves fast there,
# the maximum sits in a front cell, and our mesh (same cell size, its own placement) puts
# the front up to one cell away (about 0.45 m of depth on that slope), so three times it.
ERR_FACTOR = {10.0: 3.0, 30.0: 1.0, 70.0: 1.0, 330.0: 1.0}
VEL_REL = 0.05  # mean velocity of the wet cells against the exact (uniform) velocity


@pytest.fixture(scope="module")
def exact():
    return Thacker(synth.thacker().meta)


def _d(f, t, e=1e-4):
    return (f(t + e) - f(t - e)) / (2 * e)


def _d2(f, t, e=1e-3):
    return (f(t + e) - 2 * f(t) + f(t - e)) / (e * e)


def test_exact_velocity_is_a_damped_oscillator(exact):
    g, tau, m = exact.m["g"], exact.m["tau"], exact.m
    for ax, c, v0, dv0 in ((exact.ax, m["A"], m["u0"], m["du0"]), (exact.ay, m["B"], m["v0"], m["dv0"])):
        assert ax.v(0.0) == pytest.approx(v0, abs=1e-12)
        assert ax.dv(0.0) == pytest.approx(dv0, rel=1e-12)
        assert _d(ax.v, 3.0) == pytest.approx(ax.dv(3.0), rel=1e-6)
        # mass balance of a planar surface over the paraboloid: V'' + tau V' + 2 g c V = 0
        for t in (0.5, 5.0, 20.0):
            res = _d2(ax.v, t) + tau * ax.dv(t) + 2.0 * g * c * ax.v(t)
            assert abs(res) <= 1e-5 * (abs(_d2(ax.v, t)) + abs(ax.dv(t)) + 1e-6)


def test_exact_level_and_volume_follow_the_mass_balance(exact):
    g, tau, m = exact.m["g"], exact.m["tau"], exact.m

    def level(t):
        return exact.level_at_centre(t)

    def K(t):  # level of the apex after completing the squares: volume = pi K^2 / (2 sqrt(AB))
        su = tau * exact.ax.v(t) + exact.ax.dv(t)
        sv = tau * exact.ay.v(t) + exact.ay.dv(t)
        return level(t) + su * su / (4.0 * m["A"] * g * g) + sv * sv / (4.0 * m["B"] * g * g)

    assert level(0.0) == m["w0"]
    for t in (0.3, 4.0, 25.0, 100.0):
        u, v = exact.velocity(t)
        su = tau * u + exact.ax.dv(t)
        sv = tau * v + exact.ay.dv(t)
        # constant part of w_t + v . grad(w - z) = 0 on the wet region
        assert _d(level, t) == pytest.approx((u * su + v * sv) / g, rel=1e-5, abs=1e-9)
        assert K(t) == pytest.approx(K(0.0), rel=1e-12)
    # the raster's own volume agrees with the closed form at t = 0
    sc = synth.thacker(a=0.5)
    x, y = synth.centres(sc.nq, sc.nr, sc.a)
    sigma = 1.5 * math.sqrt(3.0) * sc.a ** 2
    vol = sigma * exact.depth(0.0, x + sc.meta["ox"], y + sc.meta["oy"]).sum()
    assert vol == pytest.approx(math.pi * K(0.0) ** 2 / (2 * math.sqrt(m["A"] * m["B"])), rel=2e-3)


def test_linear_resistance_decays_a_uniform_flow_implicitly():
    """A uniform flow on a flat periodic raster has no edge sums, so each step is the
    implicit decay v^{n+1} = v^n / (1 + dt tau) of the linear resistance alone."""
    nq, nr, tau, dt, n = 12, 10, 0.7, 0.05, 20
    N = nq * nr
    P = oracle.PERIODIC
    sc = synth.Scenario(name="decay", nq=nq, nr=nr, a=1.0, z=np.zeros(N), theta=np.ones(N),
                        alpha_p=np.zeros(N), alpha_s=0.0, side=(P, P, P, P), h0=np.full(N, 0.5),
                        v10=np.full(N, 0.3), v20=np.full(N, -0.2), dt_max=dt, tau_lin=tau,
                        t_end=n * dt)
    r = ref_run(sc, max_steps=n)
    assert r["books"]["steps"] == n
    f = (1.0 + dt * tau) ** n
    np.testing.assert_allclose(r["v1"], 0.3 / f, rtol=1e-12)
    np.testing.assert_allclose(r["v2"], -0.2 / f, rtol=1e-12)
    np.testing.assert_allclose(r["h"], 0.5, rtol=1e-13)
    # without the resistance nothing decays
    r0 = ref_run(synth.Scenario(**{**sc.__dict__, "tau_lin": 0.0}), max_steps=n)
    np.testing.assert_allclose(r0["v1"], 0.3, rtol=1e-13)


@pytest.mark.parametrize("t", [10.0, 30.0])
def test_oracle_thacker_against_the_exact_solution(exact, t):
    sc = synth.thacker(t_end=t)
    x, y = synth.centres(sc.nq, sc.nr, sc.a)
    x, y = x + sc.meta["ox"], y + sc.meta["oy"]
    r = ref_run(sc, nthreads=8)
    err = surface_error(r["h"], sc.z, exact.depth(t, x, y))
    wet = r["h"] > 0.1
    u, v = exact.velocity(t)
    print(f"[thacker oracle t={t:g}] err {err:.4f} (paper {PAPER_ERR[t]}), u {r['v1'][wet].mean():.4f} "
          f"({u:.4f}), v {r['v2'][wet].mean():.4f} ({v:.4f}), steps {r['books']['steps']}", flush=True)
    assert err <= ERR_FACTOR[t] * PAPER_ERR[t]
    assert abs(r["v1"][wet].mean() - u) <= VEL_REL * math.hypot(u, v)
    assert abs(r["v2"][wet].mean() - v) <= VEL_REL * math.hypot(u, v)
    # closed walls, no rain: the water volume is kept up to the clamp tally
    b = r["books"]
    assert b["outflow"] == 0.0 and b["rain"] == 0.0
    assert b["stored"] == pytest.approx(b["initial"] + b["clamp"], rel=1e-12)
