"""Infiltration in the mass source (the paper's future extension by an algebraic law, Sec. 4;
the scalar equation for h^{n+1} of Appendix A) in the oracle.

With i(h) = f h / (h + c) taken at h^{n+1}, a still, flat, closed lake obeys the implicit
Euler step of theta h' = r - i(h). Pins: one step solves its scalar equation to rounding;
the deep-water limit drops the depth by dt f / theta; many steps follow the exact solution of
the ODE, theta [(h - h0) + c ln(h / h0)] = -f t, at first order in dt; under rain r < f the
depth settles at the equilibrium r c / (f - r); the books close with the soil's water booked
as outflow; f = 0 changes nothing.
"""
import math

import numpy as np
import pytest

import oracle
import synth

F, C_INF, TH = 1e-5, 0.01, 0.8


def _lake(h0=0.05, n=6, cfl=0.5, f=F, c=C_INF, rain=0.0, theta=TH, dt_max=1.0):
    G = oracle.grid(n, n, 1.0, (synth.WALL,) * 4)
    N = n * n
    p = oracle.params(cfl=cfl, dt_max=dt_max, f_inf=f, h_inf=c)
    r = oracle.rain(0, rain, 0.0, float("inf"))
    return G, p, r, np.zeros(N), np.full(N, theta), np.full(N, h0)


def _run(G, p, r, z, th, h, t_end, max_steps=10 ** 9):
    N = G.n
    return oracle.run(G, z, th, np.zeros(N), p, r, h, np.zeros(N), np.zeros(N), t_end,
                      max_steps=max_steps, nthreads=4)


def test_one_step_solves_the_scalar_equation():
    G, p, r, z, th, h = _lake()
    hn, v1, v2, b, _ = _run(G, p, r, z, th, h, 1e9, max_steps=1)
    dt = b.t
    x = hn[0]
    assert np.all(hn == x) and np.all(v1 == 0) and np.all(v2 == 0)
    assert TH * x + dt * F * x / (x + C_INF) == pytest.approx(TH * 0.05, rel=1e-15)
    # the water that left went into the soil, booked with the outflow
    sigma = 1.5 * math.sqrt(3.0)
    assert b.outflow == pytest.approx(G.n * sigma * TH * (0.05 - x), rel=1e-12)
    assert b.residual < 1e-14


def test_deep_water_infiltrates_at_the_full_rate():
    G, p, r, z, th, h = _lake(h0=5.0, c=1e-6)
    hn, _, _, b, _ = _run(G, p, r, z, th, h, 1e9, max_steps=1)
    assert 5.0 - hn[0] == pytest.approx(b.t * F / TH, rel=1e-6)


def _exact_depth(t, h0=0.05):
    """h(t) of theta h' = -f h / (h + c): theta [(h - h0) + c ln(h / h0)] = -f t."""
    target = -F * t / TH
    lo, hi = 1e-12, h0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (mid - h0) + C_INF * math.log(mid / h0) > target:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def test_many_steps_follow_the_exact_decay_at_first_order():
    """Implicit Euler: the error at t = 3600 s halves with the step (Courant 0.8 vs 0.4)."""
    T = 3600.0
    exact = _exact_depth(T)
    errs = []
    for cfl in (0.8, 0.4):
        G, p, r, z, th, h = _lake(cfl=cfl)
        hn, _, _, b, _ = _run(G, p, r, z, th, h, T)
        errs.append((hn[0] - exact) / exact)
        assert b.residual < 1e-12
    assert abs(errs[0]) < 1e-3
    assert errs[1] / errs[0] == pytest.approx(0.5, abs=0.05)


def test_rain_and_infiltration_reach_their_equilibrium():
    rain = 0.4 * F
    G, p, r, z, th, h = _lake(h0=0.0, rain=rain)
    hn, _, _, b, _ = _run(G, p, r, z, th, h, 30000.0)
    assert hn[0] == pytest.approx(rain * C_INF / (F - rain), rel=1e-3)
    assert b.residual < 1e-12


def test_zero_rate_changes_nothing():
    sc = synth.c1_planar(nq=24, nr=20, t_end=60.0)
    from tests._util import ref_run
    a = ref_run(sc, nthreads=4)
    sc.f_inf, sc.h_inf = 0.0, 0.01
    b = ref_run(sc, nthreads=4)
    np.testing.assert_array_equal(a["h"], b["h"])
    np.testing.assert_array_equal(a["v1"], b["v1"])
