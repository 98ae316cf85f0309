"""Given-mass-flux boundary cells, the flume of Sec. 3.3.2 and the sensitivity measures of
Sec. 3.4 in the oracle.

Pins: the flux edge's mass and momentum after one step against their closed forms; the
bare flume at its normal depth (the friction law's uniform flow) staying uniform; the
vegetated flume reaching the normal depth of its vegetated reach; delta_s and delta_p
against a grid on which hbar is linear in the coefficients.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.flume import hbar, normal_depth, sensitivities
from tests._util import ref_grid, ref_params, ref_rain, ref_run


def _channel(h_cells, v_flux, h_flux, nq=8, nr=6, a=1.0):
    """A flat frictionless channel fed through a column of flux cells at q = 0."""
    act = np.ones(nq * nr, np.uint8)
    act.reshape(nr, nq)[:, 0] = 3
    h = np.full(nq * nr, float(h_cells))
    v1 = np.zeros(nq * nr)
    h.reshape(nr, nq)[:, 0] = h_flux
    v1.reshape(nr, nq)[:, 0] = v_flux
    G = oracle.grid(nq, nr, a, (synth.WALL,) * 4, (), act, synth.WALL)
    return G, h, v1


@pytest.mark.parametrize("h_cells", [0.0, 0.5])
def test_flux_edge_one_step_closed_form(h_cells):
    """Each cell of column q = 1 (away from the walls) takes the discharge h_F v_F across its
    W edge and half of it across its NW edge, whatever depth it holds, and the momentum
    flux with it; the pressure term of a flux edge sees the cell's own depth, so on a flat
    bed it vanishes.  Without friction the first column then holds
    m1 = m + dt/sigma * 1.5 l h_F v_F and v1 = dt/sigma * 1.5 l h_F v_F^2 / m1."""
    nq, nr, a, hF, vF = 8, 6, 1.0, 0.1, 0.2
    G, h, v1 = _channel(h_cells, vF, hF, nq, nr, a)
    n = nq * nr
    p = oracle.params(cfl=0.5)
    hn, v1n, v2n, b, _ = oracle.run(G, np.zeros(n), np.ones(n), np.zeros(n), p, oracle.rain(),
                                    h, v1, np.zeros(n), t_end=1e9, max_steps=1)
    sigma = 1.5 * math.sqrt(3.0) * a * a
    c = max(vF + math.sqrt(9.81 * hF), math.sqrt(9.81 * h_cells))
    dt = 0.5 * (sigma / (6 * a)) / c
    assert b.t == pytest.approx(dt, rel=1e-15)
    H, V = hn.reshape(nr, nq), v1n.reshape(nr, nq)
    m1 = h_cells + dt / sigma * 1.5 * a * hF * vF
    for r in range(nr - 1):  # the top row's NW edge is a wall
        assert H[r, 1] == pytest.approx(m1, rel=1e-13)
        assert V[r, 1] == pytest.approx(dt / sigma * 1.5 * a * hF * vF * vF / m1, rel=1e-12)
    assert np.all(H[:, 2:] == h_cells) and np.all(V[:, 2:] == 0.0)
    np.testing.assert_array_equal(H[:, 0], hF)  # held
    assert np.all(v2n == 0.0)  # the momentum flux carries v_F, which has no y part


def test_bare_flume_at_normal_depth_stays_uniform():
    """The friction law's uniform flow (g h m = alpha_s v^2 on bare soil) is steady: the
    flume fed with q at its normal depth keeps that depth and velocity away from the ends
    and the wall rows (which see no pressure term across the walls)."""
    q, m = 0.007, 0.00105
    hn = normal_depth(q, 1.0, m, synth.ALPHA_S, synth.ALPHA_P)
    assert 9.81 * hn * m == pytest.approx(synth.ALPHA_S * (q / hn) ** 2, rel=1e-12)
    sc = synth.flume(q=q, h_in=hn, theta_v=1.0, m=m, a=0.1, t_end=60.0)
    st = ref_run(sc, nthreads=8)
    x = sc.meta["x"]
    row = np.repeat(np.arange(sc.nr), sc.nq)
    mid = (sc.active == 1) & (x > 3) & (x < 12) & (row > 0) & (row < sc.nr - 1)
    assert np.abs(st["h"][mid] / hn - 1).max() < 0.015
    assert np.abs(st["v1"][mid] * hn / q - 1).max() < 0.03


def test_vegetated_flume_reaches_the_vegetated_normal_depth():
    """With vegetation on the lower half (theta_1) and the viscous flux on, the steady depth
    over the vegetated zone is the normal depth of the vegetated reach (the free outflow
    keeps it there); the books balance to rounding."""
    q, m, tv = 0.021, 0.00105, 0.99364
    hv = normal_depth(q, tv, m, synth.ALPHA_S, synth.ALPHA_P)
    sc = synth.flume(q=q, h_in=hv, theta_v=tv, m=m, a=0.1, t_end=150.0)
    sc.visc = True
    st = ref_run(sc, nthreads=8)
    assert hbar(sc.meta["veg_zone"], st["h"]) == pytest.approx(hv, rel=0.01)
    b = st["books"]
    assert b["residual"] < 1e-12


def test_without_the_viscous_flux_the_flume_does_not_settle():
    """The reading that turns the augmented flux on for the flume: without it the low-friction
    subcritical flow keeps sloshing at q = 21 l/s."""
    q, m, tv = 0.021, 0.00105, 0.99364
    hv = normal_depth(q, tv, m, synth.ALPHA_S, synth.ALPHA_P)
    sc = synth.flume(q=q, h_in=hv, theta_v=tv, m=m, a=0.1)
    G, P, R = ref_grid(sc), ref_params(sc), ref_rain(sc)
    h, v1, v2, b = sc.h0, sc.v10, sc.v20, None
    seen = []
    for t in (50.0, 100.0, 150.0, 200.0):
        h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, P, R, h, v1, v2, t, books=b,
                                     t0=b.t if b else 0.0, nthreads=8)
        seen.append(hbar(sc.meta["veg_zone"], h))
    assert max(abs(s / hv - 1) for s in seen) > 0.05


def test_sensitivities_of_a_linear_hbar_are_its_slopes():
    a_s = 0.00709 * np.array([0.8, 0.9, 1.0, 1.1])
    a_p = 73.39 * np.array([0.9, 1.0, 1.1])
    H = 0.05 + 3.0 * a_s[:, None] + 1e-4 * a_p[None, :]
    d_s, d_p = sensitivities(H, a_s[1] - a_s[0], a_p[1] - a_p[0])
    assert d_s == pytest.approx(3.0, rel=1e-9)
    assert d_p == pytest.approx(1e-4, rel=1e-9)
    # a 2 x 2 grid by hand: delta_s averages the two columns' differences
    d_s, d_p = sensitivities([[1.0, 2.0], [4.0, 8.0]], 0.5, 2.0)
    assert d_s == pytest.approx(((4 - 1) + (8 - 2)) / 2 / 0.5)
    assert d_p == pytest.approx(((2 - 1) + (8 - 4)) / 2 / 2.0)
