"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints, hand-worked cases (tests/golden), closed forms, brute force on tiny
rasters, and invariants of the scheme.  None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import INTERIOR, OUTFLOW, PERIODIC, WALL
from tests._util import ref_run

SQ3 = math.sqrt(3.0)


def _setup(sc):
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    p = oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s)
    r = oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
    return G, p, r


# ---------------------------------------------------------------- P1 tables

def _brute_neighbours(nq, nr, a, perq, perr):
    """Neighbours by distance between hex centres (copies shifted by the periods)."""
    x, y = synth.centres(nq, nr, a)
    shifts = [(0.0, 0.0)]
    if perq:
        shifts += [(a * SQ3 * nq, 0.0), (-a * SQ3 * nq, 0.0)]
    if perr:
        base = list(shifts)
        for sx, sy in base:
            shifts += [(sx + a * SQ3 * nr / 2, sy + 1.5 * a * nr),
                       (sx - a * SQ3 * nr / 2, sy - 1.5 * a * nr)]
    n = nq * nr
    out = -np.ones((n, 6), np.int64)
    for i in range(n):
        for sx, sy in shifts:
            dx = x + sx - x[i]
            dy = y + sy - y[i]
            d = np.hypot(dx, dy)
            for j in np.nonzero(np.abs(d - SQ3 * a) < 1e-9 * a)[0]:
                ang = math.degrees(math.atan2(dy[j], dx[j])) % 360.0
                k = int(round(ang / 60.0)) % 6
                assert abs(ang - 60.0 * k) < 1e-6 or abs(ang - 360.0) < 1e-6
                out[i, k] = j
    return out


@pytest.mark.parametrize("nq,nr,perq,perr", [(5, 4, False, False), (7, 3, True, False),
                                             (4, 6, False, True), (5, 5, True, True),
                                             (1, 3, False, False)])
def test_tables_match_brute_force(nq, nr, perq, perr):
    side = [WALL, WALL, WALL, WALL]
    if perq:
        side[oracle.E] = side[oracle.W] = PERIODIC
    if perr:
        side[oracle.S] = side[oracle.N] = PERIODIC
    nbr, code = oracle.tables(nq, nr, side)
    bf = _brute_neighbours(nq, nr, 1.0, perq, perr)
    if (perq and nq < 3) or (perr and nr < 3):
        pytest.skip("period too short for a unique neighbour")
    np.testing.assert_array_equal(nbr, np.where(bf >= 0, bf, -1))
    np.testing.assert_array_equal(code == INTERIOR, bf >= 0)


def test_tables_side_codes_and_segments():
    """Out-of-range edges take their side's code; segments are matched on the outside position."""
    nq, nr = 6, 5
    side = (OUTFLOW, WALL, WALL, OUTFLOW)
    segs = ((oracle.S, 2, 4, WALL), (oracle.E, 1, 3, OUTFLOW))
    nbr, code = oracle.tables(nq, nr, side, segs)
    for r in range(nr):
        for q in range(nq):
            i = r * nq + q
            for k in range(6):
                qn, rn = q + oracle.DQ[k], r + oracle.DR[k]
                if rn < 0:
                    want = WALL if 2 <= qn < 4 else OUTFLOW
                elif rn >= nr:
                    want = WALL
                elif qn < 0:
                    want = OUTFLOW
                elif qn >= nq:
                    want = OUTFLOW if 1 <= rn < 3 else WALL
                else:
                    want = INTERIOR
                assert code[i, k] == want, (q, r, k)


def test_tables_mask():
    nq = nr = 9
    act = synth.hexagon_mask(nq, nr, 3)
    nbr, code = oracle.tables(nq, nr, (WALL,) * 4, active=act, mask_code=OUTFLOW)
    for i in range(nq * nr):
        if not act[i]:
            assert (code[i] == WALL).all() and (nbr[i] == -1).all()
            continue
        for k in range(6):
            j = nbr[i, k]
            if code[i, k] == INTERIOR:
                assert act[j]
            else:
                assert code[i, k] == OUTFLOW
    # the hexagonal region of radius 3 has 1 + 3*3*4 = 37 cells and 6*(2*3+1) = 42 rim edges
    assert act.sum() == 37
    n_rim = int((code[act.astype(bool)] == OUTFLOW).sum())
    assert n_rim == 6 * (2 * 3 + 1)


# -------------------------------------------------------------- P2 geometry

def test_geometry_closed_forms(golden):
    for a in (1.0, 2.0, 0.115, 0.888231):
        sigma, l, phi = oracle.geometry(a)
        assert sigma == pytest.approx(1.5 * SQ3 * a * a, rel=1e-15)
        assert l == a
        assert phi == pytest.approx(SQ3 / 4.0 * a, rel=1e-15)
    g = golden("paper_grids.txt")
    # a "radius" read as the edge length reproduces the paper's printed cell count: 487123
    # hexagons of edge 0.888231 m tile the 1000 m square of the Thacker test to 0.2 %
    # (read as the inradius, the same square would hold 365 000 cells, 25 % fewer)
    sigma, _, _ = oracle.geometry(g["thacker_radius"])
    assert g["thacker_square"] ** 2 / sigma == pytest.approx(g["thacker_cells"], rel=2e-3)
    sigma_in, _, _ = oracle.geometry(2.0 * g["thacker_radius"] / SQ3)
    assert abs(g["thacker_square"] ** 2 / sigma_in / g["thacker_cells"] - 1.0) > 0.2
    # and puts the derived 650 centres on a 1000 m row
    assert SQ3 * g["thacker_radius"] * g["thacker_row_cells"] == pytest.approx(
        g["thacker_row_length"], rel=1e-6)
    sigma, _, _ = oracle.geometry(g["radial_radius"])
    annulus = math.pi * (g["radial_r1"] ** 2 - g["radial_r0"] ** 2)
    assert g["radial_cells"] * sigma == pytest.approx(annulus, rel=0.01)


def test_normals_antisymmetric():
    for k in range(6):
        n = oracle.normal(k)
        m = oracle.normal((k + 3) % 6)
        assert n[0] == -m[0] and n[1] == -m[1]
        assert math.hypot(*n) == pytest.approx(1.0, abs=1e-16)
        assert math.degrees(math.atan2(n[1], n[0])) % 360 == pytest.approx(60.0 * k, abs=1e-12)


# ------------------------------------------------------------ P3 operators

def test_pressure_operator_linear_surface():
    """S = -sigma * theta h * grad w for a linear free surface over uniform theta h."""
    nq, nr, a, g = 5, 5, 1.3, 9.81
    G = oracle.grid(nq, nr, a)
    x, y = synth.centres(nq, nr, a)
    gx, gy = 0.013, -0.021
    z = gx * x + gy * y + 3.0
    h = np.full(nq * nr, 0.4)
    th = np.full(nq * nr, 0.7)
    zero = np.zeros(nq * nr)
    i = 2 * nq + 2
    out = oracle.cell_sums(G, g, z, th, h, zero, zero, i)
    sigma = 1.5 * SQ3 * a * a
    m = 0.7 * 0.4
    assert out[3] == pytest.approx(-sigma * m * g * gx, rel=1e-13)
    assert out[4] == pytest.approx(-sigma * m * g * gy, rel=1e-13)
    assert out[0] == 0.0 and out[1] == 0.0 and out[2] == 0.0


def test_uniform_flow_has_no_net_flux():
    nq, nr, a = 5, 5, 1.0
    G = oracle.grid(nq, nr, a)
    n = nq * nr
    out = oracle.cell_sums(G, 9.81, np.zeros(n), np.full(n, 0.6), np.full(n, 0.2),
                           np.full(n, 0.3), np.full(n, -0.7), 2 * nq + 2)
    scale = 0.6 * 0.2 * 0.76 * a
    assert abs(out[0]) < 1e-15 * scale * 10
    assert abs(out[1]) < 1e-15 * scale * 10 and abs(out[2]) < 1e-15 * scale * 10
    assert out[3] == 0.0 and out[4] == 0.0


def test_two_cell_worked_cases(golden):
    gv = golden("two_cell_edges.txt")
    G = oracle.grid(2, 1, 1.0)
    z = np.zeros(2)
    s_i = oracle.cell_sums(G, 9.81, z, [1.0, 1.0], [1.0, 0.5], [0, 0], [0, 0], 0)
    s_j = oracle.cell_sums(G, 9.81, z, [1.0, 1.0], [1.0, 0.5], [0, 0], [0, 0], 1)
    for key, val in (("L", 0), ("J1", 1), ("S1", 3)):
        assert s_i[val] == pytest.approx(gv[f"i_{key}_i"], abs=1e-15)
        assert s_j[val] == pytest.approx(gv[f"i_{key}_j"], abs=1e-15)
    assert s_i[4] == 0.0
    th = [0.8, 0.5]
    s_i = oracle.cell_sums(G, 9.81, z, th, [1.0, 0.5], [0.2, 0.1], [0, 0], 0)
    s_j = oracle.cell_sums(G, 9.81, z, th, [1.0, 0.5], [0.2, 0.1], [0, 0], 1)
    for key, val in (("L", 0), ("J1", 1), ("S1", 3)):
        assert s_i[val] == pytest.approx(gv[f"ii_{key}_i"], rel=1e-14)
        assert s_j[val] == pytest.approx(gv[f"ii_{key}_j"], rel=1e-14)


def test_flux_antisymmetry_random_state():
    """Each interior flux enters its two cells with opposite signs: sum of L is the outflow."""
    sc = synth.c1_planar(nq=9, nr=7)
    G, p, r = _setup(sc)
    h, v1, v2 = synth.random_state(sc, 3)
    tot, out = 0.0, 0.0
    for i in range(sc.n):
        s = oracle.cell_sums(G, sc.g, sc.z, sc.theta, h, v1, v2, i)
        tot += s[0]
        out += s[5]
    assert tot == pytest.approx(-out, abs=1e-14)


# ---------------------------------------------------------------- P4 mu

def test_mu_worked_case(golden):
    gv = golden("mu_solve.txt")
    m = oracle.mu(1.0, 1.0, 3.0, 4.0)
    assert m == pytest.approx(gv["mu"], rel=1e-14)
    assert m * 3.0 == pytest.approx(gv["v1"], rel=1e-14)
    assert m * 4.0 == pytest.approx(gv["v2"], rel=1e-14)


@pytest.mark.parametrize("alpha,beta,g1,g2", [(0.3, 0.0, 0.2, -0.1), (0.0, 2.0, 0.5, 0.5),
                                              (1e-3, 5.0, -0.02, 0.3), (2.0, 0.7, 0.0, 0.0)])
def test_mu_solves_the_friction_equation(alpha, beta, g1, g2):
    m = oracle.mu(alpha, beta, g1, g2)
    v = np.array([m * g1, m * g2])
    res = alpha * v + beta * np.linalg.norm(v) * v - np.array([g1, g2])
    assert np.abs(res).max() <= 1e-14 * max(1.0, abs(g1) + abs(g2))
    if beta == 0.0 and alpha > 0:
        assert m == pytest.approx(1.0 / alpha, rel=1e-15)
    if alpha == 0.0 and np.hypot(g1, g2) > 0:
        assert np.linalg.norm(v) == pytest.approx(math.sqrt(np.hypot(g1, g2) / beta), rel=1e-14)


def test_mu_zero_denominator():
    assert oracle.mu(0.0, 0.0, 0.0, 0.0) == 0.0
    assert oracle.mu(0.0, 0.0, 1.0, 0.0) == 0.0


# ----------------------------------------------------------------- P6 dt

def test_cfl_worked_case(golden):
    gv = golden("cfl_step.txt")
    nq, nr = 3, 3
    G = oracle.grid(nq, nr, 1.0)
    h = np.full(9, 0.01)
    v1 = np.zeros(9)
    v2 = np.zeros(9)
    h[4] = 0.1
    v1[4], v2[4] = 0.3, -0.4
    c = oracle.cmax(G, 9.81, np.ones(9), h, v1, v2)
    p = oracle.params(cfl=0.5, dt_max=1.0)
    assert oracle.dt(1.0, p, c, 0.0, 1e9) == pytest.approx(gv["tau"], rel=1e-15)
    assert oracle.dt(1.0, p, 0.0, 0.0, 1e9) == 1.0
    assert oracle.dt(1.0, p, c, 10.0, 10.05) == pytest.approx(0.05, rel=1e-13)


# --------------------------------------------------------- P7 / P8 books

@pytest.mark.parametrize("which", ["planar", "catchment"])
def test_mass_books_and_positivity(which):
    if which == "planar":
        sc = synth.c1_planar(t_end=200.0)
    else:
        sc = synth.catchment(48, 40, 2.0, config=2, t_end=120.0)
    G, p, r = _setup(sc)
    h, v1, v2, b, dl = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                  sc.t_end, log_dt=True)
    assert b.t == sc.t_end
    assert b.residual <= 1e-12
    assert (h >= 0).all()
    assert b.clamp <= 1e-14 * max(b.stored, 1e-300)
    assert b.rain > 0
    # the rain books are r * t * total area (constant rain)
    sigma = oracle.geometry(sc.a)[0]
    assert b.rain == pytest.approx(sc.i_a * sc.t_end * sigma * sc.n, rel=1e-12)
    assert dl.sum() == pytest.approx(sc.t_end, rel=1e-14)


def test_books_resume_is_bitwise():
    sc = synth.c1_planar(nq=16, nr=12, t_end=80.0)
    G, p, r = _setup(sc)
    args = (G, sc.z, sc.theta, sc.alpha_p, p, r)
    h1, a1, b1_, bk1, _ = oracle.run(*args, sc.h0, sc.v10, sc.v20, 80.0)
    h, a, b_, bk, _ = oracle.run(*args, sc.h0, sc.v10, sc.v20, 30.0)
    h2, a2, b2_, bk2, _ = oracle.run(*args, h, a, b_, 80.0, books=bk)
    np.testing.assert_array_equal(h1, h2)
    np.testing.assert_array_equal(a1, a2)
    assert bk1.stored == bk2.stored and bk1.steps == bk2.steps


# ---------------------------------------------------------- P9 still water

@pytest.mark.parametrize("emerged", [False, True])
def test_lake_at_rest_is_bitwise_still(emerged):
    sc = synth.lake_at_rest(emerged=emerged)
    G, p, r = _setup(sc)
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                 sc.t_end)
    assert b.steps > 10
    np.testing.assert_array_equal(h, sc.h0)
    assert (v1 == 0).all() and (v2 == 0).all()
    if emerged:
        assert (sc.h0 == 0).sum() > 10


def test_tilted_lake_moves():
    """Planted mistake check: a non-flat surface is not still (the test above is not vacuous)."""
    sc = synth.lake_at_rest()
    G, p, r = _setup(sc)
    h0 = sc.h0.copy()
    h0[5] += 1.0 / 1024
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, h0, sc.v10, sc.v20, 5.0)
    assert np.abs(v1).max() > 0


# ------------------------------------------------------- P10 symmetry

def _rot60(nq, nr):
    c = nq // 2
    idx = -np.ones(nq * nr, np.int64)
    for r in range(nr):
        for q in range(nq):
            qq, rr = q - c, r - c
            q2, r2 = -rr + c, qq + rr + c
            if 0 <= q2 < nq and 0 <= r2 < nr:
                idx[r * nq + q] = r2 * nq + q2
    return idx


@pytest.mark.parametrize("crater,rim", [(False, WALL), (True, OUTFLOW), (False, OUTFLOW)])
def test_sixfold_symmetry(crater, rim):
    sc = synth.cone(R=8, crater=crater, rim=rim, t_end=40.0)
    G, p, r = _setup(sc)
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                 sc.t_end)
    act = sc.active.astype(bool)
    rot = _rot60(sc.nq, sc.nr)
    c60, s60 = 0.5, math.sqrt(3) / 2
    src = np.nonzero(act)[0]
    dst = rot[src]
    assert (dst >= 0).all() and act[dst].all()
    hs = np.abs(h[act]).max()
    vs = np.hypot(v1, v2)[act].max()
    assert hs > 0 and vs > 0
    np.testing.assert_allclose(h[dst], h[src], rtol=0, atol=1e-12 * hs)
    np.testing.assert_allclose(v1[dst], c60 * v1[src] - s60 * v2[src], rtol=0, atol=1e-12 * vs)
    np.testing.assert_allclose(v2[dst], s60 * v1[src] + c60 * v2[src], rtol=0, atol=1e-12 * vs)


def test_symmetry_check_catches_a_broken_cone():
    """Planted mistake check: perturbing one cell breaks the symmetry test's condition."""
    sc = synth.cone(R=8, t_end=10.0)
    z = sc.z.copy()
    z[sc.nq * 10 + 10] += 0.05
    G, p, r = _setup(sc)
    h, _, _, _, _ = oracle.run(G, z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20, sc.t_end)
    act = sc.active.astype(bool)
    rot = _rot60(sc.nq, sc.nr)
    src = np.nonzero(act)[0]
    assert np.abs(h[rot[src]] - h[src]).max() > 1e-9


# --------------------------------------------------------- P11 kinematic wave

def _kinematic_depth(q, S, theta, alpha_p, alpha_s, g=9.81):
    # theta^3 g S h^3 = q^2 (alpha_p (1-theta) h + theta alpha_s), largest real root
    coeffs = [theta ** 3 * g * S, 0.0, -q * q * alpha_p * (1 - theta), -q * q * theta * alpha_s]
    roots = np.roots(coeffs)
    roots = roots[np.abs(roots.imag) < 1e-12].real
    return roots[roots > 0].max()


@pytest.mark.slow
def test_kinematic_wave_on_planar_slope():
    sc = synth.kinematic_strip(nq=6, nr=64, t_end=3600.0)
    G, p, r = _setup(sc)
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                 sc.t_end)
    H = h.reshape(sc.nr, sc.nq)
    V1 = v1.reshape(sc.nr, sc.nq)
    # (i) translation invariance along the periodic direction, exactly
    assert (H == H[:, :1]).all()
    assert np.abs(V1).max() <= 1e-15
    # (ii) steady state: every row's net outflow equals the rain on the rows above it
    sigma = oracle.geometry(sc.a)[0]
    L = np.array([oracle.cell_sums(G, sc.g, sc.z, sc.theta, h, v1, v2, r_ * sc.nq)[0]
                  for r_ in range(sc.nr)])
    above = np.cumsum(L[::-1])[::-1]          # sum of L over rows >= r (one cell per row)
    expect = -sc.i_a * sigma * np.arange(sc.nr, 0, -1)
    np.testing.assert_allclose(above, expect, rtol=1e-6)
    # (iii) kinematic profile away from the ends: discharge per unit width q = r X
    X = 1.5 * sc.a * (np.arange(sc.nr)[::-1] + 0.5)
    ok = []
    for r_ in range(8, sc.nr - 16):
        hk = _kinematic_depth(sc.i_a * X[r_], sc.meta["slope"], 0.8, synth.ALPHA_P, synth.ALPHA_S)
        ok.append(abs(H[r_, 0] / hk - 1.0))
    assert max(ok) < 0.05, max(ok)


def _sheet_on_plane(slope, h0=0.1, v_down=0.5, nq=7, nr=12, sides=(OUTFLOW, PERIODIC,
                                                                      OUTFLOW, PERIODIC)):
    """A uniform sheet flowing down a plane z = slope * y, periodic across the slope."""
    n = nq * nr
    _, y = synth.centres(nq, nr, 1.0)
    return synth.Scenario(name="sheet", nq=nq, nr=nr, a=1.0, z=slope * y,
                          theta=np.full(n, 0.8), alpha_p=np.full(n, synth.ALPHA_P), side=sides,
                          h0=np.full(n, h0), v10=np.zeros(n), v20=np.full(n, -v_down),
                          t_end=1e9)


def test_outflow_ghost_continues_the_plane():
    """The free-outflow ghost (the cell's own h, v and theta; the bed extrapolated linearly
    through the opposite neighbour) continues a uniform sheet on a plane: one step from
    such a sheet changes every cell alike, the rim rows (two OUTFLOW edges each, the
    downstream rim losing water through them and the upstream rim gaining it) exactly as
    the interior.  A flat ghost bed, a reflecting ghost or a dropped edge would each set
    the rim rows apart."""
    sc = _sheet_on_plane(0.02)
    G, p, r = _setup(sc)
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                 sc.t_end, max_steps=1)
    assert b.steps == 1
    for f, ref in ((h, sc.h0[0]), (v1, 0.0), (v2, v2.mean())):
        assert np.abs(f - f.mean()).max() <= 1e-13 * max(abs(ref), 1e-3), np.abs(f - f.mean()).max()
    # the step did something: friction against gravity, and the sheet's own outflow and
    # inflow balance (the depth is unchanged)
    assert abs(v2.mean() + 0.5) > 1e-6
    np.testing.assert_allclose(h, sc.h0, rtol=1e-14)
    # against a check that is not vacuous: with WALL sides instead, the rim rows differ
    walled = _sheet_on_plane(0.02, sides=(WALL, PERIODIC, WALL, PERIODIC))
    Gw, pw, rw = _setup(walled)
    hw, _, v2w, _, _ = oracle.run(Gw, walled.z, walled.theta, walled.alpha_p, pw, rw, walled.h0,
                                  walled.v10, walled.v20, walled.t_end, max_steps=1)
    assert np.abs(hw - hw.mean()).max() > 1e-6


# ------------------------------------------------------------- P12 rain

def test_triangular_hyetograph(golden):
    gv = golden("hyetograph.txt")
    ia, ta, Td = gv["i_a"], gv["t_a"], gv["T_d"]
    assert oracle.rain_rate(1, ia, ta, Td, ta) == pytest.approx(ia, rel=1e-15)
    assert oracle.rain_rate(1, ia, ta, Td, 0.0) == 0.0
    assert oracle.rain_rate(1, ia, ta, Td, Td) == 0.0
    assert oracle.rain_rate(1, ia, ta, Td, Td + 1) == 0.0
    assert oracle.rain_rate(1, ia, ta, Td, 0.5 * ta) == pytest.approx(0.5 * ia, rel=1e-15)
    t = np.linspace(0, Td, 200001)
    rr = np.array([oracle.rain_rate(1, ia, ta, Td, x) for x in t])
    V = np.trapezoid(rr, t) if hasattr(np, "trapezoid") else np.trapz(rr, t)
    assert V == pytest.approx(gv["V"], rel=1e-6)
    assert ia * Td / 2 == pytest.approx(gv["V"], rel=1e-12)


def test_triangular_rain_books_converge():
    """Right-endpoint rain books approach V * area; a Riemann sum over a function of
    total variation 2 i_a errs by at most 2 i_a dt_max, i.e. 4 dt_max / T_d relative."""
    errs = []
    for dtm in (2.0, 1.0, 0.5, 0.25):
        sc = synth.c1_planar(nq=6, nr=6, t_end=1000.0, rain_mmh=0.0).with_(
            rain_kind=1, i_a=7.32e-5, t_a=250.0, T_d=1000.0, dt_max=dtm, cfl=0.99,
            z=np.zeros(36))
        G, p, r = _setup(sc)
        _, _, _, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                   sc.t_end)
        sigma = oracle.geometry(1.0)[0]
        V = 7.32e-5 * 1000.0 / 2 * sigma * 36
        errs.append(abs(b.rain / V - 1.0))
        assert errs[-1] <= 4.0 * b.dt_max_seen / 1000.0
    assert errs[-1] < errs[0]


def test_susita_mass_table_balances(golden):
    """The paper's mass table obeys rain - out = left, the identity the books check."""
    g = golden("paper_grids.txt")
    assert g["susita_rain"] - g["susita_out"] == g["susita_left"]
    assert g["susita_rain"] - g["susita_out_veg"] == g["susita_left_veg"]


# ------------------------------------------------ soil coefficient per cell

def _uniform_flow(alpha_s, nq=12, nr=10, dt=0.05):
    N = nq * nr
    P = oracle.PERIODIC
    return synth.Scenario(name="soil", nq=nq, nr=nr, a=1.0, z=np.zeros(N), theta=np.ones(N),
                          alpha_p=np.zeros(N), alpha_s=alpha_s, side=(P, P, P, P),
                          h0=np.full(N, 0.5), v10=np.full(N, 0.3), v20=np.full(N, -0.2),
                          dt_max=dt, t_end=dt)


def test_soil_coefficient_per_cell():
    """eq_tsa_darcy with alpha_s varying over the raster: a uniform flow on a flat periodic
    raster has no edge sums, so one step is the friction solve of each cell alone,
    v' = 2 gamma / (alpha + sqrt(alpha^2 + 4 beta |gamma|)) with gamma = theta h v,
    alpha = theta h and beta = dt theta alpha_s of that cell (Appendix A, miu-formula)."""
    rng = np.random.default_rng(31)
    dt = 0.05
    field = rng.uniform(0.001, 0.05, 120)
    r = ref_run(_uniform_flow(field, dt=dt), max_steps=1)
    assert r["books"]["steps"] == 1
    m, g1, g2 = 0.5, 0.5 * 0.3, 0.5 * -0.2
    G = math.hypot(g1, g2)
    D = m + np.sqrt(m * m + 4.0 * dt * field * G)
    np.testing.assert_allclose(r["v1"], 2.0 * g1 / D, rtol=1e-13)
    np.testing.assert_allclose(r["v2"], 2.0 * g2 / D, rtol=1e-13)
    # a field holding one value everywhere is the scalar coefficient, bit for bit
    a = ref_run(_uniform_flow(np.full(120, 0.00709)), max_steps=3)
    b = ref_run(_uniform_flow(0.00709), max_steps=3)
    for k in ("h", "v1", "v2"):
        np.testing.assert_array_equal(a[k], b[k])
