"""Pins of the artificial-viscosity flux (eqs. eq_artif_visc, eq_visc1) and of the Riemann
problem with vegetation (Sec. 3.2.3) on the oracle.  No GPU needed.

The exact solution of the Riemann problem comes from a cited paper that is not here, so
its wave structure is parity unpinned; what is pinned is what the mathematics fixes: the
viscous flux is a sum of antisymmetric edge exchanges that vanishes for a uniform velocity
and across dry cells (so it conserves momentum and only dissipates), and the left state of
this problem is supercritical (Froude 3.6), so no wave can travel upstream of the jump:
the exact solution keeps it unchanged for x < 9 m, which the scheme does only with the
viscous flux.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests._util import ref_grid, ref_params, ref_run, rel_l1

P = oracle.PERIODIC


def _flat(nq=14, nr=12, seed=3, dry=False, uniform_v=False):
    rng = np.random.default_rng(seed)
    n = nq * nr
    h = rng.uniform(0.05, 0.5, n)
    if dry:
        h[rng.random(n) < 0.3] = 0.0
    v1 = np.full(n, 0.7) if uniform_v else rng.normal(0.0, 0.5, n)
    v2 = np.full(n, -0.2) if uniform_v else rng.normal(0.0, 0.5, n)
    sc = synth.Scenario(name="flat", nq=nq, nr=nr, a=1.0, z=np.zeros(n),
                        theta=rng.uniform(0.5, 1.0, n), alpha_p=np.zeros(n), alpha_s=0.0,
                        side=(P, P, P, P), h0=h, v10=v1, v20=v2, visc=True)
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    return sc, G


def test_viscous_sums_two_cell_worked_case(golden):
    """eq_visc1 by value: c_ij is the larger wave speed and mu_ij the harmonic mean of
    theta h (a minimum, a mean or another mean of either would miss these figures)."""
    gv = golden("two_cell_viscosity.txt")
    G = oracle.grid(2, 1, 1.0)
    th = np.array([gv["theta_i"], gv["theta_j"]])
    h = np.array([gv["h_i"], gv["h_j"]])
    v1 = np.array([gv["v1_i"], gv["v1_j"]])
    v2 = np.array([gv["v2_i"], gv["v2_j"]])
    Vi = oracle.visc_sums(G, gv["g"], th, h, v1, v2, 0)
    Vj = oracle.visc_sums(G, gv["g"], th, h, v1, v2, 1)
    np.testing.assert_allclose(Vi, [gv["V1_i"], gv["V2_i"]], rtol=1e-14)
    np.testing.assert_allclose(Vj, [gv["V1_j"], gv["V2_j"]], rtol=1e-14)
    h_dry = np.array([gv["h_i"], 0.0])
    Vd = oracle.visc_sums(G, gv["g"], th, h_dry, v1, v2, 0)
    np.testing.assert_array_equal(Vd, [gv["dry_V1_i"], gv["dry_V2_i"]])


def test_viscous_sums_vanish_for_a_uniform_velocity():
    sc, G = _flat(uniform_v=True)
    for i in range(G.n):
        np.testing.assert_array_equal(
            oracle.visc_sums(G, sc.g, sc.theta, sc.h0, sc.v10, sc.v20, i), [0.0, 0.0])


def test_viscous_sums_are_edge_antisymmetric_and_skip_dry_cells():
    sc, G = _flat(dry=True)
    V = np.array([oracle.visc_sums(G, sc.g, sc.theta, sc.h0, sc.v10, sc.v20, i)
                  for i in range(G.n)])
    # every edge exchange appears twice with opposite signs: the total is zero
    scale = np.abs(V).sum()
    assert scale > 0.0
    assert abs(V[:, 0].sum()) <= 1e-13 * scale and abs(V[:, 1].sum()) <= 1e-13 * scale
    # a dry cell exchanges nothing (mu_ij = 0 when either side is dry)
    dry = sc.h0 == 0.0
    assert dry.any()
    np.testing.assert_array_equal(V[dry], 0.0)


def test_viscous_flux_conserves_momentum_and_dissipates():
    """A shear layer on a flat periodic raster without friction: momentum is the same with
    and without the viscous flux, the kinetic energy is lower with it."""
    nq, nr = 16, 16
    n = nq * nr
    r = np.repeat(np.arange(nr), nq)
    v1 = np.where(r < nr // 2, 0.4, -0.4)
    base = synth.Scenario(name="shear", nq=nq, nr=nr, a=1.0, z=np.zeros(n), theta=np.ones(n),
                          alpha_p=np.zeros(n), alpha_s=0.0, side=(P, P, P, P),
                          h0=np.full(n, 0.3), v10=v1, v20=np.zeros(n), t_end=20.0)
    out = {}
    for visc in (False, True):
        sc = synth.Scenario(**{**base.__dict__, "visc": visc})
        res = ref_run(sc, max_steps=60)
        m = res["h"]
        out[visc] = ((m * res["v1"]).sum(), (m * res["v2"]).sum(),
                     (m * (res["v1"] ** 2 + res["v2"] ** 2)).sum())
    assert out[True][0] == pytest.approx(out[False][0], abs=1e-9 * n)
    assert out[True][1] == pytest.approx(out[False][1], abs=1e-9 * n)
    assert out[True][2] < 0.99 * out[False][2]


def _left_state(r, sc, x):
    act = sc.active.astype(bool)
    sel = act & (x > 1.0) & (x < sc.meta["x_jump"] - 0.5)
    th, z, h, u = sc.meta["left"]
    return (np.abs(r["h"][sel] - h).max() / h, np.abs(r["v1"][sel] - u).max() / u,
            np.abs(r["v2"][sel]).max() / u)


def test_riemann_supercritical_inflow_is_kept_only_with_the_viscous_flux():
    sc = synth.riemann(n_section=281)
    x, _ = synth.centres(sc.nq, sc.nr, sc.a)
    x = x + sc.meta["ox"]
    r = ref_run(sc, nthreads=8)
    dh, du, dv = _left_state(r, sc, x)
    print(f"[riemann oracle] left state: |dh|/h {dh:.2e}, |du|/u {du:.2e}, |v2|/u {dv:.2e}, "
          f"steps {r['books']['steps']}", flush=True)
    assert dh <= 1e-2 and du <= 1e-2 and dv <= 1e-2
    assert r["books"]["residual"] <= 1e-12
    # the channel's flow stays one-dimensional: across the width the free surface is flat
    # (median over 2-cell bins along the channel; the shock fronts cross a few bins)
    H = r["h"] + sc.z
    act = sc.active.astype(bool)
    bins = np.floor(x / (2.0 * sc.a * math.sqrt(3.0))).astype(int)
    spread = [H[act & (bins == b)].std() for b in np.unique(bins[act])]
    assert np.median(spread) <= 1e-3
    # without it the scheme rings upstream of the jump
    r0 = ref_run(synth.Scenario(**{**sc.__dict__, "visc": False}), nthreads=8)
    assert max(_left_state(r0, sc, x)) > 0.05


# ------------------------------------------------------------ the sheared layer

def _shear(t_end=30.0):
    """A sheared layer over a rough vegetated bed (plant drag, random z and theta), periodic,
    with the viscous flux: the flow decays towards rest over 30 s."""
    nq, nr = 40, 34
    n = nq * nr
    r = np.repeat(np.arange(nr), nq)
    rng = np.random.default_rng(11)
    return synth.Scenario(name="shear", nq=nq, nr=nr, a=1.0, z=rng.uniform(0, 0.05, n),
                          theta=rng.uniform(0.6, 1.0, n), alpha_p=np.full(n, synth.ALPHA_P),
                          side=(P, P, P, P), h0=rng.uniform(0.05, 0.4, n),
                          v10=np.where(r < nr // 2, 0.5, -0.5), v20=rng.normal(0, 0.1, n),
                          t_end=t_end, visc=True)


_NX = [1.0, 0.5, -0.5, -1.0, -0.5, 0.5]
_S3H = 0.86602540378443864676
_NY = [0.0, _S3H, _S3H, 0.0, -_S3H, -_S3H]


def _steps(sc, on_step=None):
    """The oracle's trajectory step by step; on_step(k, t, h, v1, v2) sees each start state
    and may return a velocity increment (cell, component, value) applied before the step."""
    G = ref_grid(sc)
    p, r = ref_params(sc), oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
    h, v1, v2 = sc.h0.copy(), sc.v10.copy(), sc.v20.copy()
    b = oracle.books_init(G, sc.theta, h)
    k = 0
    while b.t < sc.t_end:
        if on_step is not None:
            kick = on_step(k, b.t, h, v1, v2)
            if kick is not None:
                cell, comp, dv = kick
                (v1 if comp == 0 else v2)[cell] += dv
        h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, h, v1, v2, sc.t_end,
                                     max_steps=1, books=b, nthreads=1)
        k += 1
    th = sc.theta
    return {"h": h, "v1": v1, "v2": v2, "q1": th * h * v1, "q2": th * h * v2}


def shear_branch_events(sc):
    """Steps at which an interior edge's normal velocity v_n (eq. fvm_2D_eq.04) is nonzero but
    below FP32 resolution, |v_n| < 2^-23 max(|v_i|, |v_j|): there the upwind choice of the
    interface mass (eqs. fvm_2D_eq.05-.06) is decided by less than one FP32 rounding of the
    velocities.  Returns [(step, t, cell, edge, v_n)], each edge once."""
    G = ref_grid(sc)
    ev = []

    def scan(k, t, h, v1, v2):
        sp = np.hypot(v1, v2)
        for e in range(3):  # each edge once: directions 0..2 of every cell
            j = G.nbr[:, e]
            vn = (v1 + v1[j]) * 0.5 * _NX[e] + (v2 + v2[j]) * 0.5 * _NY[e]
            small = (vn != 0.0) & (np.abs(vn) < 2.0 ** -23 * np.maximum(sp, sp[j]))
            for i in np.nonzero(small)[0]:
                ev.append((k, t, int(i), e, float(vn[i])))

    _steps(sc, scan)
    return ev


def branch_flipped_run(sc, event):
    """The oracle's trajectory with the one edge of `event` taking the other upwind branch: a
    velocity increment of three times |v_n| at its step (well inside FP32 rounding of the
    velocities) reverses the sign of v_n and changes nothing else of note."""
    k0, _, i, e, vn = event
    comp = 1 if _NY[e] != 0.0 else 0
    n_c = _NY[e] if comp else _NX[e]
    dv = -3.0 * vn / (0.5 * n_c)  # v_n + 0.5 n_c dv = -2 v_n

    def kick(k, t, h, v1, v2):
        return (i, comp, dv) if k == k0 else None

    return _steps(sc, kick)


def test_shear_layer_has_one_upwind_decision_below_fp32_resolution():
    """On the decaying sheared layer the scheme's upwind choice of the interface mass (eqs.
    fvm_2D_eq.05-.06) is discontinuous in v_n at 0.  Over 30 s exactly one edge meets a v_n
    below FP32 resolution (-9.65e-10 m/s at t = 15.75 s, 8e-8 of the flow speed there), and
    taking the other branch there, by a velocity change of 6.7e-9 m/s, moves q at 30 s by
    1e-2 relative L1 in FP64: the gap an FP32 state (rounded at 6e-8) cannot avoid.  The same
    change that keeps the branch moves it by less than 1e-8."""
    sc = _shear()
    ev = shear_branch_events(sc)
    assert len(ev) == 1, ev
    k, t, i, e, vn = ev[0]
    assert 15.5 < t < 16.0 and abs(vn) < 1e-9
    base = _steps(sc)
    flip = branch_flipped_run(sc, ev[0])
    dq = max(rel_l1(flip["q1"], base["q1"]), rel_l1(flip["q2"], base["q2"]))
    assert dq > 3e-3, dq
    # the same increment with the opposite sign keeps the branch (v_n becomes 4 v_n)
    keep = branch_flipped_run(sc, (k, t, i, e, -vn))
    dq_keep = max(rel_l1(keep["q1"], base["q1"]), rel_l1(keep["q2"], base["q2"]))
    assert dq_keep < 1e-8, dq_keep
