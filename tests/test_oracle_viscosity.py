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
from tests._util import ref_params, ref_run

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
