"""Surrogate windows inside the solver (features, prediction, water-balance gate, fallback)
against the oracle's window definitions (needs an MI355X).

* one accepted window equals the oracle chain features -> network (bf16 emulation) -> apply,
  and its books (t, rain, outflow, stored) follow the window definitions;
* with a zero tolerance every window falls back, and the result is bit for bit the plain
  solver advanced window by window.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import surrogate as so
from tests.test_gpu_parity import hx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

SCALES = (0.05, 0.01, 10.0, 0.01, 0.002, 0.1)  # H, Q, Z, dH, dQ, S
FS = (SCALES[0], SCALES[1], SCALES[2], SCALES[5], SCALES[3], SCALES[4])  # oracle order
WINDOW, K = 1.6, 16


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def wet_planar(nq=70, nr=40, seed=11):
    sc = synth.c1_planar(nq=nq, nr=nr, rain_mmh=100.0)
    h, v1, v2 = synth.random_state(sc, seed, depth=0.05, speed=0.2, dry_frac=0.1)
    return sc.with_(h0=h, v10=v1, v20=v2)


def make_surrogate(hx, seed=4):
    sur = hx.Surrogate(4, 32)
    p = so.init_params(seed, 4, 32, out_scale=0.1).astype(np.float32)
    sur.set_params(p)
    sur.set_scales(SCALES)
    return sur, p


def oracle_inputs(sc, t0=0.0):
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    p = oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s)
    r = oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
    th = np.where(G.active, sc.theta, 0.0)
    depth = so.window_rain_depth(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d, t0, WINDOW, K)
    ext = so.extrapolation(G, sc.z, th, sc.alpha_p, p, r, t0, WINDOW, sc.h0, sc.v10, sc.v20)
    f = so.features(G, sc.h0, sc.v10, sc.v20, sc.z, th, depth, ext, *FS)
    return G, th, depth, ext, f


@pytest.mark.parametrize("masked", [False, True])
def test_features_kernel(hx, masked):
    """Window inputs of an FP64 simulation (probe step included) against the oracle's."""
    if masked:
        sc = synth.cone(R=9, rim=synth.OUTFLOW)
        h, v1, v2 = synth.random_state(sc, 3, depth=0.05, speed=0.2)
        sc = sc.with_(h0=h, v10=v1, v20=v2)
    else:
        sc = wet_planar()
    sim = hx.Sim.from_scenario(sc, "fp64")
    sur, _ = make_surrogate(hx)
    f = sim.surrogate_features(sur, WINDOW, K).cpu().numpy()
    _, th, _, _, ref = oracle_inputs(sc)
    act = th > 0
    np.testing.assert_allclose(f[act], ref[act], rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(f[~act], 0.0)
    # the state is untouched
    st = sim.state_numpy()
    np.testing.assert_array_equal(st["h"][act], sc.h0[act])


def wet_cone(R=20):
    """Hexagonal domain cut by the mask, OUTFLOW rim: the taps stop at the mask."""
    sc = synth.cone(R=R, rim=synth.OUTFLOW)
    h, v1, v2 = synth.random_state(sc, 5, depth=0.05, speed=0.2)
    return sc.with_(h0=h, v10=v1, v20=v2)


def wet_strip(nq=70, nr=24):
    """Slope periodic in q: the taps wrap across the seam."""
    sc = synth.kinematic_strip(nq=nq, nr=nr, rain_mmh=100.0)
    h, v1, v2 = synth.random_state(sc, 6, depth=0.05, speed=0.2, dry_frac=0.1)
    return sc.with_(h0=h, v10=v1, v20=v2)


SCENES = {"planar": wet_planar, "cone": wet_cone, "strip": wet_strip}


@pytest.mark.parametrize("prec,scene", [("fp64", "planar"), ("fp32", "planar"),
                                        ("fp64", "cone"), ("fp32", "strip")])
def test_accepted_window_matches_oracle_chain(hx, prec, scene):
    sc = SCENES[scene]()
    sim = hx.Sim.from_scenario(sc, prec)
    b0 = sim.books()
    sur, p = make_surrogate(hx)
    print(f"[surrogate window {prec} {scene} {sc.nq}x{sc.nr}]", flush=True)
    acc, fb = sim.run_surrogate(sur, WINDOW, WINDOW, K, residual_tol=math.inf, project=False)
    assert (acc, fb) == (1, 0)
    assert sim.surrogate_stats()["kept"] == 1
    st = sim.state_numpy()
    b = sim.books()

    G, th, depth, ext, f = oracle_inputs(sc)
    out, _, _ = so.forward(G, p, f, 4, 32, bf16=True)
    hn, v1n, v2n = so.apply_window(sc.h0, sc.v10, sc.v20, th, out, SCALES[3], SCALES[4], ext)
    a = G.active  # cells outside the domain hold no water on the device
    e_h = rel_l2(st["h"][a] - sc.h0[a], (hn - sc.h0)[a])
    e_q1 = rel_l2((st["q1"] - th * sc.h0 * sc.v10)[a], (th * hn * v1n - th * sc.h0 * sc.v10)[a])
    e_q2 = rel_l2((st["q2"] - th * sc.h0 * sc.v20)[a], (th * hn * v2n - th * sc.h0 * sc.v20)[a])
    print(f"  change rel L2: h {e_h:.2e} q1 {e_q1:.2e} q2 {e_q2:.2e}")
    assert e_h <= 1e-3 and e_q1 <= 1e-3 and e_q2 <= 1e-3
    assert np.all(st["h"] >= 0.0)
    np.testing.assert_array_equal(st["h"][~a], 0.0)

    sigma, _, _ = oracle.geometry(sc.a)
    assert b["t"] == WINDOW
    assert b["rain"] - b0["rain"] == pytest.approx(sigma * int(G.active.sum()) * depth, rel=1e-12)
    # outflow volume by the trapezoid rule on the rates of the start and predicted states
    o0 = so.outflow_rate(G, sc.g, sc.z, th, sc.h0, sc.v10, sc.v20)
    o1 = so.outflow_rate(G, sc.g, sc.z, th, st["h"], st["v1"], st["v2"])
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert b["outflow"] - b0["outflow"] == pytest.approx(0.5 * (o0 + o1) * WINDOW, rel=tol)
    assert b["stored"] == pytest.approx(sigma * float(np.sum(th * st["h"])), rel=tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projection_closes_the_balance(hx, prec):
    """With projection the kept state is the unprojected one with every depth scaled by
    (S0 + R - O) / S', and its stored volume is S0 + R - O."""
    sc = wet_planar()
    sur, _ = make_surrogate(hx)
    runs = {}
    for proj in (False, True):
        sim = hx.Sim.from_scenario(sc, prec)
        b0 = sim.books()
        assert sim.run_surrogate(sur, WINDOW, WINDOW, K, math.inf, project=proj) == (1, 0)
        runs[proj] = (sim.state_numpy(), sim.books(), b0)
    (a, ba, b0), (p, bp, _) = runs[False], runs[True]
    target = b0["stored"] + (ba["rain"] - b0["rain"]) - (ba["outflow"] - b0["outflow"])
    f = target / ba["stored"]
    print(f"[projection {prec}] factor {f:.6f}")
    assert bp["stored"] == pytest.approx(target, rel=1e-12)
    tol = 1e-15 if prec == "fp64" else 3e-7
    np.testing.assert_allclose(p["h"], a["h"] * f, rtol=tol, atol=0)
    np.testing.assert_array_equal(p["v1"], a["v1"])
    sigma, _, _ = oracle.geometry(sc.a)
    assert sigma * float(np.sum(sc.theta * p["h"])) == pytest.approx(target, rel=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("backoff", [None, 0])
def test_zero_tolerance_falls_back_to_the_solver(hx, prec, backoff):
    sc = wet_planar(nq=66, nr=33, seed=12)
    t_end = 5 * WINDOW + 0.7
    sim = hx.Sim.from_scenario(sc, prec)
    if backoff is not None:
        sim.set_surrogate_backoff(backoff)
    sur, _ = make_surrogate(hx, seed=5)
    print(f"[surrogate fallback {prec} backoff {backoff}]", flush=True)
    acc, fb = sim.run_surrogate(sur, t_end, WINDOW, K, residual_tol=0.0)
    assert (acc, fb) == (0, 6)
    # by default windows are tried on spans 1, 2 and 5 and refused on their residual: after
    # the second refusal in a row the solver also advances spans 3 and 4 (back-off); without
    # the back-off a window is tried on every whole span.  Then the short last span.
    st = sim.surrogate_stats()
    refused = 3 if backoff is None else 5
    assert st == {"kept": 0, "refused_residual": refused, "refused_wave_speed": 0,
                  "refused_nonfinite": 0}, st
    ref = hx.Sim.from_scenario(sc, prec)
    t = 0.0
    for _ in range(5):  # the window ends as the surrogate loop forms them
        t = t + WINDOW
        ref.run(t)
    ref.run(t_end)
    a, r = sim.state_numpy(), ref.state_numpy()
    for k in ("h", "v1", "v2"):
        np.testing.assert_array_equal(a[k], r[k])
    ba, br = sim.books(), ref.books()
    for k in ("t", "initial", "stored", "rain", "outflow", "clamp", "steps"):
        assert ba[k] == br[k], k


def test_surrogate_window_rejects_bad_arguments(hx):
    sc = wet_planar(nq=20, nr=12)
    sim = hx.Sim.from_scenario(sc, "fp32")
    sur, _ = make_surrogate(hx)
    for window, k, tol in ((0.0, 16, 1e-3), (math.inf, 16, 1e-3), (1.0, 16, -1.0)):
        with pytest.raises(hx.HexsvError):
            sim.run_surrogate(sur, 10.0, window, k, tol)
    with pytest.raises(hx.HexsvError):
        sim.set_surrogate_backoff(-1)
    with pytest.raises(hx.HexsvError):
        hx.Surrogate(4, 32, k=0)
    torch.cuda.synchronize()


def test_window_length_defaults_to_the_surrogates_k(hx):
    """k <= 0 in the window calls takes the k the surrogate was created with."""
    sc = wet_planar(nq=40, nr=24)
    sur, _ = make_surrogate(hx)
    assert sur.k == 16
    out = []
    for k in (16, 0):
        sim = hx.Sim.from_scenario(sc, "fp64")
        assert sim.run_surrogate(sur, 2 * WINDOW, WINDOW, k, math.inf, project=False) == (2, 0)
        out.append(sim.state_numpy()["h"])
    np.testing.assert_array_equal(out[0], out[1])
