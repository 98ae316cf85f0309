"""Given-mass-flux cells on the GPU, the flume of Sec. 3.3.2 and the ensemble-driven
sensitivity sweep of Sec. 3.4: tables and parity with the FP64 oracle (single runs and
batched ensembles, with and without the viscous flux), then delta_s and delta_p of the
steady vegetated flume over a grid of friction coefficients (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.flume import hbar, normal_depth, sensitivities
from tests._util import ref_run
from tests.test_gpu_parity import TOL, assert_books, assert_parity, gpu_run, hx  # noqa: F401

pytestmark = pytest.mark.gpu

Q, M, TV = 0.021, 0.00105, 0.99364


def _flume(q=Q, m=M, alpha_s=synth.ALPHA_S, alpha_p=synth.ALPHA_P, a=0.1, t_end=20.0, h_in=None,
           visc=True):
    hv = h_in or normal_depth(q, TV, m, synth.ALPHA_S, synth.ALPHA_P)
    sc = synth.flume(q=q, h_in=hv, theta_v=TV, m=m, alpha_s=alpha_s, alpha_p=alpha_p, a=a,
                     t_end=t_end)
    sc.visc = visc
    return sc


def test_tables_with_flux_cells_bit_exact(hx):
    sc = _flume()
    nbr_ref, code_ref = oracle.tables(sc.nq, sc.nr, sc.side, sc.segs, sc.active, sc.mask_code)
    grid = hx.Grid.from_scenario(sc)
    nbr, code, _, _ = grid.tables()
    np.testing.assert_array_equal(nbr.cpu().numpy(), nbr_ref)
    np.testing.assert_array_equal(code.cpu().numpy(), code_ref)
    assert (code_ref == oracle.FLUX).sum() > 0


def assert_flume_parity(got, ref, precision, label):
    """As assert_parity, but with the two velocity (and discharge) components pooled: across
    the flume v2 is rounding noise, so a relative norm of it alone measures nothing."""
    if precision == "fp64":
        return assert_parity(got, ref, precision, label)
    def pooled(a, b):
        num = np.abs(got[a] - ref[a]).sum() + np.abs(got[b] - ref[b]).sum()
        return num / (np.abs(ref[a]).sum() + np.abs(ref[b]).sum())
    eh = np.abs(got["h"] - ref["h"]).sum() / np.abs(ref["h"]).sum()
    ev, eq = pooled("v1", "v2"), pooled("q1", "q2")
    print(f"[parity {label} {precision}] rel L1 h={eh:.3e} v={ev:.3e} q={eq:.3e}", flush=True)
    assert eh <= TOL[precision]["h"] and eq <= TOL[precision]["q"] and ev <= TOL[precision]["q"]


@pytest.mark.parametrize("visc", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_flume_parity_with_the_oracle(hx, precision, visc):
    # without the viscous flux the flume sloshes and rounding differences grow: 5 s there
    sc = _flume(visc=visc, t_end=20.0 if visc else 5.0)
    ref = ref_run(sc, nthreads=8)
    got = gpu_run(hx, sc, precision)
    if precision == "fp64":
        assert got["books"]["steps"] == ref["books"]["steps"]
    assert_flume_parity(got, ref, precision, f"flume{'-visc' if visc else ''}")
    assert_books(got, ref, 1e-12 if precision == "fp64" else 1e-5)
    f = sc.active == 3
    np.testing.assert_array_equal(got["h"][f], sc.h0[f].astype(np.float32 if precision == "fp32"
                                                                 else np.float64))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_flume_ensemble_with_viscosity_matches_the_oracle(hx, precision):
    scs = [_flume(alpha_s=synth.ALPHA_S * k, alpha_p=synth.ALPHA_P * (2 - k)) for k in (0.8, 1.2)]
    ens = hx.Ensemble.from_scenarios(scs, precision, mode="batched")
    assert ens.info()["mode"] == "batched"
    ens.run(scs[0].t_end)
    for s, sc in enumerate(scs):
        ref = ref_run(sc, nthreads=8)
        got = ens.state_numpy(s)
        got["books"] = ens.books(s)
        if precision == "fp64":
            assert got["books"]["steps"] == ref["books"]["steps"]
        assert_flume_parity(got, ref, precision, f"flume-ensemble-{s}")
        assert_books(got, ref, 1e-12 if precision == "fp64" else 1e-5)


def test_viscosity_and_boundary_cells_move_an_ensemble_to_batched_steps(hx):
    sc = synth.c1_planar(nq=40, nr=30, t_end=10.0)
    ens = hx.Ensemble.from_scenarios([sc, sc], "fp32", mode="persistent")
    assert ens.info()["mode"] == "persistent"
    ens.set_viscosity(True)
    assert ens.info()["mode"] == "batched"
    fl = _flume(visc=False)
    assert hx.Ensemble.from_scenarios([fl, fl], "fp32", mode="persistent").info()["mode"] == \
        "batched"
    with pytest.raises(hx.HexsvError) as ei:
        hx._check(hx.lib().hexsv_ensemble_set_viscosity(ens._h, 2))
    assert ei.value.code == hx.EINVAL


def test_sensitivity_sweep_of_the_vegetated_flume(hx):
    """delta_s, delta_p (Sec. 3.4) of the steady mean depth over the vegetated zone on a 3 x 3
    grid of (alpha_s, alpha_p) around the paper's fitted values, for three discharges at the
    flume's slope and two more slopes: one batched FP64 ensemble of 45 flumes (a = 5 cm,
    300 s).  The grid's
    hbar are finite and grow with both coefficients, hbar at the centre is the normal depth
    of the vegetated reach, delta_p grows with the discharge (the paper's first
    observation; delta_s stays near 0.55 m here), and the deltas agree with the oracle's
    formula on the same grid."""
    from paper_2406_14933_amd import sensitivity

    a_s = synth.ALPHA_S * np.array([0.9, 1.0, 1.1])
    a_p = synth.ALPHA_P * np.array([0.9, 1.0, 1.1])
    envs = [(q, M) for q in (0.007, 0.015, 0.021)] + [(0.015, m) for m in (0.0005, 0.002)]
    facts, zones = [], []
    for q, m in envs:
        hv = normal_depth(q, TV, m, synth.ALPHA_S, synth.ALPHA_P)
        facts.append(lambda s, p, q=q, m=m, hv=hv: _flume(q, m, s, p, a=0.05, t_end=300.0,
                                                          h_in=hv))
        zones.append(facts[-1](a_s[1], a_p[1]).meta["veg_zone"])
    res, sec = sensitivity.sweep(facts, a_s, a_p, zones, 300.0, "fp64")
    for (q, m), r in zip(envs, res):
        hv = normal_depth(q, TV, m, synth.ALPHA_S, synth.ALPHA_P)
        ref = sensitivities(r["H"], a_s[1] - a_s[0], a_p[1] - a_p[0])
        print(f"[sensitivity q={q * 1e3:g} l/s m={m * 1e3:g} mm/m] hbar(centre) "
              f"{r['H'][1, 1]:.5f} (normal depth {hv:.5f}), delta_s {r['delta_s']:.4f} m, "
              f"delta_p {r['delta_p']:.3e} m^2", flush=True)
        assert np.all(np.isfinite(r["H"]))
        assert r["delta_s"] == pytest.approx(ref[0], rel=1e-12)
        assert r["delta_p"] == pytest.approx(ref[1], rel=1e-12)
        assert r["delta_s"] > 0 and r["delta_p"] > 0
        assert np.all(np.diff(r["H"], axis=0) > 0) and np.all(np.diff(r["H"], axis=1) > 0)
        assert r["H"][1, 1] == pytest.approx(hv, rel=0.02)
    print(f"[sensitivity] {len(envs) * 9} flumes x 300 s in one ensemble: {sec:.2f} s", flush=True)
    d_p = [r["delta_p"] for r in res[:3]]
    assert d_p[0] < d_p[1] < d_p[2]


def test_autotune_keeps_a_viscous_flux_ensemble_batched(hx):
    """The autotuner times batched variants only when the ensemble carries the viscous flux
    or boundary cells (the persistent kernel is built for neither), and restores the state:
    the tuned run still matches the oracle bit for bit."""
    scs = [_flume(alpha_s=synth.ALPHA_S * k) for k in (0.9, 1.1)]
    ens = hx.Ensemble.from_scenarios(scs, "fp64")
    ens.autotune(ksteps=4)
    assert ens.info()["mode"] == "batched"
    ens.run(scs[0].t_end)
    for s, sc in enumerate(scs):
        ref = ref_run(sc, nthreads=8)
        got = ens.state_numpy(s)
        got["books"] = ens.books(s)
        assert got["books"]["steps"] == ref["books"]["steps"]
        assert_parity(got, ref, "fp64", f"flume-tuned-{s}")
