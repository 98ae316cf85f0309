"""Batched ensemble (one persistent kernel over uneven rasters) against the oracle and
against the single-catchment GPU path (needs an MI355X)."""
import numpy as np
import pytest
import torch

import synth
from tests._util import ref_run, rel_l1
from tests.test_gpu_parity import TOL, assert_parity, hx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def mixed_scenarios():
    return [
        synth.ensemble_member(0, nmin=40, nmax=40, t_end=90.0),
        synth.ensemble_member(1, nmin=70, nmax=70, t_end=120.0),
        synth.catchment(90, 77, 2.0, config=2, t_end=60.0),
        synth.cone(R=14, rim=synth.OUTFLOW, t_end=45.0),
        synth.kinematic_strip(nq=6, nr=48, t_end=150.0),
        synth.ensemble_member(2, nmin=130, nmax=130, t_end=70.0).with_(nr=130),
        synth.c1_planar(nq=64, nr=64, t_end=100.0),
    ]


@pytest.mark.parametrize("mode,tile", [("persistent", 0), ("persistent", 1), ("persistent", 2),
                                       ("batched", 2), ("batched", 0), ("batched", 5)])
def test_ensemble_fp64_matches_oracle_and_single(hx, mode, tile):
    scs = mixed_scenarios()
    ens = hx.Ensemble.from_scenarios(scs, "fp64", steps_per_launch=23, tile=tile, mode=mode)
    assert ens.info()["mode"] == mode
    ens.run([sc.t_end for sc in scs])
    for s, sc in enumerate(scs):
        got = ens.state_numpy(s)
        got["books"] = ens.books(s)
        ref = ref_run(sc)
        assert got["books"]["t"] == sc.t_end
        assert got["books"]["steps"] == ref["books"]["steps"], s
        assert_parity(got, ref, "fp64", f"ens{s}")
        single = hx.Sim.from_scenario(sc, "fp64", tile=2)
        single.run(sc.t_end)
        st = single.state_numpy()
        # the same per-cell arithmetic and the same time steps: bit-identical states
        np.testing.assert_array_equal(got["h"], st["h"])
        np.testing.assert_array_equal(got["v1"], st["v1"])
        np.testing.assert_array_equal(got["v2"], st["v2"])
        if mode == "batched" and tile == 2:
            # same tiles and the same reduction tree as the single-catchment path
            assert got["books"]["stored"] == single.books()["stored"]
        assert got["books"]["stored"] == pytest.approx(single.books()["stored"], rel=1e-13)
        assert got["books"]["residual"] <= 1e-12


@pytest.mark.parametrize("mode", ["persistent", "batched"])
def test_ensemble_fp32_members(hx, mode):
    scs = [synth.ensemble_member(s, nmin=60, nmax=140, t_end=600.0) for s in range(6)]
    ens = hx.Ensemble.from_scenarios(scs, "fp32", mode=mode)
    ens.run([sc.t_end for sc in scs])
    for s, sc in enumerate(scs):
        got = ens.state_numpy(s)
        ref = ref_run(sc)
        assert_parity(got, ref, "fp32", f"ens32-{s}")
        # FP32 state: each step rounds every cell's depth, so the FP64 books drift by
        # about sqrt(steps) * 2^-24 relative to the stored volume
        assert ens.books(s)["residual"] <= 1e-4


@pytest.mark.parametrize("mode", ["persistent", "batched"])
def test_ensemble_step_limit_and_resume(hx, mode):
    scs = mixed_scenarios()[:3]
    ens = hx.Ensemble.from_scenarios(scs, "fp64", steps_per_launch=10, mode=mode)
    ens.run([sc.t_end for sc in scs], max_steps=17)
    for s in range(3):
        assert ens.books(s)["steps"] == 17
    ens.run([sc.t_end for sc in scs])
    for s, sc in enumerate(scs):
        ref = ref_run(sc)
        got = ens.state_numpy(s)
        assert ens.books(s)["t"] == sc.t_end
        assert_parity(got, ref, "fp64", f"resume{s}")


@pytest.mark.parametrize("tile", [2, 0])
def test_ensemble_resumes_from_mixed_parities(hx, tile):
    """Runs to each scenario's own stop leave the scenarios at different step counts, so
    their buffer parities differ when the next run starts (the batched launches' per-tile
    load hints carry them); every scenario still ends bit-identical to a single-catchment
    run with the same stops."""
    scs = mixed_scenarios()
    stops = [0.37 * sc.t_end + 3.1 * s for s, sc in enumerate(scs)]
    ens = hx.Ensemble.from_scenarios(scs, "fp64", steps_per_launch=7, tile=tile, mode="batched")
    ens.run(stops)
    parities = {ens.books(s)["steps"] % 2 for s in range(len(scs))}
    assert parities == {0, 1}, parities
    ens.run([sc.t_end for sc in scs])
    for s, sc in enumerate(scs):
        single = hx.Sim.from_scenario(sc, "fp64", tile=tile)
        single.run(stops[s])
        single.run(sc.t_end)
        got, st = ens.state_numpy(s), single.state_numpy()
        assert ens.books(s)["steps"] == single.books()["steps"], s
        for k in ("h", "v1", "v2"):
            np.testing.assert_array_equal(got[k], st[k])


def test_ensemble_timing_counts_cell_updates(hx):
    scs = mixed_scenarios()[:4]
    ens = hx.Ensemble.from_scenarios(scs, "fp32")
    ens.timing(True)
    ens.run([1e9] * 4, max_steps=40)
    tm = ens.timing()
    assert tm["cell_updates"] == sum(40 * int(np.count_nonzero(
        sc.active if sc.active is not None else np.ones(sc.n))) for sc in scs)
    assert tm["gpu_ms"] > 0 and tm["launches"] >= 1


def test_ensemble_autotune_restores_state(hx, tmp_path):
    scs = mixed_scenarios()
    ref = hx.Ensemble.from_scenarios(scs, "fp64", tile=0)
    ref.run([sc.t_end for sc in scs])
    ens = hx.Ensemble.from_scenarios(scs, "fp64")
    cache = str(tmp_path / "tune.json")
    best, ms = ens.autotune(ksteps=4, cache_path=cache)
    assert best // 100 in (1, 2) and ms > 0
    info = ens.info()
    assert info["tile"] == best % 100
    assert info["mode"] == {1: "persistent", 2: "batched"}[best // 100]
    ens.run([sc.t_end for sc in scs])
    for s in range(len(scs)):
        np.testing.assert_array_equal(ens.state_numpy(s)["h"], ref.state_numpy(s)["h"])
        assert ens.books(s)["steps"] == ref.books(s)["steps"]
    assert "gfx950/ensemble/fp64" in open(cache).read()


def test_sim_autotune_and_cache(hx, tmp_path, monkeypatch):
    sc = synth.catchment(200, 150, 2.0, config=2, t_end=30.0)
    sim = hx.Sim.from_scenario(sc, "fp64")
    sim.run(10.0)
    before = sim.state_numpy()
    cache = str(tmp_path / "tune.json")
    best, ms = sim.autotune(nlaunch=5, cache_path=cache)
    assert 0 <= best < len(hx.tile_shapes()) and ms > 0
    after = sim.state_numpy()
    np.testing.assert_array_equal(before["h"], after["h"])
    assert sim.info()["tile"] == best
    sim.run(sc.t_end)
    monkeypatch.setenv("HEXSV_TUNE_CACHE", cache)
    sim2 = hx.Sim.from_scenario(sc, "fp64")
    assert sim2.info()["tile"] == best
    sim2.run(10.0)
    sim2.run(sc.t_end)
    np.testing.assert_array_equal(sim2.state_numpy()["h"], sim.state_numpy()["h"])


def test_standalone_autotune_writes_the_cache(hx, tmp_path, monkeypatch):
    """hexsv_autotune tunes on the library's own workload and leaves a cache entry that a
    simulation (or ensemble) of that size bucket then starts from."""
    import json
    cache = str(tmp_path / "tune.json")
    print("[standalone autotune step fp32 2^16]", flush=True)
    best, ms = hx.autotune(cache, "step", "fp32", 1 << 16)
    assert 0 <= best < len(hx.tile_shapes()) and ms > 0
    entry = json.load(open(cache))["gfx950/step/fp32/2^16"]
    assert entry["tile"] == best and len(entry["all_us"]) == len(hx.tile_shapes())
    monkeypatch.setenv("HEXSV_TUNE_CACHE", cache)
    sc = synth.c1_planar(nq=256, nr=256, t_end=5.0)
    sim = hx.Sim.from_scenario(sc, "fp32")
    assert sim.info()["tile"] == best
    sim.run(sc.t_end)
    print("[standalone autotune ensemble fp32 8 x 64^2]", flush=True)
    eb, ems = hx.autotune(cache, "ensemble", "fp32", 8 * 64 * 64)
    assert ems > 0
    keys = json.load(open(cache))
    assert "gfx950/step/fp32/2^16" in keys and "gfx950/ensemble/fp32/2^15" in keys
    with pytest.raises(hx.HexsvError):
        hx.autotune(cache, "step", "fp32", 10)
    torch.cuda.synchronize()


def test_full_ensemble_one_step_sampled(hx):
    """The whole 256-scenario ensemble (128^2 .. 512^2, about 29.9 M cells) in the batched
    FP32 mode the benchmark times: after 40 steps, each scenario's next step matches the
    oracle's step of the same state on sampled cells (its four sides and random interior
    cells), and its time step is the oracle's from that state."""
    import oracle
    from tests._util import ref_grid, ref_params, ref_rain
    from tests.test_gpu_parity import assert_parity
    scs = synth.c3_ensemble(n_scen=256)
    ens = hx.Ensemble.from_scenarios(scs, "fp32", mode="batched", steps_per_launch=20)
    print(f"[full ensemble] {ens.info()['cells']} cells", flush=True)
    ens.run([sc.t_end for sc in scs], max_steps=40)
    s0 = [ens.state_numpy(s) for s in range(len(scs))]
    b0 = [ens.books(s) for s in range(len(scs))]
    ens.run([sc.t_end for sc in scs], max_steps=1)
    rng = np.random.Generator(np.random.PCG64(17))
    worst = {"h": 0.0, "q": 0.0, "dt": 0.0}
    for s, sc in enumerate(scs):
        st1, b1 = ens.state_numpy(s), ens.books(s)
        G = ref_grid(sc)
        st0 = s0[s]
        th0 = np.where(G.active, sc.theta, 0.0)
        cmax = oracle.cmax(G, sc.g, th0, st0["h"], st0["v1"], st0["v2"])
        dt_ref = oracle.dt(sc.a, ref_params(sc), cmax, b0[s]["t"], sc.t_end)
        dt = b1["t"] - b0[s]["t"]
        worst["dt"] = max(worst["dt"], abs(dt / dt_ref - 1.0))
        assert dt == pytest.approx(dt_ref, rel=1e-6), (s, dt, dt_ref)
        n, nq = sc.n, sc.nq
        cells = np.unique(np.concatenate([
            rng.integers(0, n, 300), np.arange(0, nq), np.arange(n - nq, n),
            np.arange(0, n, nq), np.arange(nq - 1, n, nq)]).astype(np.int32))
        hn, v1n, v2n, _ = oracle.step_cells(G, sc.z, sc.theta, sc.alpha_p, ref_params(sc),
                                            ref_rain(sc), dt, b1["t"], st0["h"], st0["v1"],
                                            st0["v2"], cells)
        th = sc.theta[cells]
        ref = {"h": hn, "v1": v1n, "v2": v2n, "q1": th * hn * v1n, "q2": th * hn * v2n}
        got = {k: st1[k][cells] for k in ("h", "v1", "v2")}
        got["q1"] = th * got["h"] * got["v1"]
        got["q2"] = th * got["h"] * got["v2"]
        e = assert_parity(got, ref, "fp32", f"ens{s}") if s % 64 == 0 else None
        if e is None:
            from tests._util import rel_l1
            e = {"h": rel_l1(got["h"], ref["h"]),
                 "q": max(rel_l1(got["q1"], ref["q1"]), rel_l1(got["q2"], ref["q2"]))}
            assert e["h"] <= 1e-4 and e["q"] <= 1e-3, (s, e)
        worst["h"] = max(worst["h"], e["h"])
        worst["q"] = max(worst["q"], e["q"])
    print(f"[full ensemble] worst over 256 scenarios: h {worst['h']:.2e} q {worst['q']:.2e} "
          f"dt {worst['dt']:.2e}", flush=True)
