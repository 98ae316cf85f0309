"""Infiltration in the mass source on the GPU: parity with the FP64 oracle (a rained-on slope
and a still lake draining into the soil), the switch's edge cases, and its cost on the
1024 x 1024 catchment (needs an MI355X)."""
import numpy as np
import pytest

import synth
from tests._util import ref_run
from tests.test_gpu_parity import assert_books, assert_parity, gpu_run, hx  # noqa: F401

pytestmark = pytest.mark.gpu


def _slope():
    sc = synth.c1_planar(t_end=600.0)  # 50 mm/h on a 5 % slope, theta 0.8
    sc.f_inf, sc.h_inf = 1e-5, 0.005   # up to 36 mm/h into the soil, half of it at 5 mm
    return sc


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_infiltration_parity_with_the_oracle(hx, precision):
    sc = _slope()
    ref = ref_run(sc, nthreads=8)
    got = gpu_run(hx, sc, precision)
    if precision == "fp64":
        assert got["books"]["steps"] == ref["books"]["steps"]
    assert_parity(got, ref, precision, "infiltration")
    assert_books(got, ref, 1e-12 if precision == "fp64" else 1e-5)
    # the soil took water: less is stored than without infiltration
    plain = ref_run(synth.c1_planar(t_end=600.0), nthreads=8)
    assert ref["books"]["stored"] < 0.9 * plain["books"]["stored"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_still_lake_drains_into_the_soil(hx, precision):
    """FP64 matches the oracle bit for bit.  FP32 is held to the books only (5e-4 of the
    water): on a deep, nearly frictionless lake each step takes about 2e-6 m off depths near
    0.5 m, which FP32 rounds at 3e-8 m, and that grid-scale level noise stirs mm/s currents
    and moves the soil's share by a few 1e-3 (the FP32 state is built for overland flow,
    where the parity above holds to 1e-5)."""
    sc = synth.lake_at_rest()
    sc.theta[:] = 0.8
    sc.t_end, sc.f_inf, sc.h_inf = 600.0, 2e-5, 0.02
    ref = ref_run(sc, nthreads=8)
    got = gpu_run(hx, sc, precision)
    if precision == "fp64":
        assert_parity(got, ref, precision, "infiltration-lake")
    assert_books(got, ref, 1e-12 if precision == "fp64" else 5e-4)
    assert got["books"]["outflow"] > 0.0


def test_switch_edge_cases(hx):
    sc = synth.c1_planar(nq=40, nr=30, t_end=60.0)
    a = gpu_run(hx, sc, "fp32")
    sim = hx.Sim.from_scenario(sc, "fp32")
    sim.set_infiltration(1e-5, 0.01)
    sim.set_infiltration(0.0, 0.0)  # off again: the plain kernel, bit for bit
    sim.run(sc.t_end)
    b = sim.state_numpy()
    np.testing.assert_array_equal(a["h"], b["h"])
    np.testing.assert_array_equal(a["v1"], b["v1"])
    for f, c in ((-1e-5, 0.01), (float("nan"), 0.01), (1e-5, 0.0), (1e-5, -1.0),
                 (float("inf"), 0.01)):
        with pytest.raises(hx.HexsvError) as ei:
            sim.set_infiltration(f, c)
        assert ei.value.code == hx.EDOMAIN
    sim.set_infiltration(1e-5, 0.01)
    with pytest.raises(hx.HexsvError) as ei:
        sim.run_surrogate(hx.Surrogate(), sc.t_end + 10.0, 1.0, 4)
    assert ei.value.code == hx.EUNSUPPORTED
    with pytest.raises(hx.HexsvError) as ei:
        sim.surrogate_features(hx.Surrogate(), 1.0, 4)
    assert ei.value.code == hx.EUNSUPPORTED


def test_cost_on_the_catchment(hx):
    """The extended kernel instance on the 1024 x 1024 catchment, against the plain one."""
    sc = synth.c2_catchment()
    times = {}
    for name, f in (("plain", 0.0), ("infiltration", 1e-5)):
        sim = hx.Sim.from_scenario(sc, "fp32")
        if f:
            sim.set_infiltration(f, 0.005)
        sim.run(1e30, max_steps=200)
        times[name] = min(sim.time_kernel(100) for _ in range(3)) * 1e3
    print(f"[infiltration cost] k_step 1024^2 FP32: plain {times['plain']:.2f} us, with "
          f"infiltration {times['infiltration']:.2f} us", flush=True)
    assert times["infiltration"] < 1.5 * times["plain"]
