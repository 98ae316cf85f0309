"""The linear soil resistance on the GPU (the Thacker test's law, Sec. 3.2.2 / Appendix B):
parity with the FP64 oracle, and the non-oscillating Thacker problem at the paper's
resolution against its exact solution at the paper's four times (needs an MI355X)."""
import math
import time

import numpy as np
import pytest

import synth
from oracle.thacker import Thacker, surface_error
from tests._util import ref_run
from tests.test_gpu_parity import assert_books, assert_parity, gpu_run, hx  # noqa: F401
from tests.test_oracle_thacker import ERR_FACTOR, PAPER_ERR, VEL_REL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thacker_parity_with_the_oracle(hx, precision):
    sc = synth.thacker(a=1.65, t_end=10.0)
    ref = ref_run(sc, nthreads=8)
    got = gpu_run(hx, sc, precision)
    assert got["books"]["steps"] == ref["books"]["steps"] or precision == "fp32"
    assert_parity(got, ref, precision, "thacker")
    assert_books(got, ref, 1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thacker_against_the_exact_solution(hx, precision):
    sc = synth.thacker()
    ex = Thacker(sc.meta)
    x, y = synth.centres(sc.nq, sc.nr, sc.a)
    x, y = x + sc.meta["ox"], y + sc.meta["oy"]
    sim = hx.Sim.from_scenario(sc, precision)
    for t in sorted(PAPER_ERR):
        t0 = time.perf_counter()
        sim.run(t)
        st = sim.state_numpy()
        el = time.perf_counter() - t0
        err = surface_error(st["h"], sc.z, ex.depth(t, x, y))
        wet = st["h"] > 0.1
        u, v = ex.velocity(t)
        um, vm = st["v1"][wet].mean(), st["v2"][wet].mean()
        print(f"[thacker {precision} t={t:g}] err {err:.4f} (paper {PAPER_ERR[t]}), "
              f"u {um:.4f} ({u:.4f}), v {vm:.4f} ({v:.4f}), steps {sim.books()['steps']}, "
              f"{el:.2f} s", flush=True)
        assert err <= ERR_FACTOR[t] * PAPER_ERR[t]
        scale = max(math.hypot(u, v), 1e-3)  # late times: both components near zero
        assert abs(um - u) <= VEL_REL * scale + 1e-4
        assert abs(vm - v) <= VEL_REL * scale + 1e-4
    # closed walls, no rain: volume kept up to the clamp tally (the FP32 state rounds each
    # step's depths to about 1e-7, which over 4e4 steps drifts the volume by about 1e-5)
    b = sim.books()
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert b["stored"] == pytest.approx(b["initial"] + b["clamp"], rel=tol)


def test_zero_resistance_changes_nothing_and_bad_values_are_refused(hx):
    sc = synth.c1_planar(nq=40, nr=30, t_end=60.0)
    a = gpu_run(hx, sc, "fp32")
    sim = hx.Sim.from_scenario(sc, "fp32")
    sim.set_linear_friction(0.0)
    sim.run(sc.t_end)
    b = sim.state_numpy()
    np.testing.assert_array_equal(a["h"], b["h"])
    np.testing.assert_array_equal(a["v1"], b["v1"])
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(hx.HexsvError) as ei:
            sim.set_linear_friction(bad)
        assert ei.value.code == hx.EDOMAIN
