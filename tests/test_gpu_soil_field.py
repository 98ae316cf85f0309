"""A Darcy-Weisbach soil coefficient per cell (eq_tsa_darcy with a soil that varies over the
raster) against the FP64 oracle (needs an MI355X).

The extended step instance reads the field as a seventh per-cell array; FP64 is bitwise
the oracle's, FP32 within the stated tolerances, and a field holding one value everywhere
gives the scalar run bit for bit in FP64.
"""
import numpy as np
import pytest
import torch

import synth
from tests._util import ref_run
from tests.test_gpu_parity import assert_books, assert_parity, gpu_run, hx  # noqa: F401

pytestmark = pytest.mark.gpu


def soil_planar(field=True, t_end=300.0):
    sc = synth.c1_planar(nq=70, nr=45, t_end=t_end)  # ragged tiles in both directions
    if field:
        rng = np.random.default_rng(41)
        # patches of rougher and smoother soil around the paper's 0.00709
        soil = 0.00709 * np.exp(rng.normal(0.0, 0.8, sc.n))
        sc = sc.with_(alpha_s=soil)
    return sc


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_soil_field_parity(hx, precision):
    sc = soil_planar()
    print(f"[soil field {precision} {sc.nq}x{sc.nr}]", flush=True)
    ref = ref_run(sc)
    got = gpu_run(hx, sc, precision)
    assert_parity(got, ref, precision, "soil-field")
    assert_books(got, ref, 1e-11 if precision == "fp64" else 1e-3)
    if precision == "fp64":
        assert got["books"]["steps"] == ref["books"]["steps"]
        for k in ("h", "v1", "v2"):
            np.testing.assert_array_equal(got[k], ref[k])
    # the field matters: the scalar coefficient gives another flow
    plain = ref_run(soil_planar(field=False))
    assert np.abs(plain["v1"] - ref["v1"]).max() > 1e-3


def test_uniform_field_is_the_scalar(hx):
    sc = soil_planar(field=False, t_end=120.0)
    a = gpu_run(hx, sc.with_(alpha_s=np.full(sc.n, sc.alpha_s)), "fp64")
    b = gpu_run(hx, sc, "fp64")
    for k in ("h", "v1", "v2"):
        np.testing.assert_array_equal(a[k], b[k])


def test_soil_field_is_validated(hx):
    sc = soil_planar(t_end=10.0)
    grid = hx.Grid.from_scenario(sc)
    sim = hx.Sim(grid, "fp32")
    bad = sc.alpha_s.copy()
    bad[17] = -1.0
    with pytest.raises(hx.HexsvError) as ei:
        sim.set_fields(sc.z, sc.theta, sc.alpha_p, bad)
    assert ei.value.code == hx.EDOMAIN and "first cell 17" in str(ei.value)
    sim.set_fields(sc.z, sc.theta, sc.alpha_p, sc.alpha_s)
    sim.set_state(sc.h0, sc.v10, sc.v20)
    sur = hx.Surrogate(4, 32)
    sur.set_params(np.zeros(sur.num_params, np.float32))
    with pytest.raises(hx.HexsvError) as ei:
        sim.run_surrogate(sur, 5.0, 1.0, 16)
    assert ei.value.code == hx.EUNSUPPORTED
    torch.cuda.synchronize()
