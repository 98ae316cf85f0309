"""The plant coefficient alpha_p (eq_tpa) as a field that varies over the raster (the paper
gives it one value; the step reads it per cell) against the oracle, in a single domain and
in a batched ensemble beside scenarios with the one value (needs an MI355X)."""
import numpy as np
import pytest

import synth
from tests._util import ref_run
from tests.test_gpu_parity import assert_books, assert_parity, gpu_run, hx  # noqa: F401

pytestmark = pytest.mark.gpu


def plant_planar(field=True, t_end=300.0):
    sc = synth.c1_planar(nq=70, nr=45, t_end=t_end)  # ragged tiles in both directions
    if field:
        rng = np.random.default_rng(43)
        sc = sc.with_(alpha_p=synth.ALPHA_P * np.exp(rng.normal(0.0, 0.7, sc.n)))
    return sc


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plant_field_parity(hx, precision):
    sc = plant_planar()
    print(f"[plant field {precision} {sc.nq}x{sc.nr}]", flush=True)
    ref = ref_run(sc)
    got = gpu_run(hx, sc, precision)
    assert_parity(got, ref, precision, "plant-field")
    assert_books(got, ref, 1e-11 if precision == "fp64" else 1e-3)
    if precision == "fp64":
        assert got["books"]["steps"] == ref["books"]["steps"]
        for k in ("h", "v1", "v2"):
            np.testing.assert_array_equal(got[k], ref[k])
    # the field matters: the uniform coefficient gives another flow
    plain = ref_run(plant_planar(field=False))
    assert np.abs(plain["v1"] - ref["v1"]).max() > 1e-4


def test_ensemble_mixes_uniform_and_field_scenarios(hx):
    """A batched ensemble of scenarios with and without a varying plant field: each is the
    oracle's run bit for bit (FP64)."""
    scs = [plant_planar(field=True, t_end=120.0), plant_planar(field=False, t_end=120.0),
           synth.ensemble_member(3, nmin=90, nmax=90, t_end=120.0)]
    ens = hx.Ensemble.from_scenarios(scs, "fp64", mode="batched")
    ens.run([sc.t_end for sc in scs])
    for s, sc in enumerate(scs):
        got = ens.state_numpy(s)
        ref = ref_run(sc)
        for k in ("h", "v1", "v2"):
            np.testing.assert_array_equal(got[k], ref[k])
