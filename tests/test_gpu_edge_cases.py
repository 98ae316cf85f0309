"""Degenerate and extreme inputs on the GPU: rasters of one cell, one row or one column,
ragged tails against the tile shape, a raster with no active cell, and the size limit
(needs an MI355X)."""
import numpy as np
import pytest

import synth
from tests._util import ref_run
from tests.test_gpu_parity import assert_books, assert_parity, gpu_run, hx  # noqa: F401

pytestmark = pytest.mark.gpu


def _small(nq, nr, side=(synth.OUTFLOW, synth.WALL, synth.WALL, synth.WALL)):
    n = nq * nr
    x, y = synth.centres(nq, nr, 1.0)
    return synth.Scenario(
        name=f"small-{nq}x{nr}", nq=nq, nr=nr, a=1.0, z=0.05 * y + 0.01 * x,
        theta=np.full(n, 0.8), alpha_p=np.full(n, synth.ALPHA_P), side=side, rain_kind=0,
        i_a=200.0 / 3.6e6, t_end=120.0, h0=np.full(n, 0.01))


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (2, 3), (65, 17), (129, 33)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_and_ragged_rasters(hx, shape, precision):
    """Rasters smaller than one tile, one row or one column wide, and sizes that leave a
    ragged last tile in both directions (64 x 16 tiles)."""
    sc = _small(*shape)
    ref = ref_run(sc, nthreads=4)
    got = gpu_run(hx, sc, precision)
    if precision == "fp64":
        assert got["books"]["steps"] == ref["books"]["steps"]
    assert_parity(got, ref, precision, f"{shape[0]}x{shape[1]}")
    assert_books(got, ref, 1e-12 if precision == "fp64" else 1e-5)


def test_periodic_single_row(hx):
    sc = _small(9, 1, side=(synth.WALL, synth.PERIODIC, synth.WALL, synth.PERIODIC))
    ref = ref_run(sc, nthreads=4)
    got = gpu_run(hx, sc, "fp64")
    assert_parity(got, ref, "fp64", "periodic-row")


def test_raster_without_active_cells(hx):
    """Every cell masked: the run reaches t_end with nothing stored, rained or lost."""
    sc = _small(20, 12)
    sc.active = np.zeros(sc.n, np.uint8)
    sim = hx.Sim.from_scenario(sc, "fp32")
    assert sim.grid.active_cells == 0
    sim.run(sc.t_end)
    b = sim.books()
    assert b["t"] == sc.t_end
    assert b["stored"] == 0.0 and b["rain"] == 0.0 and b["outflow"] == 0.0


def test_fields_beyond_the_32_bit_offsets_are_refused(hx):
    """Each field is addressed by a 32-bit byte offset: a raster whose FP32 field would
    reach 4 GiB is refused before anything is allocated."""
    grid = hx.Grid(40000, 27000, 1.0)  # 1.08e9 cells, 4.32 GB per FP32 field
    with pytest.raises(hx.HexsvError) as ei:
        hx.Sim(grid, "fp32")
    assert ei.value.code == hx.EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sheet_on_a_plane_with_outflow_rims(hx, precision):
    """The uniform sheet of the outflow-ghost pin (OUTFLOW rims up- and downstream, periodic
    across the slope) on a raster of ragged 64 x 16 tiles: FP64 bit for bit the oracle's
    over 30 steps, and after one step every cell alike, rims included."""
    from tests.test_oracle_pins import _sheet_on_plane
    sc = _sheet_on_plane(0.02, nq=70, nr=45)
    ref = ref_run(sc, max_steps=30)
    got = gpu_run(hx, sc, precision, max_steps=30)
    assert got["books"]["steps"] == 30
    if precision == "fp64":
        for k in ("h", "v1", "v2"):
            np.testing.assert_array_equal(got[k], ref[k])
    assert_parity(got, ref, precision, "sheet")
    one = gpu_run(hx, sc, precision, max_steps=1)
    tol = 1e-13 if precision == "fp64" else 2e-6
    for k in ("h", "v2"):
        assert np.abs(one[k] - one[k].mean()).max() <= tol * np.abs(one[k]).max(), k
