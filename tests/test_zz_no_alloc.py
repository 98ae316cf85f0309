"""The allocation-free surrogate forward (hexsv_surrogate_forward_noalloc) against the
allocating one through the C-ABI (needs an MI355X).

Both run the same kernels in the same order, so the outputs agree bit for bit; the
static workspace keeps the last call's contents, so a second, smaller call checks that
nothing stale leaks into it.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import surrogate as so
from tests.test_gpu_parity import hx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _net(hx, seed):
    rng = np.random.default_rng(seed)
    p = (so.init_params(seed, 4, 32, out_scale=1.0)
         + rng.normal(scale=0.02, size=so.num_params(4, 32))).astype(np.float32)
    sur = hx.Surrogate(4, 32)
    sur.set_params(p)
    return sur, rng


def test_noalloc_forward_equals_forward_on_two_calls(hx):
    sur, rng = _net(hx, 51)
    calls = [(2, 300, 401, None),  # 240 600 cells: near the workspace's limit
             (1, 70, 45, "cone")]  # then a smaller, masked raster
    for batch, nq, nr, kind in calls:
        grid = None
        if kind == "cone":
            act = synth.hexagon_mask(nq, nr, 20)
            grid = hx.Grid(nq, nr, 1.0, (synth.WALL,) * 4, (), act, synth.OUTFLOW)
        print(f"[noalloc] batch {batch} {nq}x{nr} {kind}", flush=True)
        f = torch.from_numpy(rng.normal(size=(batch * nq * nr, so.FEATURES))
                             .astype(np.float32)).cuda()
        ref = sur.forward(f, nq, nr, grid=grid)
        out = torch.full((batch * nq * nr, 4), float("nan"), dtype=torch.float32, device="cuda")
        sur.forward_noalloc(f, nq, nr, out, grid=grid)
        torch.cuda.synchronize()
        assert torch.equal(out[:, :3], ref[:, :3])


def test_noalloc_forward_refuses_beyond_its_workspace(hx):
    sur, _ = _net(hx, 52)
    f = torch.zeros((513 * 512, so.FEATURES), dtype=torch.float32, device="cuda")
    out = torch.empty((513 * 512, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(hx.HexsvError) as e:
        sur.forward_noalloc(f, 513, 512, out)
    assert e.value.code == hx.EINVAL and "static workspace" in str(e.value)
    torch.cuda.synchronize()
