"""BF16 MFMA hex-convolution surrogate kernels against the FP64 oracle (needs an MI355X).

The oracle rounds features, weights and hidden activations to bfloat16 exactly where the
GPU does and accumulates in FP64; remaining differences come from FP32 accumulation order
(and the rare bfloat16 rounding it flips), so values agree to about 1e-2 relative L2.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import surrogate as so
from tests.test_gpu_parity import hx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def setup(seed, nq, nr, batch, layers=4):
    rng = np.random.default_rng(seed)
    p = so.init_params(seed, layers, 32, out_scale=1.0)
    p = (p + rng.normal(scale=0.02, size=p.shape)).astype(np.float32)
    feats = rng.normal(size=(batch, nq * nr, so.FEATURES)).astype(np.float32)
    tgt = rng.normal(size=(batch, nq * nr, 3)).astype(np.float32)
    G = oracle.grid(nq, nr, 1.0)
    return p, feats, tgt, G


@pytest.mark.parametrize("nq,nr,batch,layers", [(70, 9, 2, 4), (64, 4, 1, 4), (33, 17, 3, 3),
                                                (130, 6, 1, 5)])
def test_forward_matches_oracle(hx, nq, nr, batch, layers):
    p, feats, _, G = setup(1, nq, nr, batch, layers)
    sur = hx.Surrogate(layers, 32)
    sur.set_params(p)
    out = sur.forward(feats.reshape(-1, so.FEATURES), nq, nr).cpu().numpy().reshape(batch, nq * nr, 4)
    for b in range(batch):
        ref, _, _ = so.forward(G, p, feats[b].astype(np.float64), layers, 32, bf16=True)
        e = rel_l2(out[b, :, :3], ref)
        print(f"[surrogate fwd {nq}x{nr} b{b}] rel L2 {e:.2e}")
        assert e <= 1e-2


@pytest.mark.parametrize("nq,nr,batch", [(70, 9, 2), (40, 12, 1)])
def test_gradient_matches_oracle(hx, nq, nr, batch):
    layers = 4
    p, feats, tgt, G = setup(2, nq, nr, batch, layers)
    sur = hx.Surrogate(layers, 32)
    sur.set_params(p)
    loss, g = sur.gradient(feats.reshape(-1, so.FEATURES), tgt.reshape(-1, 3), nq, nr)
    g = g.cpu().numpy()
    rl, rg = so.loss_and_grad(G, p, [f.astype(np.float64) for f in feats],
                              [t.astype(np.float64) for t in tgt], layers, 32, bf16=True)
    assert loss == pytest.approx(rl, rel=2e-3)
    k = 0
    for li, (ci, co) in enumerate(so.layer_shapes(layers, 32)):
        nw = co * ci * 7
        ew = rel_l2(g[k:k + nw], rg[k:k + nw])
        eb = rel_l2(g[k + nw:k + nw + co], rg[k + nw:k + nw + co])
        print(f"[surrogate grad layer {li}] W rel L2 {ew:.2e}  b rel L2 {eb:.2e}")
        assert ew <= 2e-2 and eb <= 2e-2
        k += nw + co


def test_adam_step_matches_oracle(hx):
    nq, nr = 40, 12
    p, feats, tgt, G = setup(3, nq, nr, 1)
    sur = hx.Surrogate(4, 32)
    sur.set_params(p)
    _, g = sur.gradient(feats.reshape(-1, so.FEATURES), tgt.reshape(-1, 3), nq, nr)
    f = torch.from_numpy(feats.reshape(-1, so.FEATURES)).cuda()
    t = torch.from_numpy(tgt.reshape(-1, 3)).cuda()
    sur.train_step(f, t, nq, nr, 1e-3)
    p1 = sur.params().cpu().numpy()
    ref, _, _ = so.adam_update(p.astype(np.float64), 0.0, 0.0, g.cpu().numpy().astype(np.float64),
                               1, 1e-3)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(hx):
    nq, nr, batch = 64, 32, 4
    rng = np.random.default_rng(4)
    p = so.init_params(5, 4, 32)
    sur = hx.Surrogate(4, 32)
    sur.set_params(p)
    feats = rng.normal(size=(batch * nq * nr, so.FEATURES)).astype(np.float32)
    # a smooth target the network can represent: local linear combinations of features
    tgt = np.stack([0.5 * feats[:, 0] - 0.3 * feats[:, 5], 0.2 * feats[:, 1],
                    -0.4 * feats[:, 2] + 0.1 * feats[:, 3]], axis=1).astype(np.float32)
    f = torch.from_numpy(feats).cuda()
    t = torch.from_numpy(tgt).cuda()
    losses = [sur.train_step(f, t, nq, nr, 3e-3) for _ in range(300)]
    print(f"[surrogate train] loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.3 * losses[0]


# Rasters whose neighbour rule is not the walled parallelogram's: a hexagonal domain cut by
# the mask with an OUTFLOW rim (a cone's domain), a strip periodic in q with a ragged last
# tile, and a raster periodic on both sides.  The oracle convolves through the tables of the
# scheme (ref_tables), so these check that the kernels' taps follow the same rule: wrapped
# across periodic seams, zero across the mask unless both cells are in the domain, and the
# cell's own tap read even outside the domain.
RASTERS = {
    "cone-outflow-rim": dict(nq=73, nr=73, side=(synth.WALL,) * 4, mask_R=35,
                             mask_bc=synth.OUTFLOW),
    "strip-periodic-q": dict(nq=70, nr=9, side=(synth.OUTFLOW, synth.PERIODIC, synth.WALL,
                                                 synth.PERIODIC)),
    "torus": dict(nq=40, nr=12, side=(synth.PERIODIC,) * 4),
}


def raster(hx, kind):
    d = RASTERS[kind]
    nq, nr = d["nq"], d["nr"]
    act = synth.hexagon_mask(nq, nr, d["mask_R"]) if "mask_R" in d else None
    mbc = d.get("mask_bc", synth.WALL)
    G = oracle.grid(nq, nr, 1.0, d["side"], (), act, mbc)
    grid = hx.Grid(nq, nr, 1.0, d["side"], (), act, mbc)
    return nq, nr, G, grid


@pytest.mark.parametrize("kind", list(RASTERS))
def test_forward_follows_the_raster_tables(hx, kind):
    nq, nr, G, grid = raster(hx, kind)
    batch, layers = 2, 4
    rng = np.random.default_rng(21)
    p = (so.init_params(21, layers, 32, out_scale=1.0)
         + rng.normal(scale=0.02, size=so.num_params(layers, 32))).astype(np.float32)
    # inputs everywhere, cells outside the domain included (their own tap reads them)
    feats = rng.normal(size=(batch, nq * nr, so.FEATURES)).astype(np.float32)
    sur = hx.Surrogate(layers, 32)
    sur.set_params(p)
    print(f"[surrogate fwd {kind} {nq}x{nr}]", flush=True)
    out = sur.forward(feats.reshape(-1, so.FEATURES), nq, nr, grid=grid).cpu().numpy()
    out = out.reshape(batch, nq * nr, 4)
    plain = sur.forward(feats.reshape(-1, so.FEATURES), nq, nr).cpu().numpy()
    plain = plain.reshape(batch, nq * nr, 4)
    for b in range(batch):
        ref, _, _ = so.forward(G, p, feats[b].astype(np.float64), layers, 32, bf16=True)
        e = rel_l2(out[b, :, :3], ref)
        # the walled-parallelogram rule differs from these tables
        e_plain = rel_l2(plain[b, :, :3], ref)
        print(f"  b{b}: rel L2 {e:.2e} (walled-parallelogram rule: {e_plain:.2e})")
        assert e <= 1e-2
        assert e_plain > 10 * e


@pytest.mark.parametrize("kind", list(RASTERS))
def test_gradient_follows_the_raster_tables(hx, kind):
    nq, nr, G, grid = raster(hx, kind)
    layers, batch = 4, 2
    rng = np.random.default_rng(22)
    p = (so.init_params(22, layers, 32, out_scale=1.0)
         + rng.normal(scale=0.02, size=so.num_params(layers, 32))).astype(np.float32)
    feats = rng.normal(size=(batch, nq * nr, so.FEATURES)).astype(np.float32)
    tgt = rng.normal(size=(batch, nq * nr, 3)).astype(np.float32)
    sur = hx.Surrogate(layers, 32)
    sur.set_params(p)
    print(f"[surrogate grad {kind} {nq}x{nr}]", flush=True)
    loss, g = sur.gradient(feats.reshape(-1, so.FEATURES), tgt.reshape(-1, 3), nq, nr, grid=grid)
    g = g.cpu().numpy()
    rl, rg = so.loss_and_grad(G, p, [f.astype(np.float64) for f in feats],
                              [t.astype(np.float64) for t in tgt], layers, 32, bf16=True)
    assert loss == pytest.approx(rl, rel=2e-3)
    k = 0
    for li, (ci, co) in enumerate(so.layer_shapes(layers, 32)):
        nw = co * ci * 7
        ew = rel_l2(g[k:k + nw], rg[k:k + nw])
        eb = rel_l2(g[k + nw:k + nw + co], rg[k + nw:k + nw + co])
        print(f"  layer {li}: W rel L2 {ew:.2e}  b rel L2 {eb:.2e}")
        assert ew <= 2e-2 and eb <= 2e-2
        k += nw + co


FUSED_CASES = {
    # ragged 16 x 16 tiles in both directions, a batch of samples
    "walled-ragged": dict(nq=70, nr=37, batch=3),
    # rasters smaller than the fused kernel's 4-cell halo: wraps of more than one period
    "tiny-torus": dict(nq=5, nr=3, batch=2, side=(synth.PERIODIC,) * 4),
    "one-cell": dict(nq=1, nr=1, batch=2),
}


@pytest.mark.parametrize("kind", list(FUSED_CASES) + list(RASTERS))
def test_fused_forward_equals_the_layer_chain(hx, kind):
    """The 4-layer network in one kernel (activations kept on chip, 4-cell halo) gives the
    layer-by-layer launches' outputs bit for bit, on walled, masked and periodic rasters."""
    if kind in FUSED_CASES:
        d = FUSED_CASES[kind]
        nq, nr, batch = d["nq"], d["nr"], d["batch"]
        grid = hx.Grid(nq, nr, 1.0, d["side"], (), None, synth.WALL) if "side" in d else None
    else:
        nq, nr, _, grid = raster(hx, kind)
        batch = 2
    rng = np.random.default_rng(23)
    p = (so.init_params(23, 4, 32, out_scale=1.0)
         + rng.normal(scale=0.02, size=so.num_params(4, 32))).astype(np.float32)
    feats = torch.from_numpy(rng.normal(size=(batch * nq * nr, so.FEATURES))
                             .astype(np.float32)).cuda()
    sur = hx.Surrogate(4, 32)
    sur.set_params(p)
    print(f"[fused forward {kind} {nq}x{nr} batch {batch}]", flush=True)
    sur.set_fused(True)
    fused = sur.forward(feats, nq, nr, grid=grid)
    sur.set_fused(False)
    chain = sur.forward(feats, nq, nr, grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(fused[:, :3], chain[:, :3])
    assert torch.isfinite(fused[:, :3]).all()


def test_conv_refuses_a_mismatched_or_dirichlet_grid(hx):
    sur = hx.Surrogate(4, 32)
    sur.set_params(so.init_params(1, 4, 32))
    f = torch.zeros((20 * 12, so.FEATURES), dtype=torch.float32, device="cuda")
    with pytest.raises(hx.HexsvError) as e:
        sur.forward(f, 20, 12, grid=hx.Grid(12, 20, 1.0))
    assert e.value.code == hx.EINVAL
    act = np.ones(20 * 12, np.uint8)
    act[:20] = 2  # a row of Dirichlet cells
    with pytest.raises(hx.HexsvError) as e:
        sur.forward(f, 20, 12, grid=hx.Grid(20, 12, 1.0, active=act))
    assert e.value.code == hx.EUNSUPPORTED
    torch.cuda.synchronize()
