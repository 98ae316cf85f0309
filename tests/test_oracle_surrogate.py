"""Pins of the surrogate oracle (hex convolution, network gradients, bf16, Adam)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import surrogate as so

SQ3 = math.sqrt(3.0)


def _brute_conv(nq, nr, x, W, b):
    """Hex convolution from hex-centre geometry: neighbour in direction k is the centre at
    distance sqrt(3)*a and angle 60k degrees; missing neighbours contribute nothing."""
    xs, ys = synth.centres(nq, nr, 1.0)
    n = nq * nr
    cout = W.shape[0]
    y = np.zeros((cout, n))
    for i in range(n):
        taps = [i] + [-1] * 6
        for j in range(n):
            dx, dy = xs[j] - xs[i], ys[j] - ys[i]
            if abs(math.hypot(dx, dy) - SQ3) < 1e-9:
                k = int(round(math.degrees(math.atan2(dy, dx)) % 360 / 60.0)) % 6
                taps[1 + k] = j
        for o in range(cout):
            acc = b[o]
            for t, j in enumerate(taps):
                if j >= 0:
                    acc += float(W[o, :, t] @ x[:, j])
            y[o, i] = acc
    return y


def test_hexconv_matches_geometry():
    rng = np.random.default_rng(0)
    nq, nr, cin, cout = 5, 4, 3, 2
    G = oracle.grid(nq, nr, 1.0)
    x = rng.normal(size=(cin, nq * nr))
    W = rng.normal(size=(cout, cin, 7))
    b = rng.normal(size=cout)
    np.testing.assert_allclose(oracle.hexconv_fwd(G, x, W, b), _brute_conv(nq, nr, x, W, b),
                               rtol=1e-13, atol=1e-13)


def test_hexconv_single_tap_is_a_matmul():
    rng = np.random.default_rng(1)
    G = oracle.grid(6, 5, 1.0)
    x = rng.normal(size=(4, 30))
    W = np.zeros((3, 4, 7))
    W[:, :, 0] = rng.normal(size=(3, 4))
    b = rng.normal(size=3)
    np.testing.assert_allclose(oracle.hexconv_fwd(G, x, W, b), W[:, :, 0] @ x + b[:, None],
                               rtol=1e-13, atol=1e-13)


def test_hexconv_backward_is_the_adjoint():
    rng = np.random.default_rng(2)
    G = oracle.grid(7, 6, 1.0)
    n = 42
    x = rng.normal(size=(5, n))
    W = rng.normal(size=(4, 5, 7))
    dy = rng.normal(size=(4, n))
    zero = np.zeros(4)
    y = oracle.hexconv_fwd(G, x, W, zero)
    dx, dW, db = oracle.hexconv_bwd(G, x, W, dy)
    # <dy, A x> == <A^T dy, x>
    assert (dy * y).sum() == pytest.approx((dx * x).sum(), rel=1e-12)
    # y is linear in W: the directional derivative is exact
    D = rng.normal(size=W.shape)
    y2 = oracle.hexconv_fwd(G, x, W + 0.5 * D, zero)
    assert ((dy * (y2 - y)).sum()) == pytest.approx(0.5 * (dW * D).sum(), rel=1e-11)
    np.testing.assert_allclose(db, dy.sum(axis=1), rtol=1e-13)


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    G = oracle.grid(6, 5, 1.0)
    layers, ch = 3, 4
    p = so.init_params(7, layers, ch, out_scale=1.0).astype(np.float64)
    p += rng.normal(scale=0.05, size=p.shape)
    xs = [rng.normal(size=(30, so.FEATURES)) for _ in range(2)]
    ts = [rng.normal(size=(30, so.OUTPUTS)) for _ in range(2)]

    def smooth_loss(q):
        # squared error keeps the check smooth: same backward path with dy = 2 diff / count
        tot = 0.0
        for x0, t in zip(xs, ts):
            out, _, _ = so.forward(G, q, x0, layers, ch, bf16=False)
            tot += ((out - t) ** 2).sum()
        return tot / (2 * 30 * so.OUTPUTS)

    def smooth_grad(q):
        g = np.zeros_like(q)
        count = 2 * 30 * so.OUTPUTS
        for x0, t in zip(xs, ts):
            out, acts, params = so.forward(G, q, x0, layers, ch, bf16=False)
            dy = 2 * (out - t) / count
            gl = []
            for li in range(len(params) - 1, -1, -1):
                dx, dW, db = so._conv_bwd(G, acts[li], params[li][0], dy)
                gl.append((dW, db))
                if li > 0:
                    dy = dx * (acts[li] > 0)
            g += so.flatten(gl[::-1])
        return g

    g = smooth_grad(p)
    idx = rng.choice(len(p), 40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (smooth_loss(p + e) - smooth_loss(p - e)) / 2e-6
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_l1_loss_gradient_sign_structure():
    """The L1 gradient is the squared-error path with dy = sign(diff)/count."""
    rng = np.random.default_rng(4)
    G = oracle.grid(5, 4, 1.0)
    p = so.init_params(1, 2, 3, out_scale=1.0).astype(np.float64)
    x = rng.normal(size=(20, so.FEATURES))
    t = rng.normal(size=(20, so.OUTPUTS))
    loss, g = so.loss_and_grad(G, p, [x], [t], 2, 3, bf16=False)
    out, _, _ = so.forward(G, p, x, 2, 3, bf16=False)
    assert loss == pytest.approx(np.abs(out - t).mean(), rel=1e-14)
    # directional derivative of a piecewise-linear loss away from kinks
    d = rng.normal(size=p.shape)
    eps = 1e-7
    l2, _ = so.loss_and_grad(G, p + eps * d, [x], [t], 2, 3, bf16=False)
    assert (l2 - loss) / eps == pytest.approx(g @ d, rel=1e-4)


def test_bf16_rounding_matches_torch():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.7182818, 3.1e-5, 65504.0, 1e-40,
                     0.0, -0.0, 1.7e38], np.float32)
    ours = so.bf16_round(vals)
    ref = torch.tensor(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)
    assert ours[1] == 1.0 and ours[2] == 1 + 2 ** -6  # ties to even
    rng = np.random.default_rng(5)
    r = rng.normal(size=10000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 10000)
    np.testing.assert_array_equal(so.bf16_round(r),
                                  torch.tensor(r).to(torch.bfloat16).to(torch.float64).numpy())


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        t.grad = torch.tensor(g.copy())
        opt.step()
        p, m, v = so.adam_update(p, m, v, g, step, 1e-2)
    np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_param_layout():
    shapes = so.layer_shapes(4, 32)
    assert shapes == [(11, 32), (32, 32), (32, 32), (32, 3)]
    n = so.num_params(4, 32)
    assert n == 11 * 32 * 7 + 32 + 2 * (32 * 32 * 7 + 32) + 32 * 3 * 7 + 3
    p = so.init_params(0)
    assert p.shape == (n,) and p.dtype == np.float32
    back = so.flatten(so.unflatten(p))
    np.testing.assert_array_equal(back, p.astype(np.float64))


# ------------------------------------------------------ surrogate windows

def test_outflow_rate_closed_form():
    """Uniform sheet flowing straight south over an OUTFLOW south side: every cell of row r=0
    has two outflow edges (directions 4 and 5) with v.n = V sqrt(3)/2, so the rate is
    2 nq a theta h V sqrt(3)/2; the other sides are walls."""
    nq, nr, a, th, h, V = 12, 10, 1.5, 0.8, 0.02, 0.3
    G = oracle.grid(nq, nr, a, side=(oracle.OUTFLOW, oracle.WALL, oracle.WALL, oracle.WALL))
    n = nq * nr
    z = np.zeros(n)
    rate = so.outflow_rate(G, 9.81, z, np.full(n, th), np.full(n, h), np.zeros(n),
                           np.full(n, -V))
    assert rate == pytest.approx(2 * nq * a * th * h * V * SQ3 / 2, rel=1e-14)
    # flow along the outlet carries nothing out; a dry raster neither
    assert so.outflow_rate(G, 9.81, z, np.full(n, th), np.full(n, h), np.full(n, V),
                           np.zeros(n)) == pytest.approx(0.0, abs=1e-15)
    assert so.outflow_rate(G, 9.81, z, np.full(n, th), np.zeros(n), np.zeros(n),
                           np.full(n, -V)) == 0.0


def test_outflow_rate_matches_the_books_of_one_step():
    """The outflow booked by one tiny solver step is dt times the rate of the state."""
    sc = synth.c1_planar(nq=16, nr=12)
    h, v1, v2 = synth.random_state(sc, 5)
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side)
    rate = so.outflow_rate(G, sc.g, sc.z, sc.theta, h, v1, v2)
    dt = 2.0 ** -20
    p = oracle.params(sc.g, sc.cfl, dt, sc.h_dry, sc.alpha_s)
    _, _, _, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, oracle.rain(), h, v1, v2, dt)
    assert b.steps == 1 and rate > 0
    assert b.outflow == pytest.approx(dt * rate, rel=1e-12)


def test_apply_window_zero_change_keeps_the_state():
    rng = np.random.default_rng(3)
    n = 200
    th = rng.uniform(0.3, 1.0, n)
    th[:10] = 0.0  # inactive
    h = rng.uniform(0.0, 0.1, n)
    h[10:40] = 0.0  # dry
    v1, v2 = rng.normal(size=n), rng.normal(size=n)
    v1[10:40] = v2[10:40] = 0.0
    hn, v1n, v2n = so.apply_window(h, v1, v2, th, np.zeros((n, 3)), 0.1, 0.01)
    np.testing.assert_array_equal(hn, h)
    wet = th * h > 1e-6
    np.testing.assert_allclose(v1n[wet], v1[wet], rtol=1e-14)
    np.testing.assert_allclose(v2n[wet], v2[wet], rtol=1e-14)
    assert np.all(v1n[(th > 0) & ~wet] == 0.0)
    # a negative predicted depth is clamped to dry, with zero velocity
    out = np.zeros((n, 3))
    out[:, 0] = -10.0
    hn, v1n, _ = so.apply_window(h, v1, v2, th, out, 0.1, 0.01)
    assert np.all(hn[th > 0] == 0.0) and np.all(v1n[th > 0] == 0.0)
    np.testing.assert_array_equal(hn[:10], h[:10])


def test_apply_window_worked_case(golden):
    """One cell by hand: the new velocity is the predicted discharge over the predicted
    mass theta h' (not over the start mass), and a depth driven below zero dries the cell."""
    gv = golden("apply_window.txt")
    one = lambda k: np.array([gv[k]])
    out = np.array([[gv["out0"], gv["out1"], gv["out2"]]])
    ext = (one("x_h"), one("x_q1"), one("x_q2"))
    hn, v1n, v2n = so.apply_window(one("h"), one("v1"), one("v2"), one("theta"), out,
                                   gv["dH"], gv["dQ"], ext)
    assert hn[0] == pytest.approx(gv["h_new"], rel=1e-15)
    assert v1n[0] == pytest.approx(gv["v1_new"], rel=1e-14)
    assert v2n[0] == pytest.approx(gv["v2_new"], rel=1e-14)
    out[0, 0] = gv["dry_out0"]
    hn, v1n, v2n = so.apply_window(one("h"), one("v1"), one("v2"), one("theta"), out,
                                   gv["dH"], gv["dQ"], ext)
    assert hn[0] == 0.0 and v1n[0] == 0.0 and v2n[0] == 0.0


def test_features_definition():
    G = oracle.grid(3, 1, 1.0)
    h = np.array([0.1, 0.0, 0.2])
    v1 = np.array([1.0, 0.0, -2.0])
    v2 = np.array([0.5, 0.0, 0.0])
    z = np.array([3.0, 4.0, 5.0])
    th = np.array([0.5, 1.0, 0.0])
    ext = (np.array([1e-3, 2e-3, 9.0]), np.array([4e-4, 0.0, 9.0]), np.array([-2e-4, 0.0, 9.0]))
    f = so.features(G, h, v1, v2, z, th, 0.004, ext, 0.1, 0.01, 10.0, 0.5, 1e-3, 2e-4)
    np.testing.assert_allclose(f[0, :6], [1.0, 5.0, 2.5, 0.3, 0.5, 0.04])
    np.testing.assert_allclose(f[0, 8:], [1.0, 2.0, -1.0])
    np.testing.assert_allclose(f[1, :6], [0.0, 0.0, 0.0, 0.4, 1.0, 0.04])
    np.testing.assert_array_equal(f[2], np.zeros(so.FEATURES))  # inactive


def test_extrapolation_of_still_water():
    """Lake at rest: the probe step changes nothing (well-balanced scheme, Sec. 2.2), so the
    extrapolation is exactly zero; with rain r on a flat lake only the depth grows, by
    window * r / theta."""
    sc = synth.lake_at_rest(nq=12, nr=10)
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    p = oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s)
    x = so.extrapolation(G, sc.z, sc.theta, sc.alpha_p, p, oracle.rain(), 0.0, 1.6,
                         sc.h0, sc.v10, sc.v20)
    for a in x:
        np.testing.assert_array_equal(a, 0.0)
    n = sc.n
    z = np.zeros(n)
    th = np.full(n, 0.8)
    r = 50.0 / 3.6e6
    x = so.extrapolation(G, z, th, np.full(n, 73.39), p, oracle.rain(0, r), 0.0, 1.6,
                         np.full(n, 0.3), np.zeros(n), np.zeros(n))
    np.testing.assert_allclose(x[0], 1.6 * r / 0.8, rtol=1e-9)
    np.testing.assert_array_equal(x[1], 0.0)
    np.testing.assert_array_equal(x[2], 0.0)


@pytest.mark.parametrize("side", [(oracle.WALL,) * 4, (oracle.WALL, oracle.PERIODIC) * 2])
def test_terrain_slope_is_exact_on_a_plane(side):
    """Every cell, also at the raster's edges and corners (one-sided differences), recovers
    the gradient of a plane; with a periodic side the wrap makes the plane non-planar across
    the seam, so only cells away from it are checked there."""
    nq, nr, a = 9, 7, 1.3
    G = oracle.grid(nq, nr, a, side=side)
    x, y = synth.centres(nq, nr, a)
    z = 0.07 * x - 0.13 * y + 2.0
    s = so.terrain_slope(G, z)
    q = np.tile(np.arange(nq), nr)
    keep = np.ones(G.n, bool) if side[1] == oracle.WALL else (q > 0) & (q < nq - 1)
    np.testing.assert_allclose(s[keep], np.tile([0.07, -0.13], (keep.sum(), 1)), rtol=1e-12)


def test_terrain_slope_of_a_cone_points_outward():
    sc = synth.cone(R=6, H=2.0)
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    s = so.terrain_slope(G, sc.z)
    x, y = synth.centres(sc.nq, sc.nr, sc.a)
    c = (sc.nr // 2) * sc.nq + sc.nq // 2
    dx, dy = x - x[c], y - y[c]
    inner = G.active & (np.hypot(dx, dy) > 1.0) & (G.nbr >= 0).all(axis=1)
    # the cone falls away from its centre: the gradient points inward
    assert np.all(s[inner, 0] * dx[inner] + s[inner, 1] * dy[inner] < 0)


def test_window_rain_depth():
    i = 100.0 / 3.6e6
    assert so.window_rain_depth(0, i, 0.0, float("inf"), 10.0, 1.6, 16) == pytest.approx(1.6 * i)
    # rain stops at T_d: sub-steps ending after it add nothing
    assert so.window_rain_depth(0, i, 0.0, 11.0, 10.0, 1.6, 16) == pytest.approx(1.0 * i)
    # triangular hyetograph: the right-endpoint sum tends to the integral (area i T_d / 2)
    T = 1800.0
    tot = sum(so.window_rain_depth(1, i, 0.25 * T, T, w * 1.6, 1.6, 16) for w in range(1125))
    assert tot == pytest.approx(0.5 * i * T, rel=1e-3)


def test_gate_residual_is_zero_on_an_exact_balance():
    S0, R, O0, O1, w = 100.0, 2.0, 0.5, 0.7, 1.6
    S1 = S0 + R - 0.5 * (O0 + O1) * w
    assert so.gate_residual(S0, S1, R, O0, O1, w) == pytest.approx(0.0, abs=1e-15)
    assert so.gate_residual(S0, S1 + 1.02, R, O0, O1, w) == pytest.approx(0.01)
