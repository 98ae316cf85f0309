"""FP64 oracle of the learned hex-convolution surrogate — TEST INFRASTRUCTURE.

The surrogate is not part of the paper's method: it is a small residual
network that maps the solver state at time t to the state change after k
explicit steps, used with the paper's solver as fallback and as the reference
for its error.  This module defines its arithmetic plainly so the GPU kernels
can be checked:

  features  x0 (N x 11): h/H, q1/Q, q2/Q, z/Z, theta, (rain depth of the window)/H,
                         the terrain slope (dz/dx, dz/dy)/S, and the change of one probe step
                         of the scheme scaled to the window, (x_h/dH, x_q1/dQ, x_q2/dQ)
  layer l:  y = b + sum_{c, t} W[o, c, t] * x[c, nbr_t(i)]   (hex_conv; tap 0 = the cell,
            tap 1+k = its neighbour in direction k, zero outside the raster)
            ReLU after layers 1..L-1; the last layer gives 3 channels
  output:   (dh/H, dq1/Q, dq2/Q) predicted for the window
  loss:     mean over cells, samples and the 3 channels of |pred - target|

``bf16=True`` rounds, as the GPU does, the features and every hidden activation to
bfloat16 (round to nearest even) and the loss gradient entering each backward layer,
while accumulating in FP64.  Parameters are a flat FP32-compatible vector laid out
layer by layer as W[o][c][t] (o < cout, c < cin, t < 7) followed by b[o].
"""
from __future__ import annotations

import math

import numpy as np

import oracle

FEATURES = 11
OUTPUTS = 3
TAPS = 7


def layer_shapes(layers=4, channels=32):
    """[(cin, cout)] of each hex-conv layer."""
    dims = [FEATURES] + [channels] * (layers - 1) + [OUTPUTS]
    return [(dims[i], dims[i + 1]) for i in range(layers)]


def num_params(layers=4, channels=32):
    return sum(co * ci * TAPS + co for ci, co in layer_shapes(layers, channels))


def unflatten(p, layers=4, channels=32):
    out, k = [], 0
    for ci, co in layer_shapes(layers, channels):
        W = np.asarray(p[k:k + co * ci * TAPS], np.float64).reshape(co, ci, TAPS)
        k += co * ci * TAPS
        b = np.asarray(p[k:k + co], np.float64)
        k += co
        out.append((W, b))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params])


def init_params(seed, layers=4, channels=32, out_scale=0.1):
    """He-normal weights (fan-in = 7 cin), zero biases, last layer scaled down."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = layer_shapes(layers, channels)
    for li, (ci, co) in enumerate(shapes):
        W = rng.normal(0.0, np.sqrt(2.0 / (TAPS * ci)), size=(co, ci, TAPS))
        if li == len(shapes) - 1:
            W *= out_scale
        parts.append((W, np.zeros(co)))
    return flatten(parts).astype(np.float32)


def bf16_round(a):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(a32), a32, out)
    return out.astype(np.float64)


def _conv(G, x, W, b):
    """x: (N, cin) -> (N, cout) via the C oracle's channel-major hex_conv."""
    y = oracle.hexconv_fwd(G, np.ascontiguousarray(x.T), W, b)
    return y.T


def _conv_bwd(G, x, W, dy):
    dx, dW, db = oracle.hexconv_bwd(G, np.ascontiguousarray(x.T), W, np.ascontiguousarray(dy.T))
    return dx.T, dW, db


def forward(G, p, x0, layers=4, channels=32, bf16=True):
    """Per-sample forward: x0 (N, 11) -> (output (N, 3), saved activations)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    params = unflatten(p, layers, channels)
    if bf16:
        params = [(bf16_round(W), np.asarray(b, np.float32).astype(np.float64)) for W, b in params]
    acts = [rnd(x0)]
    for li, (W, b) in enumerate(params):
        y = _conv(G, acts[-1], W, b)
        if li < len(params) - 1:
            acts.append(rnd(np.maximum(y, 0.0)))
        else:
            acts.append(y)
    return acts[-1], acts, params


def loss_and_grad(G, p, xs, targets, layers=4, channels=32, bf16=True):
    """Mean L1 loss over a batch and its gradient with respect to the flat parameters."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    B = len(xs)
    total = 0.0
    grads = None
    count = B * G.n * OUTPUTS
    for x0, tgt in zip(xs, targets):
        out, acts, params = forward(G, p, x0, layers, channels, bf16)
        diff = out - tgt
        total += np.abs(diff).sum()
        dy = np.sign(diff) / count
        gl = []
        for li in range(len(params) - 1, -1, -1):
            W, _ = params[li]
            dyr = rnd(dy)
            dx, dW, db = _conv_bwd(G, acts[li], W, dyr)
            gl.append((dW, db))
            if li > 0:
                dy = dx * (acts[li] > 0)
        gl = gl[::-1]
        g = flatten(gl)
        grads = g if grads is None else grads + g
    return total / count, grads


def adam_update(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on FP64 copies; returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------ surrogate windows
#
# A window advances the solver state by a fixed time span with one network
# call instead of the explicit steps; it is accepted only if the predicted
# state keeps the water balance the scheme conserves (stored volume = initial
# + rain - outflow - clamped; Sec. 4.2, Table BasinSusita reports the same
# balance).  Below are the plain definitions of the pieces.

def terrain_slope(G, z):
    """(dz/dx, dz/dy) per cell from its neighbours along the three axes of the hexagon.

    Along axis k < 3 (directions k and k+3; neighbour centres at distance sqrt(3) a along
    the edge normals +-n_k) the slope estimate is d_k = D_k / (2 sqrt(3) a), with
    D_k = z_k - z_{k+3}, or twice the one-sided difference when one of the two edges is not
    INTERIOR; axes with neither neighbour are skipped.  The gradient is the least-squares
    (minimum-norm) fit of n_k . grad z = d_k over the axes present, exact for a plane when
    two or three axes are present."""
    z = np.asarray(z, np.float64)
    s = np.zeros((G.n, 2))
    for i in range(G.n):
        M = np.zeros((2, 2))
        b = np.zeros(2)
        for k in range(3):
            j, m = G.nbr[i, k], G.nbr[i, k + 3]
            if j >= 0 and m >= 0:
                d = z[j] - z[m]
            elif j >= 0:
                d = 2.0 * (z[j] - z[i])
            elif m >= 0:
                d = 2.0 * (z[i] - z[m])
            else:
                continue
            n = np.array(oracle.normal(k))
            M += np.outer(n, n)
            b += n * d / (2.0 * math.sqrt(3.0) * G.a)
        s[i] = np.linalg.pinv(M) @ b
    return s


def extrapolation(G, z, theta, alpha_p, p, r, t0, window, h, v1, v2):
    """Change of one probe step of the scheme scaled to the window: (x_h, x_q1, x_q2).

    The probe step is the solver's next step from the state at t0 (dt = min(dt_max, CFL
    bound), rain at t0 + dt; eq. fvm_2D_eq_frac.07 with Appendix A); x = (window/dt) times its
    change of h and of q = theta h v."""
    th = np.where(G.active, np.asarray(theta, np.float64), 0.0)
    h, v1, v2 = (np.asarray(a, np.float64) for a in (h, v1, v2))
    dt = oracle.dt(G.a, p, oracle.cmax(G, p.g, th, h, v1, v2), t0, math.inf)
    cells = np.nonzero(G.active)[0]
    hn, v1n, v2n = h.copy(), v1.copy(), v2.copy()  # inactive cells: no change
    hn[cells], v1n[cells], v2n[cells], _ = oracle.step_cells(G, z, th, alpha_p, p, r, dt, t0 + dt,
                                                            h, v1, v2, cells)
    xs = window / dt
    return xs * (hn - h), xs * (th * hn * v1n - th * h * v1), xs * (th * hn * v2n - th * h * v2)


def features(G, h, v1, v2, z, theta, rain_depth, ext, H, Q, Z, S, dH, dQ):
    """Network input (N, 11) of a state: h/H, theta h v1/Q, theta h v2/Q, z/Z, theta, depth/H,
    (dz/dx)/S, (dz/dy)/S, x_h/dH, x_q1/dQ, x_q2/dQ with ext = (x_h, x_q1, x_q2) of
    :func:`extrapolation`.  All channels but theta are zero on inactive cells (theta = 0).

    Absolute elevation is kept as a channel, but bfloat16 cannot resolve the differences of
    neighbouring elevations that drive the flow, so the slope enters as channels of its own;
    likewise the probe step supplies, at full precision, the flux divergence that is a small
    difference of large discharges."""
    h, v1, v2, z, th = (np.asarray(a, np.float64) for a in (h, v1, v2, z, theta))
    act = th > 0.0
    sl = terrain_slope(G, z)
    f = np.zeros((h.size, FEATURES))
    f[:, 0] = np.where(act, h / H, 0.0)
    f[:, 1] = np.where(act, th * h * v1 / Q, 0.0)
    f[:, 2] = np.where(act, th * h * v2 / Q, 0.0)
    f[:, 3] = np.where(act, z / Z, 0.0)
    f[:, 4] = th
    f[:, 5] = np.where(act, rain_depth / H, 0.0)
    f[:, 6] = np.where(act, sl[:, 0] / S, 0.0)
    f[:, 7] = np.where(act, sl[:, 1] / S, 0.0)
    f[:, 8] = np.where(act, ext[0] / dH, 0.0)
    f[:, 9] = np.where(act, ext[1] / dQ, 0.0)
    f[:, 10] = np.where(act, ext[2] / dQ, 0.0)
    return f


def apply_window(h, v1, v2, theta, out, dH, dQ, ext=None, m_min=1e-6):
    """State after a predicted window: h' = max(h + x_h + dH out0, 0),
    q' = theta h v + x_q + dQ (out1, out2), v' = q' / (theta h') where theta h' > m_min, else 0;
    inactive cells unchanged (x = 0 when ext is None)."""
    h, v1, v2, th = (np.asarray(a, np.float64) for a in (h, v1, v2, theta))
    out = np.asarray(out, np.float64)
    xh, xq1, xq2 = (0.0, 0.0, 0.0) if ext is None else ext
    act = th > 0.0
    hn = np.maximum(h + xh + dH * out[:, 0], 0.0)
    q1 = th * h * v1 + xq1 + dQ * out[:, 1]
    q2 = th * h * v2 + xq2 + dQ * out[:, 2]
    mn = th * hn
    wet = mn > m_min
    with np.errstate(divide="ignore", invalid="ignore"):
        v1n = np.where(wet, q1 / np.where(wet, mn, 1.0), 0.0)
        v2n = np.where(wet, q2 / np.where(wet, mn, 1.0), 0.0)
    return (np.where(act, hn, h), np.where(act, v1n, v1), np.where(act, v2n, v2))


def outflow_rate(G, g, z, theta, h, v1, v2):
    """Volume flux (m^3/s) leaving through the OUTFLOW edges: the F_out of every cell, summed."""
    cells = np.nonzero((G.code == oracle.OUTFLOW).any(axis=1) & G.active)[0]
    return float(sum(oracle.cell_sums(G, g, z, theta, h, v1, v2, int(i))[5] for i in cells))


def window_rain_depth(kind, i_a, t_a, T_d, t0, window, k):
    """Rain depth of a window of k equal sub-steps, each taking r at its end (eq. .05-1)."""
    dt = window / k
    return float(sum(dt * oracle.rain_rate(kind, i_a, t_a, T_d, t0 + j * dt) for j in range(1, k + 1)))


def gate_residual(S0, S1, R, O0, O1, window):
    """Relative water-balance residual of a predicted window:
    |S1 - S0 - (R - O)| / max(S0 + R, tiny), with O the trapezoid-rule outflow volume."""
    Ow = 0.5 * (O0 + O1) * window
    return abs(S1 - S0 - (R - Ow)) / max(S0 + R, 1e-300)
