"""FP64 oracle of the learned hex-convolution surrogate — TEST INFRASTRUCTURE.

The surrogate is not part of the paper's method: it is a small residual
network that maps the solver state at time t to the state change after k
explicit steps, used with the paper's solver as fallback and judge.  This
module defines its arithmetic plainly so the GPU kernels can be checked:

  features  x0 (N x 6):  h/H, q1/Q, q2/Q, z/Z, theta, (rain depth of the window)/H
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

import numpy as np

import oracle

FEATURES = 6
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
    """Per-sample forward: x0 (N, 6) -> (output (N, 3), saved activations)."""
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
