"""Learned window surrogate of the solver: training data from solver trajectories, training on
the GPU with the library's BF16 MFMA kernels, and evaluation against the plain solver.

The surrogate is not part of the paper's method.  A window advances the state over a fixed
span ``window`` with one network call (``Sim.run_surrogate``); the library keeps a window
only if the predicted state closes the water balance of the scheme within a tolerance, and
otherwise solves that span.  This module supplies what that needs:

* ``collect``: pairs (state at t, state at t + window) of FP32 solver trajectories, run as one
  batched ensemble, turned into network inputs and normalised targets on the device;
* ``fit_scales``: normalisation from the data (root mean squares over active cells);
* ``train``: Adam on the mean L1 loss with a cosine learning-rate decay;
* ``evaluate``: plain FP32 solver against the surrogate run on held-out scenarios: relative
  L1 error of h at t_end, kept and solved windows, and wall-clock speed-up.

Every array stays in device memory; the host only orchestrates.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import hexsv


@dataclass
class Scales:
    H: float   # input depth (m)
    Q: float   # input discharge theta h v (m^2/s)
    Z: float   # input elevation (m)
    dH: float  # output depth change over a window (m)
    dQ: float  # output discharge change over a window (m^2/s)
    S: float   # input terrain slope (-)

    def as_list(self):
        return [self.H, self.Q, self.Z, self.dH, self.dQ, self.S]


@dataclass
class WindowData:
    """Training pairs of one raster shape (device tensors)."""
    nq: int
    nr: int
    feats: torch.Tensor   # (pairs, cells, 8) float32
    target: torch.Tensor  # (pairs, cells, 3) float32

    @property
    def pairs(self):
        return self.feats.shape[0]


@dataclass
class _Raw:
    s: int
    t: float
    h0: torch.Tensor
    q10: torch.Tensor
    q20: torch.Tensor
    v10: torch.Tensor
    v20: torch.Tensor
    dh: torch.Tensor
    dq1: torch.Tensor
    dq2: torch.Tensor


def pilot_dt(scenario, t_end=None):
    """Mean time step (s) of the plain FP32 solver on one scenario."""
    sim = hexsv.Sim.from_scenario(scenario, "fp32")
    sim.run(scenario.t_end if t_end is None else t_end)
    b = sim.books()
    return b["t"] / max(b["steps"], 1)


def _collect_raw(scenarios, times, window, k):
    n = len(scenarios)
    ens = hexsv.Ensemble.from_scenarios(scenarios, "fp32")
    raw = []
    for t in times:
        ens.run([t] * n)
        s0 = [ens.state(s) for s in range(n)]
        ens.run([t + window] * n)
        for s in range(n):
            a, b = s0[s], ens.state(s)
            raw.append(_Raw(
                s=s, t=t,
                h0=a["h"].float(), q10=a["q1"].float(), q20=a["q2"].float(),
                v10=a["v1"].float(), v20=a["v2"].float(),
                dh=(b["h"] - a["h"]).float(), dq1=(b["q1"] - a["q1"]).float(),
                dq2=(b["q2"] - a["q2"]).float()))
    return raw


def _rms(chunks):
    s = sum(float((c.double() ** 2).sum()) for c in chunks)
    n = sum(c.numel() for c in chunks)
    return math.sqrt(s / max(n, 1))


def fit_scales(scenarios, raw):
    """Root mean squares over active cells and samples (elevation: largest |z|)."""
    act = [torch.as_tensor(np.asarray(sc.theta) > 0, device="cuda") for sc in scenarios]
    H = _rms([r.h0[act[r.s]] for r in raw])
    Q = _rms([torch.cat([r.q10[act[r.s]], r.q20[act[r.s]]]) for r in raw])
    dH = _rms([r.dh[act[r.s]] for r in raw])
    dQ = _rms([torch.cat([r.dq1[act[r.s]], r.dq2[act[r.s]]]) for r in raw])
    Z = max(float(np.abs(sc.z).max()) for sc in scenarios)
    S = max(float(sc.meta.get("slope", 0.1)) for sc in scenarios)
    tiny = 1e-12
    return Scales(max(H, tiny), max(Q, tiny), max(Z, 1.0), max(dH, tiny), max(dQ, tiny), S)


def collect(scenarios, times, window, k, sur, scales=None):
    """Training pairs from FP32 solver trajectories of same-shape scenarios.

    Every scenario is advanced as one batched ensemble to each time in `times` and then by
    `window`.  A pair becomes the network input of the first state (``Sim.surrogate_features``:
    the window's rain depth and the probe step's change scaled to the window included) and
    the target (true change - probe extrapolation) / (dH, dQ, dQ), i.e. the correction the
    network has to supply.  Returns (data, scales)."""
    nq, nr = scenarios[0].nq, scenarios[0].nr
    if any((sc.nq, sc.nr) != (nq, nr) for sc in scenarios):
        raise ValueError("collect needs scenarios of one raster shape")
    raw = _collect_raw(scenarios, times, window, k)
    if scales is None:
        scales = fit_scales(scenarios, raw)
    sur.set_scales(scales.as_list())
    sims = [hexsv.Sim.from_scenario(sc, "fp32") for sc in scenarios]
    F = hexsv.Surrogate.FEATURES
    feats = torch.empty((len(raw), nq * nr, F), dtype=torch.float32, device="cuda")
    target = torch.empty((len(raw), nq * nr, 3), dtype=torch.float32, device="cuda")
    for p, r in enumerate(raw):
        sim = sims[r.s]
        sim.set_state(r.h0.double(), r.v10.double(), r.v20.double(), r.t)
        f = sim.surrogate_features(sur, window, k)
        feats[p] = f
        target[p, :, 0] = r.dh / scales.dH - f[:, 8]
        target[p, :, 1] = r.dq1 / scales.dQ - f[:, 9]
        target[p, :, 2] = r.dq2 / scales.dQ - f[:, 10]
    return WindowData(nq, nr, feats, target), scales


def rollout_pairs(sur, scenarios, times, window, k, scales, tol=1e-5):
    """Pairs whose start states come from surrogate runs of the scenarios, i.e. the states the
    network meets once it drives a simulation, with the plain solver's change over the
    window from each such state as the target (the same correction form as ``collect``).
    Training on them as well keeps a run from drifting away from the data it was fitted on.
    The runs try a window on every span (no back-off after refusals), so that they sample
    the states the network drives a run into wherever it is used."""
    nq, nr = scenarios[0].nq, scenarios[0].nr
    F = hexsv.Surrogate.FEATURES
    n = len(scenarios) * len(times)
    feats = torch.empty((n, nq * nr, F), dtype=torch.float32, device="cuda")
    target = torch.empty((n, nq * nr, 3), dtype=torch.float32, device="cuda")
    p = 0
    for sc in scenarios:
        run = hexsv.Sim.from_scenario(sc, "fp32")
        run.set_surrogate_backoff(0)
        probe = hexsv.Sim.from_scenario(sc, "fp32")
        th = torch.as_tensor(np.asarray(sc.theta, np.float64), device="cuda")
        for t in times:
            run.run_surrogate(sur, t, window, k, tol)
            a = run.state()
            probe.set_state(a["h"], a["v1"], a["v2"], t)
            f = probe.surrogate_features(sur, window, k)
            probe.run(t + window)
            b = probe.state()
            feats[p] = f
            target[p, :, 0] = ((b["h"] - a["h"]) / scales.dH).float() - f[:, 8]
            target[p, :, 1] = ((b["q1"] - a["q1"]) / scales.dQ).float() - f[:, 9]
            target[p, :, 2] = ((b["q2"] - a["q2"]) / scales.dQ).float() - f[:, 10]
            p += 1
    del th
    return WindowData(nq, nr, feats, target)


def merge(*sets: WindowData) -> WindowData:
    return WindowData(sets[0].nq, sets[0].nr, torch.cat([d.feats for d in sets]),
                      torch.cat([d.target for d in sets]))


def train(sur, data: WindowData, steps, batch=2, lr=2e-3, lr_end=1e-4, seed=0, log=None):
    """Adam on the mean L1 loss over random mini-batches, cosine decay lr -> lr_end.
    Returns the loss of every step."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(0, data.pairs, (batch,), generator=g).cuda()
        f = data.feats.index_select(0, idx).contiguous()
        t = data.target.index_select(0, idx).contiguous()
        rate = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
        losses.append(sur.train_step(f, t, data.nq, data.nr, rate))
        if log and (it % max(steps // 10, 1) == 0 or it == steps - 1):
            log(f"train step {it}: loss {losses[-1]:.4f} lr {rate:.2e}")
    return losses


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def evaluate(sur, scenarios, window, k, tol=1e-3, t_end=None, project=True, log=None):
    """Plain FP32 solver against the surrogate run, scenario by scenario, to t_end.

    Returns per-scenario rows (relative L1 error of h at t_end, kept and solved windows,
    wall times) and the totals."""
    rows = []
    for n, sc in enumerate(scenarios):
        if log and n % 10 == 0:
            log(f"evaluate scenario {n} of {len(scenarios)}")
        te = sc.t_end if t_end is None else t_end
        plain = hexsv.Sim.from_scenario(sc, "fp32")
        _, tp = _timed(lambda: plain.run(te))
        surr = hexsv.Sim.from_scenario(sc, "fp32")
        (acc, fb), ts = _timed(lambda: surr.run_surrogate(sur, te, window, k, tol, project))
        hp = plain.state()["h"]
        hs = surr.state()["h"]
        err = float((hs - hp).abs().sum() / hp.abs().sum().clamp_min(1e-300))
        st = surr.surrogate_stats()
        rows.append({"scenario": sc.name, "err_h": err, "accepted": acc, "fallback": fb,
                     "refused_residual": st["refused_residual"],
                     "refused_wave_speed": st["refused_wave_speed"],
                     "refused_nonfinite": st["refused_nonfinite"],
                     "plain_s": tp, "surrogate_s": ts, "plain_steps": plain.books()["steps"],
                     "surrogate_steps": surr.books()["steps"]})
    tp = sum(r["plain_s"] for r in rows)
    ts = sum(r["surrogate_s"] for r in rows)
    acc = sum(r["accepted"] for r in rows)
    fb = sum(r["fallback"] for r in rows)
    refused = {k: sum(r[k] for r in rows)
               for k in ("refused_residual", "refused_wave_speed", "refused_nonfinite")}
    return {"rows": rows, "speedup": tp / ts, "plain_s": tp, "surrogate_s": ts, **refused,
            "err_h_max": max(r["err_h"] for r in rows),
            "err_h_mean": sum(r["err_h"] for r in rows) / len(rows),
            "accepted": acc, "fallback": fb, "accept_frac": acc / max(acc + fb, 1)}
