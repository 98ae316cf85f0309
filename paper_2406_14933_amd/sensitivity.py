"""Sensitivity of a steady flow to the friction coefficients (Sec. 3.4), run as one GPU ensemble.

For environmental variables p (a scenario factory) the sweep advances every point
(alpha_s^i, alpha_p^j) of a regular grid as one scenario of a batched ensemble to a time at
which the flow is steady, takes the mean depth hbar over a zone (eq. eq_h_bar) and forms the
mean forward differences delta_s and delta_p of hbar along the two axes of the grid.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import hexsv


def mean_depth(h: torch.Tensor, zone: torch.Tensor) -> float:
    """hbar of eq. eq_h_bar: the mean of h over the cells of the zone (on the device)."""
    return float((h * zone).sum() / zone.sum())


def deltas(H: np.ndarray, ds: float, dp: float):
    """delta_s, delta_p of Sec. 3.4 from H[i, j] = hbar(alpha_s^i, alpha_p^j)."""
    H = np.asarray(H, np.float64)
    if H.shape[0] < 2 or H.shape[1] < 2:
        raise ValueError("the grid needs at least two points along each axis")
    return float(np.diff(H, axis=0).mean() / ds), float(np.diff(H, axis=1).mean() / dp)


def sweep(scenarios, alpha_s, alpha_p, zone, t_end, precision="fp64", ensemble=None):
    """Run the grid alpha_s x alpha_p of every factory in `scenarios` as one ensemble.

    scenarios: list of callables (alpha_s, alpha_p) -> Scenario (one per environment p);
    zone: boolean cell mask (per factory, or one for all) over which hbar is taken;
    alpha_s, alpha_p: the regular grids (increasing, evenly spaced).
    Returns, per factory, {"H": (Ns, Np) hbar, "delta_s", "delta_p"} and the run's seconds.
    """
    a_s = np.asarray(alpha_s, np.float64)
    a_p = np.asarray(alpha_p, np.float64)
    ds, dp = float(np.diff(a_s).mean()), float(np.diff(a_p).mean())
    zones = zone if isinstance(zone, (list, tuple)) else [zone] * len(scenarios)
    scs = [make(s, p) for make in scenarios for s in a_s for p in a_p]
    ens = ensemble or hexsv.Ensemble.from_scenarios(scs, precision, mode="batched")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(t_end)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    out = []
    k = 0
    for f in range(len(scenarios)):
        z = torch.as_tensor(np.asarray(zones[f], np.float64), device="cuda")
        H = np.empty((len(a_s), len(a_p)))
        for i in range(len(a_s)):
            for j in range(len(a_p)):
                H[i, j] = mean_depth(ens.state(k)["h"], z)
                k += 1
        d_s, d_p = deltas(H, ds, dp)
        out.append({"H": H, "delta_s": d_s, "delta_p": d_p})
    return out, seconds
