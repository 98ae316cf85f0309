"""Throughput of the hex-raster porous Saint-Venant time stepper on one MI355X.

One benchmark "step" is one explicit time step of the whole scheme over the
catchment: CFL bound, six-edge fluxes, mass update with rain and clamping,
closed-form friction solve, FP64 books.  The headline workload is the
4096 x 4096 fractal catchment (edge 2 m, 150 mm/h storm then recession) in
FP32, whose 604 MB per step streams from HBM (the largest single-domain
configuration); the line also carries the same catchment in FP64, the
1024 x 1024 catchment (its 38 MB stay in the 256 MB Infinity Cache, so it is
labelled cache-resident), the batched 256-scenario ensemble, the surrogate and
the FP64 oracle on the host.  Inputs are synthetic (seeded) and already
resident in HBM when the timed region starts.  The K timed steps are whole
replays of captured graphs (graph length = the largest divisor of K up to 100),
so the per-step figure does not depend on K.

Prints ONE JSON line:  python bench.py [--steps K] [--warmup W] [--workload c4|c2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "hex cell-updates/s: FP64 vs FP32 vs batched; surrogate speedup at ≤1% error"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell-update: read h, v1, v2, z, theta, alpha_p; write h, v1, v2
BYTES_PER_CELL = {"fp32": 9 * 4, "fp64": 9 * 8}

# Measured HBM bytes of one step-kernel launch: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB
# per dispatch, in runs of their own) scaled by what the same counters read for a plain 1 GiB
# device copy (x2.000 and x1.000); the summaries with their commands are
# profiles/k_step_catchment-4096x4096_fp32.md, profiles/k_step_catchment-4096x4096_fp64.md and
# profiles/k_ens_step_ensemble-256-catchments.md.
# A figure holds only for the kernel source it was taken on (digest below); otherwise the line
# reports null.
TRAFFIC = {
    ("catchment-4096x4096-edge2m-storm150mmh", "fp32", 4): {
        "bytes": 654594432, "digest": "46b96e45981a54c7"},
    ("catchment-4096x4096-edge2m-storm150mmh", "fp64", 2): {
        "bytes": 1245442368, "digest": "46b96e45981a54c7"},
}
# the batched ensemble's k_ens_step (64 x 16 tiles) per launch over all 256 scenarios, 300 s
# into the storms (the timed launches)
ENS_TRAFFIC = {("fp32", 2): {"bytes": 1105684704, "digest": "944c3fd997bee966"}}


# Surrogate network FLOPs per cell (7 taps, 4 layers): what the MFMA units execute (11 input
# features padded to 16 channels, 3 outputs to 16) and the algorithmic count (11 and 3).
NET_FLOP_EXECUTED = 2 * 7 * (16 * 32 + 32 * 32 + 32 * 32 + 32 * 16)
NET_FLOP_ALGORITHMIC = 2 * 7 * (11 * 32 + 32 * 32 + 32 * 32 + 32 * 3)


def step_kernel_digest():
    """Digest of the source of the step kernel (device helpers, tile phases, and k_step
    with its launchers: the part of hexsv_kernels.h from its namespace to k_prime)."""
    d = os.path.join(ROOT, "paper_2406_14933_amd", "csrc")
    h = hashlib.sha256()
    for f in ("hexsv_device.h", "hexsv_tile.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(d, "hexsv_kernels.h"), "rb") as fh:
        txt = fh.read()
    h.update(txt[txt.index(b"namespace hexsv {"):txt.index(b"void k_prime(")])
    return h.hexdigest()[:16]


def traffic_of(wname, precision, tile):
    t = TRAFFIC.get((wname, precision, tile))
    return t["bytes"] if t and t["digest"] == step_kernel_digest() else None


def ens_kernel_digest():
    """Digest of the batched ensemble step kernel's source (with the tile phases)."""
    d = os.path.join(ROOT, "paper_2406_14933_amd", "csrc")
    h = hashlib.sha256()
    for f in ("hexsv_device.h", "hexsv_tile.h", "hexsv_ensemble.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def ens_traffic_of(precision, tile):
    t = ENS_TRAFFIC.get((precision, tile))
    return t["bytes"] if t and t["digest"] == ens_kernel_digest() else None


def workload(name):
    import synth
    if name == "c2":
        return synth.c2_catchment(), "catchment-1024x1024-edge2m-rain100mmh"
    if name == "c4":
        return synth.c4_large(), "catchment-4096x4096-edge2m-storm150mmh"
    if name == "c1":
        return synth.c1_planar(), "planar-64x64-edge1m-slope5pct"
    raise SystemExit(f"unknown workload {name}")


def graph_length(steps):
    """Largest divisor of the timed step count up to 100: the timed run is whole replays."""
    return max(d for d in range(1, min(steps, 100) + 1) if steps % d == 0)


SPIN_UP_S = 300.0  # simulated time of the storm before the timed steps (setup, untimed)


def time_gpu(sc, wname, precision, steps, warmup, tile, spin_up=SPIN_UP_S):
    """Time `steps` solver steps (whole graph replays) after `warmup` steps.

    The timed state is the catchment `spin_up` seconds into its storm, which the setup
    reaches with the solver itself: a wet, flowing catchment, as over most of the run (the
    first steps from the dry start are unrepresentative: nearly every cell is dry).

    The step kernel's duration is taken inside the graphs: hipEvents on the simulation's
    stream around the timed replays, divided by the steps they took (each step is one
    launch; the per-replay fold and the launch gaps are included, so this is an upper bound
    on the kernel's own duration).  Back-to-back launches outside graphs are reported too."""
    import torch
    from paper_2406_14933_amd import hexsv
    spg = graph_length(steps)
    sim = hexsv.Sim.from_scenario(sc, precision, tile=tile, steps_per_graph=spg)
    sim.run(min(spin_up, sc.t_end))
    t_end = 1e30  # never reached: the step count bounds the run
    sim.run(t_end, max_steps=max(warmup, 1))
    torch.cuda.synchronize()
    sim.timing(True)
    b0 = sim.books()
    t0 = time.perf_counter()
    sim.run(t_end, max_steps=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = sim.timing()
    b1 = sim.books()
    sim.timing(False)
    assert b1["steps"] - b0["steps"] == steps, (b0["steps"], b1["steps"])
    graph_us = 1e3 * tm["gpu_ms"] / max(tm["steps"], 1)
    iso_us = 1e3 * sim.time_kernel(max(20, min(200, steps)))
    cells = sim.grid.active_cells
    bpc = BYTES_PER_CELL[precision]
    achieved = bpc * cells / (graph_us * 1e-6) / 1e9
    return {
        "wall_s": wall,
        "value": cells * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "graph_replays": tm["replays"],
        "steps_per_graph": spg,
        "kernel_us": graph_us,
        "isolated_kernel_us": iso_us,
        "cells": cells,
        "info": sim.info(),
        "residual": b1["residual"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_of(wname, precision, sim.info()["tile"]),
                     "kernel": "k_step", "kernel_us": graph_us,
                     "kernel_us_source": "in-graph hipEvents per step",
                     "isolated_kernel_us": iso_us, "bytes_per_cell": bpc,
                     "bytes_per_launch": bpc * cells},
    }


def time_ensemble(precision, launches, ksteps, n_scen, tune, spin_up=SPIN_UP_S):
    """Batched ensemble of uneven catchments: every scenario advances `launches * ksteps`
    steps; the mode (persistent kernel or batched steps) and tile come from the autotuner.
    As for the single catchment, the timed steps start `spin_up` seconds into the storms
    (the setup runs every scenario there with the solver itself), on wet, flowing
    catchments; the scenarios reach it at different step counts."""
    import torch

    import synth
    from paper_2406_14933_amd import hexsv
    scs = synth.c3_ensemble(n_scen=n_scen)
    ens = hexsv.Ensemble.from_scenarios(scs, precision, steps_per_launch=ksteps)
    del scs
    if tune:
        ens.autotune(ksteps=10)
    ens.run([spin_up] * n_scen)
    ens.run([1e30] * n_scen, max_steps=ksteps)  # warm-up launch
    torch.cuda.synchronize()
    ens.timing(True)
    t0 = time.perf_counter()
    ens.run([1e30] * n_scen, max_steps=launches * ksteps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ens.timing()
    ens.timing(False)
    info = ens.info()
    bpc = BYTES_PER_CELL[precision]
    achieved = bpc * tm["cell_updates"] / (tm["gpu_ms"] * 1e-3) / 1e9
    kernel = "k_ensemble" if info["mode"] == "persistent" else "k_ens_step"
    return {"value": tm["cell_updates"] / wall, "cells": info["cells"], "scenarios": n_scen,
            "steps_per_scenario": launches * ksteps, "wall_s": wall,
            "gpu_value": tm["cell_updates"] / (tm["gpu_ms"] * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": (ens_traffic_of(precision, info["tile"])
                                     if info["mode"] == "batched" else None),
                         "kernel": kernel, "kernel_us_source": "hipEvents around the step graphs "
                                                               "(k_ens_step and k_ens_finalize)",
                         "bytes_per_cell": bpc, "bytes_per_launch": bpc * info["cells"]},
            "info": info}


def surrogate_block(n_train=16, n_test=100, size=512, k=16, tol=3e-5, seed=1, dt_scale=3.2,
                    rounds=3, train_steps=6000):
    """The window surrogate (512 x 512 scenarios of the ensemble distribution): trained on
    FP32 solver trajectories with the library's own kernels, then evaluated on `n_test`
    held-out seeds against the plain FP32 solver, seed by seed (the single-sample regime),
    beside the same windows with a zero network (the probe step's extrapolation alone), and
    the costs of the batched regime: the plain solver on all held-out seeds as one ensemble
    and one network call over the whole batch.  The training settings (rounds of pairs
    from the network's own runs, Adam steps per round) were chosen on validation seeds
    2000.. of the same distribution, not on the held-out seeds."""
    import numpy as np

    import synth
    from paper_2406_14933_amd import hexsv
    from paper_2406_14933_amd import surrogate as S
    t_end = 1800.0
    train_sc = [synth.ensemble_member(s, size=size, config=5, t_end=t_end) for s in range(n_train)]
    test_sc = [synth.ensemble_member(1000 + s, size=size, config=5, t_end=t_end)
               for s in range(n_test)]
    def log(m):
        print(f"[bench] surrogate: {m}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    dt_fix = dt_scale * min(S.pilot_dt(sc) for sc in train_sc[:2])
    window = k * dt_fix
    sur = hexsv.Surrogate(4, 32, k=k)
    rng = np.random.default_rng(seed)
    # He-normal start, last layer scaled down: the network starts near the probe extrapolation
    p = []
    for li, (ci, co) in enumerate([(hexsv.Surrogate.FEATURES, 32), (32, 32), (32, 32), (32, 3)]):
        std = math.sqrt(2.0 / (7 * ci)) * (0.1 if li == 3 else 1.0)
        p.append(rng.normal(scale=std, size=co * ci * 7))
        p.append(np.zeros(co))
    sur.set_params(np.concatenate(p).astype(np.float32))
    times = list(np.linspace(window, t_end - 2 * window, 32))
    log(f"collecting windows from {n_train} training runs")
    data, scales = S.collect(train_sc, times, window, k, sur)
    S.train(sur, data, train_steps, batch=4, lr=1e-3, lr_end=5e-5, seed=seed, log=log)
    for rnd in range(rounds):  # pairs from the network's own runs, then more training
        log(f"rollout pairs, round {rnd}")
        ro = S.rollout_pairs(sur, train_sc, list(np.linspace(2 * window, t_end - 2 * window, 16)),
                             window, k, scales, tol=tol)
        data = S.merge(data, ro)
        S.train(sur, data, train_steps, batch=4, lr=5e-4, lr_end=2e-5, seed=seed + 1 + rnd,
                log=log)
    train_s = time.perf_counter() - t0
    print(f"[bench] surrogate: trained in {train_s:.0f} s; evaluating {n_test} held-out seeds",
          file=sys.stderr, flush=True)
    ev = S.evaluate(sur, test_sc, window, k, tol, project=True, log=log)
    zero = hexsv.Surrogate(4, 32, k=k)
    zero.set_params(np.zeros(zero.num_params, np.float32))
    zero.set_scales(scales.as_list())
    ev0 = S.evaluate(zero, test_sc, window, k, tol, project=True, log=log)
    print(f"[bench] surrogate: {ev['speedup']:.2f}x (zero network {ev0['speedup']:.2f}x)",
          file=sys.stderr, flush=True)
    batched = batched_regime(sur, test_sc, window, t_end)

    def summary(e):
        plain_steps = sum(r["plain_steps"] for r in e["rows"])
        sur_steps = sum(r["surrogate_steps"] for r in e["rows"])
        return {"speedup": e["speedup"], "err_h_max": e["err_h_max"],
                "err_h_mean": e["err_h_mean"], "accept_frac": e["accept_frac"],
                "solver_steps_avoided": 1.0 - sur_steps / max(plain_steps, 1),
                "refused": {kk: e[kk] for kk in ("refused_residual", "refused_wave_speed",
                                                 "refused_nonfinite")},
                "plain_s": e["plain_s"], "surrogate_s": e["surrogate_s"]}

    out = {"workload": f"surrogate-{n_test}-heldout-{size}x{size}-edge1m-to-{t_end:.0f}s",
           "regime": "single-sample: each held-out seed alone, solver and surrogate timed "
                     "seed by seed", **summary(ev), "tol": tol, "window_s": window, "k": k,
           "zero_network": summary(ev0), "batched": batched,
           "train_pairs": data.pairs, "train_scenarios": n_train, "train_rounds": rounds,
           "train_steps_per_round": train_steps, "train_s": train_s}
    return out


def batched_regime(sur, scs, window, t_end):
    """What the held-out batch costs as one batch: the plain FP32 solver on every seed as one
    batched ensemble to t_end, and one network call over the whole batch (random inputs; the
    cost does not depend on them).  A window advances every seed by `window` seconds, which
    the batched solver covers in window / t_end of its run (its launches go at the pace of
    the seed with the smallest steps), and needs at least the network call and a probe
    step: that time over (call + 1 step) bounds the speed-up a surrogate of this network
    could reach on the batch if it kept every window.  No batched surrogate runner is
    built, so this is a bound, not a measurement."""
    import numpy as np
    import torch

    from paper_2406_14933_amd import hexsv
    n = len(scs)
    nq, nr = scs[0].nq, scs[0].nr
    ens = hexsv.Ensemble.from_scenarios(scs, "fp32", mode="batched")
    ens.autotune(ksteps=3)
    torch.cuda.synchronize()
    ens.timing(True)
    t0 = time.perf_counter()
    ens.run([t_end] * n)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ens.timing()
    steps = [ens.books(s)["steps"] for s in range(n)]
    cells = ens.info()["cells"]
    del ens
    step_ms = wall * 1e3 / max(steps)  # one launch advances every live scenario
    f = torch.randn((n * nq * nr, hexsv.Surrogate.FEATURES), dtype=torch.float32, device="cuda")
    sur.forward(f, nq, nr)  # sizes the workspace
    torch.cuda.synchronize()
    calls = []
    for _ in range(3):
        t1 = time.perf_counter()
        sur.forward(f, nq, nr)
        torch.cuda.synchronize()
        calls.append(time.perf_counter() - t1)
    call_ms = 1e3 * min(calls)
    del f
    torch.cuda.empty_cache()
    flop = NET_FLOP_EXECUTED * n * nq * nr
    win_ms = 1e3 * wall * window / t_end  # the batched solver's time for one window span
    return {"scenarios": n, "cells": cells, "plain_s": wall,
            "plain_cell_updates_per_s": tm["cell_updates"] / wall,
            "plain_step_ms": step_ms, "steps_max": max(steps),
            "network_call_ms": call_ms, "network_tflops": flop / (call_ms * 1e-3) / 1e12,
            "network_mfma_frac": flop / (call_ms * 1e-3) / 2.5e15,
            "window_vs_steps": f"a {window:.2f} s window = {window * max(steps) / t_end:.0f} "
                               f"launches of the batch = {win_ms:.2f} ms",
            "speedup_bound": win_ms / (call_ms + step_ms)}


def window_cost(size=512, nwin=256, window=0.69, k=16):
    """Device cost of one surrogate window against the plain steps it replaces, on still
    water (every window is kept, so chains run unbroken): 512 x 512 dyadic lake at rest."""
    import numpy as np
    import torch

    import synth
    from paper_2406_14933_amd import hexsv
    sc = synth.lake_at_rest(nq=size, nr=size)
    sur = hexsv.Surrogate(4, 32)
    sur.set_params(np.zeros(sur.num_params, np.float32))
    sur.set_scales([0.03, 0.015, 100.0, 2e-5, 1.5e-5, 0.2])
    t0 = 8 * window
    s = hexsv.Sim.from_scenario(sc, "fp32")
    s.run_surrogate(sur, t0, window, k, math.inf)  # captures the window graph
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    acc, _ = s.run_surrogate(sur, t0 + nwin * window, window, k, math.inf)
    torch.cuda.synchronize()
    tw = time.perf_counter() - w0
    p = hexsv.Sim.from_scenario(sc, "fp32")
    p.run(t0)
    b0 = p.books()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    p.run(t0 + nwin * window)
    torch.cuda.synchronize()
    tp = time.perf_counter() - w0
    steps = p.books()["steps"] - b0["steps"]
    return {"workload": f"still-water-{size}x{size}", "windows": acc,
            "window_us": 1e6 * tw / nwin, "plain_step_us": 1e6 * tp / steps,
            "plain_steps_per_window": steps / nwin}


def network_cost(batch=16, size=512, calls=5, fused=False):
    """Device cost of one surrogate network call over a batch of 512 x 512 samples (random
    inputs and parameters: the cost does not depend on them), for the MFMA profile; fused:
    the one-kernel forward instead of the layer chain."""
    import numpy as np
    import torch

    from paper_2406_14933_amd import hexsv
    sur = hexsv.Surrogate(4, 32)
    sur.set_fused(fused)
    rng = np.random.default_rng(3)
    sur.set_params(rng.normal(scale=0.05, size=sur.num_params).astype(np.float32))
    f = torch.randn((batch * size * size, hexsv.Surrogate.FEATURES), dtype=torch.float32,
                    device="cuda")
    sur.forward(f, size, size)
    torch.cuda.synchronize()
    ms = []
    for _ in range(calls):
        t0 = time.perf_counter()
        sur.forward(f, size, size)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    cells = batch * size * size
    flop = NET_FLOP_EXECUTED * cells
    return {"workload": f"network-{batch}x{size}x{size}", "fused": fused, "call_ms": min(ms),
            "tflops": flop / (min(ms) * 1e-3) / 1e12, "mfma_frac": flop / (min(ms) * 1e-3) / 2.5e15,
            "flop_per_call": flop, "algorithmic_flop_per_call": NET_FLOP_ALGORITHMIC * cells}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads():
    """Threads the host gives this process: OMP_NUM_THREADS when set (the GPU machine sets its
    CPU share there), else the CPUs this process may run on."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), avail or int(env))
    return avail or 1


def cpu_baseline(sc, budget_s=12.0, budget_1_s=8.0):
    """The FP64 oracle as it stands on the host: on every thread this process has and on one
    thread, each over a bounded number of steps of the same workload from its dry start."""
    import numpy as np

    import oracle
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    p = oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s)
    r = oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
    cells = int(np.count_nonzero(G.active))
    out = {}
    for label, threads, budget in (("all", host_threads(), budget_s), ("one", 1, budget_1_s)):
        t0 = time.perf_counter()  # one probe step to size the sample
        h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10,
                                     sc.v20, 1e30, max_steps=1, nthreads=threads)
        per = time.perf_counter() - t0
        k = int(max(2, min(2000, budget / max(per, 1e-9))))
        t0 = time.perf_counter()
        oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, h, v1, v2, 1e30, max_steps=k, books=b,
                   nthreads=threads)
        dt = time.perf_counter() - t0
        out[label] = {"value": cells * k / dt, "threads": threads, "steps": k, "seconds": dt}
        print(f"[bench] cpu oracle, {threads} thread(s): {cells * k / dt:.3e} cell-updates/s",
              file=sys.stderr, flush=True)
    a = out["all"]
    return {"value": a["value"], "unit": "cell-updates/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": f"{a['steps']} FP64 steps of the full {sc.nq}x{sc.nr} raster after its "
                      f"first step from the dry start, {a['seconds']:.1f} s on {a['threads']} "
                      f"OpenMP threads; one thread: {out['one']['steps']} steps in "
                      f"{out['one']['seconds']:.1f} s",
            "single_thread_value": out["one"]["value"], "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c4", choices=["c4", "c2", "c1"])
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--side-steps", type=int, default=400,
                    help="steps of the 1024x1024 (cache-resident) side entry (0: skip)")
    ap.add_argument("--ensemble-launches", type=int, default=4,
                    help="timed launches of the 256-scenario batched ensemble (0: skip)")
    ap.add_argument("--ensemble-ksteps", type=int, default=25)
    ap.add_argument("--ensemble-scenarios", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip training and timing the window surrogate")
    ap.add_argument("--surrogate-seeds", type=int, default=100,
                    help="held-out 512x512 seeds of the surrogate evaluation")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--window-cost", action="store_true",
                    help="only time surrogate windows against plain steps on still water")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for counter calibration)")
    ap.add_argument("--network-cost", action="store_true",
                    help="only time the surrogate network over a batch of 16 512x512 samples")
    ap.add_argument("--network-fused", action="store_true",
                    help="with --network-cost: the one-kernel forward (k_hexnet4)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design (row strips with one halo row per step and a max all-reduce of dt) is "
              "described but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.window_cost:
        print(json.dumps(window_cost()))
        return
    if args.network_cost:
        print(json.dumps(network_cost(fused=args.network_fused)))
        return
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "launches": 5}))
        return
    sc, wname = workload(args.workload)
    print(f"[bench] workload {wname}: {sc.n} cells, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    main_run = time_gpu(sc, wname, args.precision, args.steps, args.warmup, args.tile)
    print(f"[bench] {args.precision}: {main_run['value']:.3e} cell-updates/s, step "
          f"{main_run['kernel_us']:.1f} us in graphs ({main_run['isolated_kernel_us']:.1f} us "
          f"back to back)", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "cells": main_run["cells"], "edge_m": sc.a,
                   "precision": args.precision, "timed_from_s": SPIN_UP_S,
                   "tile": main_run["info"],
                   "steps_per_graph": main_run["steps_per_graph"],
                   "graph_replays": main_run["graph_replays"]},
        "roofline": main_run["roofline"],
        "books_residual": main_run["residual"],
    }
    if not args.no_fp64 and args.precision == "fp32":
        other = time_gpu(sc, wname, "fp64", args.steps, args.warmup, args.tile)
        print(f"[bench] fp64: {other['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
        line["fp64"] = {"workload": wname, "value": other["value"],
                        "ms_per_step": other["ms_per_step"], "roofline": other["roofline"],
                        "books_residual": other["residual"]}
    if args.side_steps > 0 and args.workload != "c2":
        del sc
        side, sname = workload("c2")
        print(f"[bench] side: {sname}", file=sys.stderr, flush=True)
        entry = {"workload": sname, "cache_resident": True,
                 "note": "37.7 MB (FP32) per step stay in the 256 MB Infinity Cache: the "
                         "fraction of 8 TB/s is not an HBM figure"}
        for prec in ("fp32", "fp64"):
            sr = time_gpu(side, sname, prec, args.side_steps, 50, args.tile)
            print(f"[bench] side {prec}: {sr['value']:.3e} cell-updates/s", file=sys.stderr,
                  flush=True)
            entry[prec] = {"value": sr["value"], "ms_per_step": sr["ms_per_step"],
                           "steps": args.side_steps, "roofline": sr["roofline"]}
        line["cache_resident"] = entry
        sc = None
    if args.ensemble_launches > 0:
        print("[bench] batched ensemble", file=sys.stderr, flush=True)
        er = time_ensemble(args.precision, args.ensemble_launches, args.ensemble_ksteps,
                           args.ensemble_scenarios, tune=True)
        print(f"[bench] batched {args.precision}: {er['value']:.3e} cell-updates/s",
              file=sys.stderr, flush=True)
        line["batched"] = {"workload": f"ensemble-{er['scenarios']}-catchments-128..512sq",
                           "value": er["value"], "cells": er["cells"],
                           "steps_per_scenario": er["steps_per_scenario"],
                           "timed_from_s": SPIN_UP_S,
                           "roofline": er["roofline"], "config": er["info"]}
    if args.surrogate:
        print("[bench] surrogate: training on solver trajectories", file=sys.stderr, flush=True)
        sr = surrogate_block(n_test=args.surrogate_seeds)
        sr["window_cost"] = window_cost()
        print(f"[bench] surrogate: speed-up {sr['speedup']:.2f}x at rel L1 error "
              f"{sr['err_h_max']:.2e} (max over held-out); batched bound "
              f"{sr['batched']['speedup_bound']:.2f}x", file=sys.stderr, flush=True)
        line["surrogate"] = sr
    if not args.no_cpu:
        if sc is None:
            sc, _ = workload(args.workload)
        line["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
