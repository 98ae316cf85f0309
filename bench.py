"""Throughput of the hex-raster porous Saint-Venant time stepper on one MI355X.

One benchmark "step" is one explicit time step of the whole scheme over the
catchment: CFL bound, six-edge fluxes, mass update with rain and clamping,
closed-form friction solve, FP64 books.  The default workload is the 1024 x 1024
fractal catchment (edge 2 m, 100 mm/h rain) in FP32; the line also carries the
same workload in FP64.  Inputs are synthetic (seeded) and already resident in
HBM when the timed region starts.

Prints ONE JSON line:  python bench.py [--steps K] [--warmup W] [--workload c2|c4]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
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
# profiles/k_step_catchment-{4096x4096,1024x1024}_fp32.md (at 1024 x 1024 the working set sits
# in the Infinity Cache, whose hits these counters include).  A figure holds only for the
# kernel source it was taken on (digest below); otherwise the line reports null.
TRAFFIC = {
    ("catchment-4096x4096-edge2m-storm150mmh", "fp32", 2): {
        "bytes": 607022052, "digest": "2747f7c54e97d04c"},
    ("catchment-1024x1024-edge2m-rain100mmh", "fp32", 2): {
        "bytes": 38561426, "digest": "2747f7c54e97d04c"},
}


def step_kernel_digest():
    """Digest of the source of the step kernel (device helpers, tile phases, k_step)."""
    d = os.path.join(ROOT, "paper_2406_14933_amd", "csrc")
    h = hashlib.sha256()
    for f in ("hexsv_device.h", "hexsv_tile.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(d, "hexsv_kernels.h"), "rb") as fh:
        txt = fh.read()
    h.update(txt[:txt.index(b"void k_prime(")])
    return h.hexdigest()[:16]


def traffic_of(wname, precision, tile):
    t = TRAFFIC.get((wname, precision, tile))
    return t["bytes"] if t and t["digest"] == step_kernel_digest() else None


def workload(name):
    import synth
    if name == "c2":
        return synth.c2_catchment(), "catchment-1024x1024-edge2m-rain100mmh"
    if name == "c4":
        return synth.c4_large(), "catchment-4096x4096-edge2m-storm150mmh"
    if name == "c1":
        return synth.c1_planar(), "planar-64x64-edge1m-slope5pct"
    raise SystemExit(f"unknown workload {name}")


def time_gpu(sc, wname, precision, steps, warmup, tile, spg):
    """Time `steps` solver steps (graph replays) after `warmup`, then the step kernel alone."""
    import torch
    from paper_2406_14933_amd import hexsv
    sim = hexsv.Sim.from_scenario(sc, precision, tile=tile, steps_per_graph=spg)
    t_end = 1e30  # never reached: the step count bounds the run
    sim.run(t_end, max_steps=warmup)
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
    # the dominant kernel in isolation: back-to-back launches bracketed by hipEvents
    kern_ms = sim.time_kernel(max(20, min(200, steps // 10)))
    cells = sim.grid.active_cells
    bpc = BYTES_PER_CELL[precision]
    achieved = bpc * cells / (kern_ms * 1e-3) / 1e9
    return {
        "wall_s": wall,
        "value": cells * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "gpu_us_per_step": 1e3 * tm["gpu_ms"] / max(tm["steps"], 1),
        "kernel_us": kern_ms * 1e3,
        "cells": cells,
        "info": sim.info(),
        "residual": b1["residual"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_of(wname, precision, sim.info()["tile"]), "kernel": "k_step",
                     "kernel_us": kern_ms * 1e3, "bytes_per_cell": bpc,
                     "bytes_per_launch": bpc * cells},
    }


def time_ensemble(precision, launches, ksteps, n_scen, tune):
    """Batched ensemble of uneven catchments advanced by the persistent kernel."""
    import torch

    import synth
    from paper_2406_14933_amd import hexsv
    scs = synth.c3_ensemble(n_scen=n_scen)
    ens = hexsv.Ensemble.from_scenarios(scs, precision, steps_per_launch=ksteps)
    del scs
    if tune:
        ens.autotune(ksteps=max(2, ksteps // 10))
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
    return {"value": tm["cell_updates"] / wall, "cells": info["cells"], "scenarios": n_scen,
            "steps_per_scenario": launches * ksteps, "wall_s": wall,
            "gpu_value": tm["cell_updates"] / (tm["gpu_ms"] * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_ensemble", "bytes_per_cell": bpc},
            "info": info}


def surrogate_block(n_train=16, n_test=8, size=512, k=16, tol=3e-5, seed=1, dt_scale=2.4):
    """Train the window surrogate on solver trajectories (all on the GPU, the library's own
    kernels) and time it against the plain FP32 solver on held-out scenarios to t_end."""
    import numpy as np

    import synth
    from paper_2406_14933_amd import hexsv
    from paper_2406_14933_amd import surrogate as S
    t_end = 1800.0
    train_sc = [synth.ensemble_member(s, size=size, config=5, t_end=t_end) for s in range(n_train)]
    test_sc = [synth.ensemble_member(1000 + s, size=size, config=5, t_end=t_end)
               for s in range(n_test)]
    t0 = time.perf_counter()
    dt_fix = dt_scale * min(S.pilot_dt(sc) for sc in train_sc[:2])
    window = k * dt_fix
    sur = hexsv.Surrogate(4, 32)
    rng = np.random.default_rng(seed)
    # He-normal start, last layer scaled down: the network starts near the probe extrapolation
    p = []
    for li, (ci, co) in enumerate([(hexsv.Surrogate.FEATURES, 32), (32, 32), (32, 32), (32, 3)]):
        std = math.sqrt(2.0 / (7 * ci)) * (0.1 if li == 3 else 1.0)
        p.append(rng.normal(scale=std, size=co * ci * 7))
        p.append(np.zeros(co))
    sur.set_params(np.concatenate(p).astype(np.float32))
    times = list(np.linspace(window, t_end - 2 * window, 32))
    data, scales = S.collect(train_sc, times, window, k, sur)
    S.train(sur, data, 3000, batch=4, lr=1e-3, lr_end=5e-5, seed=seed)
    for rnd in range(2):  # pairs from the network's own runs, then more training
        ro = S.rollout_pairs(sur, train_sc, list(np.linspace(2 * window, t_end - 2 * window, 16)),
                             window, k, scales, tol=tol)
        data = S.merge(data, ro)
        S.train(sur, data, 3000, batch=4, lr=5e-4, lr_end=2e-5, seed=seed + 1 + rnd)
    train_s = time.perf_counter() - t0
    ev = S.evaluate(sur, test_sc, window, k, tol, project=True)
    plain_steps = sum(r["plain_steps"] for r in ev["rows"])
    sur_steps = sum(r["surrogate_steps"] for r in ev["rows"])
    return {"workload": f"surrogate-{n_test}-heldout-{size}x{size}-edge1m-to-{t_end:.0f}s",
            "speedup": ev["speedup"], "err_h_max": ev["err_h_max"],
            "err_h_mean": ev["err_h_mean"], "tol": tol, "accept_frac": ev["accept_frac"],
            "solver_steps_avoided": 1.0 - sur_steps / max(plain_steps, 1),
            "refused": {k: ev[k] for k in ("refused_residual", "refused_wave_speed",
                                           "refused_nonfinite")},
            "plain_s": ev["plain_s"], "surrogate_s": ev["surrogate_s"], "window_s": window,
            "k": k, "train_pairs": data.pairs, "train_scenarios": n_train, "train_s": train_s}


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


def cpu_baseline(sc, budget_s=12.0):
    """The FP64 oracle as it stands, on the host cores, over a bounded number of steps."""
    import numpy as np

    import oracle
    G = oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)
    p = oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s)
    r = oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
    threads = min(os.cpu_count() or 1, 16)
    # one probe step to size the sample
    t0 = time.perf_counter()
    h, v1, v2, b, _ = oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, sc.h0, sc.v10, sc.v20,
                                 1e30, max_steps=2, nthreads=threads)
    per = (time.perf_counter() - t0) / 2
    k = int(max(2, min(2000, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.run(G, sc.z, sc.theta, sc.alpha_p, p, r, h, v1, v2, 1e30, max_steps=k, books=b,
               nthreads=threads)
    dt = time.perf_counter() - t0
    cells = int(np.count_nonzero(G.active))
    return {"value": cells * k / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} FP64 steps of the full {sc.nq}x{sc.nr} raster from the dry start, "
                      f"{dt:.1f} s on {threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--steps-per-graph", type=int, default=100)
    ap.add_argument("--large-steps", type=int, default=400,
                    help="steps of the 4096x4096 catchment timed beside the main workload (0: skip)")
    ap.add_argument("--ensemble-launches", type=int, default=4,
                    help="timed launches of the 256-scenario batched ensemble (0: skip)")
    ap.add_argument("--ensemble-ksteps", type=int, default=25)
    ap.add_argument("--ensemble-scenarios", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip training and timing the window surrogate")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--window-cost", action="store_true",
                    help="only time surrogate windows against plain steps on still water")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for counter calibration)")
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
    main_run = time_gpu(sc, wname, args.precision, args.steps, args.warmup, args.tile,
                        args.steps_per_graph)
    print(f"[bench] {args.precision}: {main_run['value']:.3e} cell-updates/s, step kernel "
          f"{main_run['kernel_us']:.1f} us", file=sys.stderr, flush=True)
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
                   "precision": args.precision, "tile": main_run["info"],
                   "steps_per_graph": args.steps_per_graph},
        "roofline": main_run["roofline"],
        "gpu_us_per_step": main_run["gpu_us_per_step"],
        "books_residual": main_run["residual"],
    }
    if not args.no_fp64 and args.precision == "fp32":
        other = time_gpu(sc, wname, "fp64", args.steps, args.warmup, args.tile, args.steps_per_graph)
        print(f"[bench] fp64: {other['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
        line["fp64"] = {"value": other["value"], "ms_per_step": other["ms_per_step"],
                        "roofline": other["roofline"], "books_residual": other["residual"]}
    if args.large_steps > 0 and args.workload != "c4":
        big, bname = workload("c4")
        print(f"[bench] large: {bname}", file=sys.stderr, flush=True)
        lr = time_gpu(big, bname, args.precision, args.large_steps, 50, args.tile, args.steps_per_graph)
        print(f"[bench] large {args.precision}: {lr['value']:.3e} cell-updates/s, step kernel "
              f"{lr['kernel_us']:.1f} us", file=sys.stderr, flush=True)
        line["large"] = {"workload": bname, "value": lr["value"], "steps": args.large_steps,
                         "ms_per_step": lr["ms_per_step"], "roofline": lr["roofline"],
                         "books_residual": lr["residual"]}
        del big
    if args.ensemble_launches > 0:
        print("[bench] batched ensemble", file=sys.stderr, flush=True)
        er = time_ensemble(args.precision, args.ensemble_launches, args.ensemble_ksteps,
                           args.ensemble_scenarios, tune=True)
        print(f"[bench] batched {args.precision}: {er['value']:.3e} cell-updates/s",
              file=sys.stderr, flush=True)
        line["batched"] = {"workload": f"ensemble-{er['scenarios']}-catchments-128..512sq",
                           "value": er["value"], "cells": er["cells"],
                           "steps_per_scenario": er["steps_per_scenario"],
                           "roofline": er["roofline"], "config": er["info"]}
    if args.surrogate:
        print("[bench] surrogate: training on solver trajectories", file=sys.stderr, flush=True)
        sr = surrogate_block()
        sr["window_cost"] = window_cost()
        print(f"[bench] surrogate: speed-up {sr['speedup']:.2f}x at rel L1 error "
              f"{sr['err_h_max']:.2e} (max over held-out)", file=sys.stderr, flush=True)
        line["surrogate"] = sr
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
