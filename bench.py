#!/usr/bin/env python3
"""Benchmark of the inverted-opal Yee stepper on one MI355X.

Headline workload: the disordered slab for femtosecond-pulse transmission —
4x4x8 cubic fcc cells of an inverted opal at 20 cells/a (80x80x160) with 1 a
vacuum margins and a 12-cell CPML on z (80x80x224 = 1,433,600 cells), Gaussian
jitter delta = 0.05 a, 30 fs plane-wave pulse at 0.8 c/a, probe, transmitted power
T(t) and running-DFT spectra (100 frequencies, every 8 steps) on two planes,
energy every 100 steps.  One "step" is one full FDTD step of that slab.

Prints one JSON line: cell-updates/s of the plain stepper (inputs resident in
HBM), the roofline of the dominant kernel measured live with hipEvents, the CPU
oracle timed on a bounded sample of the same workload, and the batched
(64 uneven realizations in one graph-captured launch sequence) and lasing
(four-level gain box) figures beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
B_ALG_LINEAR = 49.0          # bytes per linear cell-update: E,H (24) + material (1) in, E,H (24) out
B_PSI_PER_AXIS = 32.0        # CPML: 2 E-side psi (r+w) + 2 H-side psi (r + w) per slab axis
METRIC = "cell-updates/s & HBM-roofline %, batched vs plain; served p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def headline_config(steps):
    from paper_0802_3775_amd import workloads as W
    return W.slab(delta=0.05, seed=13, res=20, cells=(4, 4, 8), steps=steps, nf=100, decim=8,
                  energy_interval=100)


def measure_plain(args):
    import torch
    from paper_0802_3775_amd import fdtd
    total = args.warmup + args.steps + args.kernel_steps
    cfg = headline_config(total)
    tuning = {"block": 256, "zchunk": 32, "graph_steps": 100, "max_blocks": 0}
    plan = fdtd.Plan(cfg, max_steps=total, tuning=tuning)
    ncell = plan.ncell
    log("plain: grid %s, %d cells, warmup %d" % (cfg["grid"]["n"], ncell, args.warmup))
    plan.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    log("plain: %d steps in %.3f s" % (args.steps, wall))
    # per-kernel durations with hipEvents around each launch, on the launch stream
    ms, cnt = plan.time_kernels(args.kernel_steps)
    cells = plan.class_cells()
    names = ["step_plain", "step_cpml", "step_gain", "step_cpml_gain", "dft"]
    kern = {}
    for c in range(5):
        if cnt[c] == 0:
            continue
        avg = ms[c] / cnt[c]
        if c < 4:
            nbytes = cells[c] * (B_ALG_LINEAR + (B_PSI_PER_AXIS if c in (1, 3) else 0.0))
        else:
            nbytes = cells[4] * 4 * 100 * 16 * 2
        kern[names[c]] = {"avg_ms": avg, "launches": int(cnt[c]), "cells": int(cells[c]),
                          "alg_bytes": float(nbytes), "GBps": nbytes / (avg * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    plan.close()
    return {"ncell": ncell, "wall": wall, "kernels": kern, "dominant": dom, "cfg": cfg}


def measure_cpu(cfg, budget_s):
    from oracle import oracle as O
    sim = O.OracleSim(dict(cfg, steps=100000), max_steps=100000)
    t0 = time.perf_counter()
    sim.step(2)
    t1 = time.perf_counter()
    per = (t1 - t0) / 2
    n = max(2, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    sim.step(n)
    t1 = time.perf_counter()
    ncell = cfg["grid"]["n"][0] * cfg["grid"]["n"][1] * cfg["grid"]["n"][2]
    return {"value": ncell * n / (t1 - t0), "unit": "cell-updates/s", "cores": O.threads(),
            "kind": "oracle", "sample": "%d steps of the headline slab (full %dx%dx%d grid, FP64, "
            "steps 2..%d of the run), %.1f s" % ((n,) + tuple(cfg["grid"]["n"]) + (n + 2, t1 - t0))}


def measure_batched(steps):
    import torch
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd import workloads as W
    cfgs = W.ensemble(count=64, steps=10000)
    tuning = {"block": 256, "zchunk": 32, "graph_steps": 50, "max_blocks": 0}
    total = 2 * steps + 100
    plans = [fdtd.Plan(c, max_steps=total, tuning=tuning) for c in cfgs]
    cells = sum(p.ncell for p in plans)
    log("batched: %d realizations, %d cells" % (len(plans), cells))
    # sequential plain: each realization alone
    seq = 0.0
    for p in plans:
        p.step(50)
    torch.cuda.synchronize()
    for p in plans:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.step(steps)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
    b = fdtd.Batch(plans)
    b.step(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    b.close()
    for p in plans:
        p.close()
    full = 10000.0 / steps
    return {"realizations": len(cfgs), "cells": cells, "steps_timed": steps,
            "cell_updates_per_s": cells * steps / tb,
            "sequential_cell_updates_per_s": cells * steps / seq,
            "realizations_per_hour": 3600.0 * len(cfgs) / (tb * full),
            "sequential_realizations_per_hour": 3600.0 * len(cfgs) / (seq * full),
            "note": "10k-step runs extrapolated from %d timed steps" % steps}


def measure_lasing(steps):
    import torch
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd import workloads as W
    cfg = W.lasing(pump=1e10, steps=steps + 100)
    plan = fdtd.Plan(cfg, max_steps=steps + 100,
                     tuning={"block": 256, "zchunk": 24, "graph_steps": 100, "max_blocks": 0})
    plan.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    n = plan.ncell
    plan.close()
    return {"workload": "lasing box 6x6x6 cells at 24 cells/a + 12-cell CPML (168^3), gain voids, "
            "pump 1e10 s^-1", "cells": n, "steps_timed": steps, "cell_updates_per_s": n * steps / t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); the multi-GPU "
              "decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    plain = measure_plain(args)
    value = plain["ncell"] * args.steps / plain["wall"]
    dom = plain["kernels"][plain["dominant"]]
    achieved = dom["GBps"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * plain["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disordered inverted-opal slab, 4x4x8 cubic cells at 20 cells/a "
                               "(80x80x224 with 1a margins and 12-cell z-CPML), delta=0.05a, 30 fs "
                               "plane-wave pulse, probe + T(t) + 100-frequency DFT flux on 2 planes, "
                               "energy every 100 steps",
                   "cells": plain["ncell"], "run_steps": 20000},
        "roofline": {"bound": "hbm", "kernel": plain["dominant"], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": dom["alg_bytes"],
                     "avg_launch_ms": dom["avg_ms"]},
        "kernels": plain["kernels"],
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = measure_cpu(plain["cfg"], args.cpu_seconds)
    if not args.no_extras:
        log("batched ...")
        out["batched"] = measure_batched(300)
        log("lasing ...")
        out["lasing"] = measure_lasing(1000)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
