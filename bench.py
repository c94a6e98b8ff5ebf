#!/usr/bin/env python3
"""Benchmark of the inverted-opal Yee stepper on one MI355X.

Headline workload: the disordered slab for femtosecond-pulse transmission —
4x4x8 cubic fcc cells of an inverted opal at 20 cells/a (80x80x160) with 1 a
vacuum margins and a 12-cell CPML on z (80x80x224 = 1,433,600 cells), Gaussian
jitter delta = 0.05 a, 30 fs plane-wave pulse at 0.8 c/a, probe, transmitted power
T(t) and running-DFT spectra (100 frequencies, every 8 steps) on two planes,
energy every 100 steps.  One "step" is one full FDTD step of that slab; the
default run is the workload's 20,000 steps.

Prints one JSON line: cell-updates/s of the plain stepper (inputs resident in
HBM, autotuned launch shape, hipGraph replay), the roofline of the dominant
kernel measured live with hipEvents bound to its launches (against the vendor
HBM peak, and against the rate of a 1 GiB device copy measured in the same run),
the CPU oracle timed on a bounded sample of the same workload, and beside them
the batched ensemble (64 uneven realizations, one launch per tile class per
step), the served request stream (p50/p99 latency), the lasing boxes (Lorentz and
density-matrix media), the paper's 200^3 beam and lasing boxes and the 320^3
grid.

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
METRIC = "cell-updates/s & HBM-roofline %, batched vs plain; served p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    "slab": "disordered inverted-opal slab, 4x4x8 cubic cells at 20 cells/a (80x80x224 with 1a margins and "
            "12-cell z-CPML), delta=0.05a, 30 fs plane-wave pulse, probe + T(t) + 100-frequency DFT flux on 2 "
            "planes, energy every 100 steps",
    "big": "linear slab 10x10x10 cubic cells at 32 cells/a (320x320x408, z-CPML)",
    "paper_beam": "paper's linear box 200^3 at 16 cells/a (8^3 cells of inverted opal, gamma 0.05, CPML on all "
                  "faces, TEM00 beam)",
    "paper_lasing": "paper's lasing box 200^3 at 16 cells/a (8^3 cells of eps-12 inverted opal, gamma 0.1, "
                    "density-matrix dye in the spheres, CPML on all faces, noise-seeded)",
}


def headline_config(steps, workload="slab"):
    from paper_0802_3775_amd import workloads as W
    if workload == "big":
        return W.slab(delta=0.05, seed=4242, res=32, cells=(10, 10, 10), steps=steps, nf=0)
    if workload == "paper_beam":
        return W.paper_beam(0.05, seed=31, steps=steps)
    if workload == "paper_lasing":
        return W.paper_lasing(0.1, steps=steps)
    return W.slab(delta=0.05, seed=13, res=20, cells=(4, 4, 8), steps=steps, nf=100, decim=8,
                  energy_interval=100)


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "fd_internal.h"):
        with open(os.path.join(ROOT, "paper_0802_3775_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter runs (FETCH_SIZE,
    WRITE_SIZE, each scaled by the same counter's reading for a copy of known
    size), or None if the kernel source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get("%s/%s" % (workload, kernel))
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec["hbm_bytes_per_launch"]


def copy_calibration():
    """A device copy of exactly 1 GiB (read 1 GiB, write 1 GiB) for scaling the
    HBM byte counters in profiled runs."""
    import torch
    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


def copy_bandwidth(reps=10):
    """Bytes moved per second (read + write) by the runtime's own device copy of
    1 GiB, best of reps: the HBM rate a pure streaming kernel reaches on this
    GPU, measured beside the vendor peak."""
    import torch
    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    nbytes = 2.0 * x.numel() * 4
    del x, y
    torch.cuda.empty_cache()
    return nbytes / (best * 1e-3) / 1e9


def kernel_table(plan, nsteps):
    """Per kernel class: average launch duration (a hipEvent pair bound to each
    launch on the launch stream: the kernel's own begin and end timestamps) and
    the algorithmic bytes of one launch (libfdtd counts them per cell: 49 B, +32 B
    per CPML slab axis, +84 B per Lorentz or +144 B per density-matrix gain cell,
    +4 B per cell of a gain tile for its gain ordinal; a DFT launch stores a
    40 B/point plane sample and, once per 32-sample ring, moves 128 B per plane
    point and frequency: averaged per launch)."""
    from paper_0802_3775_amd import fdtd
    ms, cnt = plan.time_kernels(nsteps)
    cells = plan.class_cells()
    nbytes = plan.class_bytes()
    kern = {}
    for c, name in enumerate(fdtd.Plan.CLASSES):
        if cnt[c] == 0:
            continue
        avg = ms[c] / cnt[c]
        kern[name] = {"avg_ms": avg, "launches": int(cnt[c]), "cells": int(cells[c]),
                      "alg_bytes": float(nbytes[c]), "GBps": nbytes[c] / (avg * 1e-3) / 1e9}
    return kern


def timed_run(plan, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def measure_plain(args):
    from paper_0802_3775_amd import fdtd, tune
    total = args.warmup + args.steps + args.kernel_steps
    cfg = headline_config(total, args.workload)
    t0 = time.perf_counter()
    if args.tuning:
        v = [int(q) for q in args.tuning.split(",")] + [1, 0]
        tuning = {"tile_x": v[0], "block": v[1], "zchunk": v[2], "graph_steps": v[3], "max_blocks": 0,
                  "merge": v[4], "parallel": v[5]}
    else:
        tuning = tune.autotune(dict(cfg), budget_s=args.tune_seconds)
    log("plain: tuning %s (%.1f s)" % (tuning, time.perf_counter() - t0))
    plan = fdtd.Plan(cfg, max_steps=total, tuning=tuning)
    log("plain: grid %s, %d cells, warmup %d" % (cfg["grid"]["n"], plan.ncell, args.warmup))
    plan.step(args.warmup)
    wall = timed_run(plan, args.steps)
    log("plain: %d steps in %.3f s" % (args.steps, wall))
    kern = kernel_table(plan, args.kernel_steps)
    ncell = plan.ncell
    plan.close()
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    return {"ncell": ncell, "wall": wall, "kernels": kern, "dominant": dom, "cfg": cfg, "tuning": tuning}


def measure_big(args):
    """The largest serving grid (10^3 cubic cells at 32 cells/a, 320x320x408): the
    state (2 GB) is far larger than the 256 MB Infinity Cache."""
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    steps = 200
    cfg = W.slab(delta=0.05, seed=4242, res=32, cells=(10, 10, 10), steps=steps + 150, nf=0)
    tuning = tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True)
    plan = fdtd.Plan(cfg, max_steps=steps + 150, tuning=tuning)
    plan.step(20)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, 100)
    n = plan.ncell
    plan.close()
    kname = max(kern, key=lambda q: kern[q]["avg_ms"] * kern[q]["launches"])
    k = kern[kname]
    return {"workload": "linear slab 10x10x10 cubic cells at 32 cells/a (320x320x408, z-CPML)",
            "cells": n, "steps_timed": steps, "cell_updates_per_s": n * steps / wall, "tuning": tuning,
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": k["GBps"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": k["GBps"] / HBM_PEAK_GBS, "avg_launch_ms": k["avg_ms"],
                         "alg_bytes_per_launch": k["alg_bytes"],
                         "traffic": recorded_traffic("big", kname)},
            "kernels": kern}


def measure_beam(args, steps=400):
    """The paper's linear workload: 200^3 box (6 um at 16 cells/a) with 8^3 cells of
    inverted opal (eps 12, r0 = a/(2 sqrt 2), uniform-radius disorder gamma = 0.05),
    CPML on all faces, single-cycle TEM00 beam (waist 2 um, 484 THz)."""
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    cfg = W.paper_beam(gamma=0.05, seed=31, steps=steps + 200)
    tuning = tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True)
    plan = fdtd.Plan(cfg, max_steps=steps + 200, tuning=tuning)
    plan.step(50)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, 100)
    n = plan.ncell
    plan.close()
    kname = max(kern, key=lambda q: kern[q]["avg_ms"] * kern[q]["launches"])
    k = kern[kname]
    return {"workload": "paper's linear box 200^3 at 16 cells/a (8^3 cells of inverted opal, gamma 0.05, "
                        "CPML on all faces, TEM00 beam)",
            "cells": n, "steps_timed": steps, "cell_updates_per_s": n * steps / wall, "tuning": tuning,
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": k["GBps"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": k["GBps"] / HBM_PEAK_GBS, "avg_launch_ms": k["avg_ms"],
                         "alg_bytes_per_launch": k["alg_bytes"], "traffic": recorded_traffic("paper_beam", kname)},
            "kernels": kern}


def measure_cpu(cfg, budget_s):
    """The FP64 oracle on the host cores, stepped in chunks until about budget_s
    seconds of stepping have been timed (the first steps are left out)."""
    from oracle import oracle as O
    sim = O.OracleSim(dict(cfg, steps=1000000), max_steps=1000000)
    sim.step(2)
    n, dt = 0, 0.0
    chunk = 4
    while dt < budget_s:
        t0 = time.perf_counter()
        sim.step(chunk)
        dt += time.perf_counter() - t0
        n += chunk
        chunk = min(64, chunk * 2)
    ncell = cfg["grid"]["n"][0] * cfg["grid"]["n"][1] * cfg["grid"]["n"][2]
    return {"value": ncell * n / dt, "unit": "cell-updates/s", "cores": O.threads(), "kind": "oracle",
            "sample": "steps 3..%d of the headline slab run (full %dx%dx%d grid, FP64 oracle), %.1f s"
                      % ((n + 2,) + tuple(cfg["grid"]["n"]) + (dt,))}


def measure_batched(args, steps=300):
    import torch
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    cfgs = W.ensemble(count=64, steps=10000)
    tuning = tune.tune_batch(cfgs, budget_s=args.tune_seconds)
    seq_tuning = tune.common_tuning(cfgs, budget_s=args.tune_seconds)  # tuned for plain runs
    total = 2 * steps + 100
    cells = 0
    seq = 0.0
    for c in cfgs:           # sequential plain: each realization alone
        p = fdtd.Plan(c, max_steps=steps + 50, tuning=seq_tuning)
        cells += p.ncell
        p.step(50)
        seq += timed_run(p, steps)
        p.close()
    plans = [fdtd.Plan(c, max_steps=total, tuning=tuning) for c in cfgs]
    log("batched: %d realizations, %d cells, tuning %s (sequential runs: %s)" % (len(plans), cells, tuning, seq_tuning))
    for p in plans:
        p.step(50)
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
    scale = 10000.0 / steps
    return {"realizations": len(cfgs), "cells": cells, "steps_timed": steps, "tuning": tuning,
            "sequential_tuning": seq_tuning,
            "cell_updates_per_s": cells * steps / tb,
            "sequential_cell_updates_per_s": cells * steps / seq,
            "realizations_per_hour": 3600.0 * len(cfgs) / (tb * scale),
            "sequential_realizations_per_hour": 3600.0 * len(cfgs) / (seq * scale),
            "note": "10k-step runs extrapolated from %d timed steps per realization" % steps}


def measure_lasing(args, steps=1000, model="lorentz"):
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    cfg = W.lasing(pump=1e10, steps=steps + 300, model=model)
    tuning = tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True)
    plan = fdtd.Plan(cfg, max_steps=steps + 300, tuning=tuning)
    plan.step(100)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, 50)
    n = plan.ncell
    plan.close()
    medium = ("Lorentz + four-level rate equations" if model == "lorentz" else
              "density-matrix dye (ground + 3 upper levels, T1 1 ns, T2 10 fs, N 5e25 m^-3, inverted start)")
    return {"workload": "lasing box 6x6x6 cells at 24 cells/a + 12-cell CPML on all faces (168^3), "
            "gain voids: %s, pump 1e10 s^-1, noise" % medium, "cells": n, "steps_timed": steps,
            "cell_updates_per_s": n * steps / wall, "tuning": tuning, "kernels": kern}


def measure_paper_lasing(args, steps=300):
    """The paper's lasing run: the 200^3 box with the density-matrix dye in the
    spheres (gamma 0.1), noise-seeded, autotuned."""
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    cfg = W.paper_lasing(0.1, steps=steps + 300)
    tuning = tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True)
    plan = fdtd.Plan(cfg, max_steps=steps + 300, tuning=tuning)
    plan.step(100)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, 50)
    n = plan.ncell
    plan.close()
    kname = max(kern, key=lambda q: kern[q]["avg_ms"] * kern[q]["launches"])
    k = kern[kname]
    return {"workload": WORKLOADS["paper_lasing"], "cells": n,
            "steps_timed": steps, "cell_updates_per_s": n * steps / wall, "tuning": tuning,
            "roofline": {"bound": "hbm", "kernel": kname, "achieved": k["GBps"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": k["GBps"] / HBM_PEAK_GBS, "avg_launch_ms": k["avg_ms"],
                         "alg_bytes_per_launch": k["alg_bytes"], "traffic": recorded_traffic("paper_lasing", kname)},
            "kernels": kern}


def measure_serving(args, plain_rate):
    """A reduced Poisson trace of mixed requests (70% linear slabs, 30% lasing
    boxes, 27k-512k-cell crystals, 2000 steps each), offered at 0.9 of the
    sequential capacity estimated from the plain stepper's rate."""
    import torch
    from paper_0802_3775_amd import serve
    from paper_0802_3775_amd import workloads as W
    base = W.serving_trace(count=args.serve_requests, seed=42, rho=1.0, capacity_per_s=1.0,
                           n_range=(2, 4), res_range=(12, 20), cell_range=(30 ** 3, 80 ** 3),
                           linear_steps=2000, lasing_steps=2000)
    work = 0.0
    for r in base:
        c = serve.request_config(r)
        work += c["grid"]["n"][0] * c["grid"]["n"][1] * c["grid"]["n"][2] * r["steps"]
    cap = plain_rate / (work / len(base))          # requests per second, sequential estimate
    lam = 0.9 * cap
    reqs = [dict(r, arrival=r["arrival"] / lam) for r in base]
    tuning = {"block": 256, "tile_x": 16, "zchunk": 2, "graph_steps": 100, "max_blocks": 0, "merge": 1,
              "parallel": 0}
    backend = serve.GpuBackend(tuning)
    free, _ = torch.cuda.mem_get_info()
    srv = serve.Server(backend, budget_bytes=int(0.5 * free), chunk=400)
    wall = srv.run(reqs)
    s_b = serve.summarize(reqs, wall, srv.results, srv.failed)
    srv2, wall2 = serve.run_sequential(backend, reqs)
    s_s = serve.summarize(reqs, wall2, srv2.results, srv2.failed)
    return {"requests": len(reqs), "offered_rate_per_s": lam, "chunk_steps": 400,
            "served": s_b, "sequential_fifo": s_s,
            "note": "reduced trace (27k-512k-cell crystals plus margins and CPML, 2000 steps per "
                    "request) so the run stays within the benchmark's time budget"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tune-seconds", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--workload", choices=tuple(WORKLOADS), default="slab",
                    help="headline slab (default); the others (320^3 grid, the paper's beam and lasing boxes) for profiling")
    ap.add_argument("--tuning", default="", help="fixed tile_x,block,zchunk,graph_steps[,merge,parallel] (skip the autotuner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration in profiled runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the stepper runs on one GPU (--gpus 1); its multi-GPU z-slab "
              "decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if args.copy_calibration:
        copy_calibration()
    plain = measure_plain(args)
    value = plain["ncell"] * args.steps / plain["wall"]
    dom = plain["kernels"][plain["dominant"]]
    copy_gbs = copy_bandwidth()
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
        "config": {"workload": WORKLOADS[args.workload],
                   "cells": plain["ncell"], "run_steps": 20000, "tuning": plain["tuning"]},
        "roofline": {"bound": "hbm", "kernel": plain["dominant"], "achieved": dom["GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["GBps"] / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(args.workload, plain["dominant"]),
                     "alg_bytes_per_launch": dom["alg_bytes"],
                     "avg_launch_ms": dom["avg_ms"],
                     "copy_GBps": copy_gbs, "frac_of_copy": dom["GBps"] / copy_gbs},
        "kernels": plain["kernels"],
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = measure_cpu(plain["cfg"], args.cpu_seconds)
    if not args.no_extras:
        log("320^3 ...")
        out["big_320"] = measure_big(args)
        log("paper beam box ...")
        out["paper_beam_200"] = measure_beam(args)
        log("lasing ...")
        out["lasing"] = measure_lasing(args)
        log("lasing, density matrix ...")
        out["lasing_density"] = measure_lasing(args, model="density")
        log("paper lasing box ...")
        out["paper_lasing_200"] = measure_paper_lasing(args)
        log("batched ...")
        out["batched"] = measure_batched(args)
        log("serving ...")
        out["serving"] = measure_serving(args, value)
    for key in ("big_320", "paper_beam_200", "paper_lasing_200"):
        rl = out.get(key, {}).get("roofline")
        if rl:
            rl["copy_GBps"] = copy_gbs
            rl["frac_of_copy"] = rl["achieved"] / copy_gbs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
