#!/usr/bin/env python3
"""Benchmark of the inverted-opal Yee stepper on one MI355X.

Headline workload: the largest single-GPU request of the serving stream -- a
disordered inverted-opal slab of 10x10x10 cubic fcc cells at 32 cells/a
(320x320x320 crystal) with 1 a vacuum margins and a 12-cell CPML on z
(320x320x408 = 41,779,200 cells, 2.1 GB of step state, far beyond the 256 MB
Infinity Cache), Gaussian jitter delta = 0.05 a, 30 fs plane-wave pulse at
0.8 c/a, probe, transmitted power T(t) and 100-frequency running-DFT spectra
every 8 steps on two planes, energy every 100 steps.  One "step" is one full
FDTD step of that grid.

Prints one JSON line: cell-updates/s of the plain stepper (inputs resident in
HBM, autotuned launch shape, hipGraph replay), the roofline of the dominant
kernel measured live with hipEvents bound to its launches (against the vendor
HBM peak, and against the rate of a 1 GiB device copy measured in the same run),
the CPU oracle timed on a bounded sample of the same workload, and beside them
the batched ensemble (64 uneven realizations, one launch per tile class per
step; its own roofline), the served request stream at the stream's request
sizes and lengths (p50/p99 latency at two offered loads), the slab of the
femtosecond-pulse transmission runs (80x80x224, cache-resident), the lasing
boxes (Lorentz and density-matrix media) and the paper's 200^3 beam and lasing
boxes.

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
    "big320": "largest serving request: disordered inverted-opal slab, 10x10x10 cubic cells at 32 cells/a "
              "(320x320x408 with 1a margins and 12-cell z-CPML, 41.8M cells, 2.1 GB of step state), delta=0.05a, "
              "30 fs plane-wave pulse, probe + T(t) + 100-frequency DFT flux on 2 planes, energy every 100 steps",
    "slab": "disordered inverted-opal slab, 4x4x8 cubic cells at 20 cells/a (80x80x224 with 1a margins and "
            "12-cell z-CPML), delta=0.05a, 30 fs plane-wave pulse, probe + T(t) + 100-frequency DFT flux on 2 "
            "planes, energy every 100 steps (state fits the 256 MB Infinity Cache)",
    "paper_beam": "paper's linear box 200^3 at 16 cells/a (8^3 cells of inverted opal, gamma 0.05, CPML on all "
                  "faces, TEM00 beam)",
    "paper_lasing": "paper's lasing box 200^3 at 16 cells/a (8^3 cells of eps-12 inverted opal, gamma 0.1, "
                    "density-matrix dye in the spheres, CPML on all faces, noise-seeded)",
    "lasing168": "lasing box 6x6x6 cells at 24 cells/a + 12-cell CPML on all faces (168^3), gain voids: Lorentz + "
                 "four-level rate equations at 1e24 m^-3, pump 1e10 s^-1, noise",
    "lasing_density": "lasing box 6x6x6 cells at 24 cells/a + 12-cell CPML on all faces (168^3), gain voids: "
                      "density-matrix dye (ground + 3 upper levels, T1 1 ns, T2 10 fs, N 5e25 m^-3, inverted start), "
                      "pump 1e10 s^-1, noise",
}


def headline_config(steps, workload="big320"):
    from paper_0802_3775_amd import workloads as W
    if workload == "big320":
        return W.slab(delta=0.05, seed=4242, res=32, cells=(10, 10, 10), steps=steps, nf=100, decim=8,
                      energy_interval=100)
    if workload == "paper_beam":
        return W.paper_beam(0.05, seed=31, steps=steps)
    if workload == "paper_lasing":
        return W.paper_lasing(0.1, steps=steps)
    if workload == "lasing168":
        return W.lasing(pump=1e10, steps=steps)
    if workload == "lasing_density":
        return W.lasing(pump=1e10, steps=steps, model="density")
    return W.slab(delta=0.05, seed=13, res=20, cells=(4, 4, 8), steps=steps, nf=100, decim=8,
                  energy_interval=100)


def cpu_sample_config(workload, steps):
    """The bounded sample of a workload the CPU oracle is timed on: for the
    320x320x408 grid its 320x320 cross-section with one cubic cell of crystal
    along z (same margins, CPML, pulse, probe and flux planes: 320x320x120), so
    the oracle's set-up (voxelizing 42M cells) stays out of the budget; other
    workloads whole."""
    from paper_0802_3775_amd import workloads as W
    if workload == "big320":
        return W.slab(delta=0.05, seed=4242, res=32, cells=(10, 10, 1), steps=steps, nf=100, decim=8,
                      energy_interval=100)
    return headline_config(steps, workload)


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "fd_internal.h"):
        with open(os.path.join(ROOT, "paper_0802_3775_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def launch_shape(tuning, cfg=None):
    """The launch parameters a kernel's memory traffic depends on (tile, z-chunk,
    class grouping, member-group size).  Without x / y CPML and gain, grouping 2
    (every tile in the most general kernel) launches what grouping 1 does."""
    t = tuning or {}
    out = {k: int(t.get(k, 0)) for k in ("tile_x", "block", "zchunk", "merge", "cache_mb")}
    if cfg is not None:
        g = cfg["grid"]
        xy = any(int(v) > 0 for v in tuple(g.get("pml_lo", (0, 0, 0)))[:2] + tuple(g.get("pml_hi", (0, 0, 0)))[:2])
        gain = any(int(m.get("gain") or 0) for m in cfg["materials"])
        if not xy and not gain:
            out["merge"] = min(out["merge"], 1)
    return out


# Launch shapes of the side measurements: the fastest of the full tuning sweeps
# (every tile, z-chunk and class grouping) on these workloads, fixed so that the
# committed counter profiles, taken in the same shapes, apply (--tune-side runs
# the quick autotuner instead).
SIDE_TUNING = {
    "slab": (32, 256, 8, 50, 1, 0),
    "paper_beam": (32, 256, 8, 200, 2, 0),
    "lasing168": (64, 256, 8, 200, 2, 0),
    "lasing_density": (32, 256, 8, 200, 2, 0),
    "paper_lasing": (32, 256, 8, 200, 2, 0),
}
BATCH_TUNING = (64, 256, 16, 50, 2, 0, 224)
# the realizations stepped one after another, each alone: the fastest shape of a
# sweep of those runs (tiles 16/32/64, 128/256 threads, z-chunks 4-16, groupings)
SEQ_TUNING = (32, 256, 8, 50, 1, 0)


def fixed_tuning(v):
    """Tuning dict from (tile_x, block, zchunk, graph_steps[, merge, parallel[, cache_mb]])."""
    v = list(v)
    if len(v) < 6:
        v += [1, 0][len(v) - 4:]  # merge 1, parallel 0
    t = {"tile_x": v[0], "block": v[1], "zchunk": v[2], "graph_steps": v[3], "max_blocks": 0,
         "merge": v[4], "parallel": v[5]}
    if len(v) > 6:
        t["cache_mb"] = v[6]
    return t


def recorded_traffic(workload, kernel, tuning, cfg):
    """HBM bytes per launch from the committed rocprofv3 counter runs (FETCH_SIZE,
    WRITE_SIZE, each scaled by the same counter's reading for a copy of known
    size), or None if the kernel source changed since they were taken or they
    were taken in another launch shape than this run's."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get("%s/%s" % (workload, kernel))
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    if launch_shape(rec.get("launch"), cfg) != launch_shape(tuning, cfg):
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


def _roofline(kern, kname, workload, tuning, cfg, copy_gbs=None):
    k = kern[kname]
    out = {"bound": "hbm", "kernel": kname, "achieved": k["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": k["GBps"] / HBM_PEAK_GBS, "avg_launch_ms": k["avg_ms"], "alg_bytes_per_launch": k["alg_bytes"],
           "traffic": recorded_traffic(workload, kname, tuning, cfg)}
    if out["traffic"]:
        # the counted HBM bytes of a launch over the same live duration: the
        # rocprofv3-counted rate beside the algorithmic one
        out["hbm_GBps"] = out["traffic"] / (k["avg_ms"] * 1e-3) / 1e9
        out["hbm_frac"] = out["hbm_GBps"] / HBM_PEAK_GBS
    if copy_gbs:
        out["copy_GBps"] = copy_gbs
        out["frac_of_copy"] = k["GBps"] / copy_gbs
    return out


def _dominant(kern):
    return max(kern, key=lambda q: kern[q]["avg_ms"] * kern[q]["launches"])


def measure_plain(args):
    from paper_0802_3775_amd import fdtd, tune
    total = args.warmup + args.steps + args.kernel_steps
    cfg = headline_config(total, args.workload)
    t0 = time.perf_counter()
    if args.tuning:
        tuning = fixed_tuning([int(q) for q in args.tuning.split(",")])
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
    return {"ncell": ncell, "wall": wall, "kernels": kern, "dominant": _dominant(kern), "cfg": cfg, "tuning": tuning}


def measure_side(args, workload, steps, warm, kernel_steps, copy_gbs):
    """A side workload in its fixed launch shape (SIDE_TUNING; quick autotuning
    with --tune-side), warmed up, steps timed, then the kernel table with the
    dominant kernel's roofline."""
    from paper_0802_3775_amd import fdtd, tune
    total = warm + steps + kernel_steps
    cfg = headline_config(total, workload)
    tuning = (tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True) if args.tune_side
              else fixed_tuning(SIDE_TUNING[workload]))
    plan = fdtd.Plan(cfg, max_steps=total, tuning=tuning)
    plan.step(warm)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, kernel_steps)
    n = plan.ncell
    plan.close()
    return {"workload": WORKLOADS[workload], "cells": n, "steps_timed": steps, "cell_updates_per_s": n * steps / wall,
            "ms_per_step": 1e3 * wall / steps, "tuning": tuning,
            "roofline": _roofline(kern, _dominant(kern), workload, tuning, cfg, copy_gbs), "kernels": kern}


def measure_lasing_density(args, steps=1000):
    from paper_0802_3775_amd import fdtd, tune
    cfg = headline_config(steps + 300, "lasing_density")
    tuning = (tune.autotune(dict(cfg), budget_s=args.tune_seconds, quick=True) if args.tune_side
              else fixed_tuning(SIDE_TUNING["lasing_density"]))
    plan = fdtd.Plan(cfg, max_steps=steps + 300, tuning=tuning)
    plan.step(100)
    wall = timed_run(plan, steps)
    kern = kernel_table(plan, 50)
    n = plan.ncell
    plan.close()
    return {"workload": WORKLOADS["lasing_density"], "cells": n, "steps_timed": steps,
            "cell_updates_per_s": n * steps / wall, "ms_per_step": 1e3 * wall / steps, "tuning": tuning,
            "roofline": _roofline(kern, _dominant(kern), "lasing_density", tuning, cfg), "kernels": kern}


def measure_cpu(workload, budget_s):
    """The FP64 oracle on the host cores, on the workload's bounded sample
    (cpu_sample_config), stepped in chunks until about budget_s seconds of
    stepping have been timed (the first steps are left out)."""
    from oracle import oracle as O
    cfg = cpu_sample_config(workload, 1000000)
    sim = O.OracleSim(cfg, max_steps=1000000)
    sim.step(2)
    n, dt = 0, 0.0
    chunk = 1
    while dt < budget_s:
        t0 = time.perf_counter()
        sim.step(chunk)
        dt += time.perf_counter() - t0
        n += chunk
        chunk = min(64, chunk * 2)
    ncell = cfg["grid"]["n"][0] * cfg["grid"]["n"][1] * cfg["grid"]["n"][2]
    what = ("the headline workload's 320x320 cross-section with one cubic cell of crystal along z (same margins, "
            "CPML, pulse, probe, flux planes and energy: %dx%dx%d)" % tuple(cfg["grid"]["n"])
            if workload == "big320" else "the full %dx%dx%d grid" % tuple(cfg["grid"]["n"]))
    return {"value": ncell * n / dt, "unit": "cell-updates/s", "cores": O.threads(), "kind": "oracle",
            "sample": "steps 3..%d of %s, FP64 oracle, %.1f s of stepping" % (n + 2, what, dt)}


def measure_batched(args, kernel_steps=30):
    """The batched ensemble (64 uneven realizations, BATCH_TUNING) against the same
    realizations stepped one after another, each alone (SEQ_TUNING); the batch's dominant
    kernel class is timed per launch (hipEvents bound to the launches) against
    the summed algorithmic bytes of its members' tiles."""
    import torch
    from paper_0802_3775_amd import fdtd, tune
    from paper_0802_3775_amd import workloads as W
    steps = args.batch_steps
    cfgs = W.ensemble(count=64, steps=10000)
    if args.batch_tuning:
        tuning = fixed_tuning([int(q) for q in args.batch_tuning.split(",")])
    elif args.tune_side:
        tuning = tune.tune_batch(cfgs, budget_s=args.tune_seconds)
    else:
        tuning = fixed_tuning(BATCH_TUNING)
    cells = sum(c["grid"]["n"][0] * c["grid"]["n"][1] * c["grid"]["n"][2] for c in cfgs)
    seq = None
    seq_tuning = None
    if not args.no_sequential:
        seq_tuning = (tune.common_tuning(cfgs, budget_s=args.tune_seconds) if args.tune_side
                      else fixed_tuning(SEQ_TUNING))
        seq = 0.0
        for c in cfgs:           # sequential plain: each realization alone
            p = fdtd.Plan(c, max_steps=steps + 50, tuning=seq_tuning)
            p.step(50)
            seq += timed_run(p, steps)
            p.close()
    total = steps + 100 + kernel_steps
    plans = [fdtd.Plan(c, max_steps=total, tuning=tuning) for c in cfgs]
    log("batched: %d realizations, %d cells, tuning %s (sequential runs: %s)" % (len(plans), cells, tuning, seq_tuning))
    b = fdtd.Batch(plans)
    b.step(100)
    torch.cuda.synchronize()
    log("batched: warm")
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log("batched: %d steps in %.3f s" % (steps, tb))
    ms, cnt = b.time_kernels(kernel_steps)
    log("batched: kernel table")
    nbytes, ncells = b.class_bytes(), b.class_cells()
    kern = {}
    for c, name in enumerate(fdtd.Plan.CLASSES):
        if cnt[c]:
            avg = ms[c] / cnt[c]
            kern[name] = {"avg_ms": avg, "launches": int(cnt[c]), "cells": int(ncells[c]),
                          "alg_bytes": float(nbytes[c]), "GBps": nbytes[c] / (avg * 1e-3) / 1e9}
    # algorithmic bytes of a whole batch step (every class, the DFT at its average
    # per-step share) over the measured time of a graph-replayed step
    step_bytes = sum(float(nbytes[c]) * cnt[c] for c in range(7)) / kernel_steps
    b.close()
    for p in plans:
        p.close()
    scale = 10000.0 / steps
    return {"realizations": len(cfgs), "cells": cells, "steps_timed": steps, "tuning": tuning,
            "sequential_tuning": seq_tuning,
            "cell_updates_per_s": cells * steps / tb,
            "sequential_cell_updates_per_s": cells * steps / seq if seq else None,
            "ms_per_step": 1e3 * tb / steps,
            "realizations_per_hour": 3600.0 * len(cfgs) / (tb * scale),
            "sequential_realizations_per_hour": 3600.0 * len(cfgs) / (seq * scale) if seq else None,
            "speedup_vs_sequential": seq / tb if seq else None,
            "roofline": _roofline(kern, _dominant(kern), "batched", tuning, None),
            "step_alg_GBps": step_bytes / (tb / steps) / 1e9,
            "step_frac": step_bytes / (tb / steps) / 1e9 / HBM_PEAK_GBS,
            "kernels": kern,
            "note": "10k-step runs extrapolated from %d timed steps per realization" % steps}


def measure_serving(args, plain_rate):
    """The serving stream at its own request sizes and lengths: crystals of
    (n res)^3 in [1e6, 3.3e7] cells (n in 4..10 cubic cells, res in 16..32 cells/a)
    plus margins and CPML, 70% linear transmission requests of 10,000 steps and
    30% Lorentz lasing requests of 20,000 steps, delta ~ U[0, 0.12] a; Poisson
    arrivals at rho times the sequential capacity estimated from the plain
    stepper's rate, for each rho; served (continuous batching) against
    sequential FIFO on the same trace.  Fewer requests than the stream's 200, so
    the benchmark stays within its time budget."""
    import torch
    from paper_0802_3775_amd import serve
    from paper_0802_3775_amd import workloads as W
    out = {}
    for rho in (0.9, 0.5):
        base = W.serving_trace(count=args.serve_requests, seed=42, rho=1.0, capacity_per_s=1.0)
        work = 0.0
        for r in base:
            c = serve.request_config(r)
            # lasing cells update at about a third of the linear rate (gain state, CPML on all faces)
            work += c["grid"]["n"][0] * c["grid"]["n"][1] * c["grid"]["n"][2] * r["steps"] * (
                3.0 if r["kind"] == "lasing" else 1.0)
        cap = plain_rate / (work / len(base))          # requests per second, sequential estimate
        lam = rho * cap
        reqs = [dict(r, arrival=r["arrival"] / lam) for r in base]
        backend = serve.GpuBackend()
        free, _ = torch.cuda.mem_get_info()
        srv = serve.Server(backend, budget_bytes=int(0.8 * free), chunk=args.serve_chunk, policy=args.serve_policy)
        wall = srv.run(reqs)
        s_b = serve.summarize(reqs, wall, srv.results, srv.failed)
        backend.close()
        backend2 = serve.GpuBackend()
        srv2, wall2 = serve.run_sequential(backend2, reqs)
        backend2.close()
        s_s = serve.summarize(reqs, wall2, srv2.results, srv2.failed)
        cells = [serve.request_cells(r) for r in reqs]
        out["rho_%.1f" % rho] = {"requests": len(reqs), "offered_rate_per_s": lam, "served": s_b,
                                 "sequential_fifo": s_s, "cells_min": min(cells), "cells_max": max(cells),
                                 "lasing_requests": sum(1 for r in reqs if r["kind"] == "lasing")}
        log("serving rho %.1f: served p50 %.2f s p99 %.2f s, FIFO p50 %.2f s p99 %.2f s" %
            (rho, s_b["p50_s"], s_b["p99_s"], s_s["p50_s"], s_s["p99_s"]))
    out["chunk_steps"] = args.serve_chunk
    out["policy"] = args.serve_policy
    out["note"] = ("%d requests per load (the stream has 200) at the stream's sizes (1M-33M crystal cells) and "
                   "lengths (10k linear / 20k lasing steps)" % args.serve_requests)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--kernel-steps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tune-seconds", type=float, default=15.0)
    ap.add_argument("--tune-side", action="store_true",
                    help="autotune the side measurements instead of their fixed launch shapes")
    ap.add_argument("--serve-requests", type=int, default=8)
    ap.add_argument("--serve-chunk", type=int, default=1000)
    ap.add_argument("--serve-policy", choices=("fifo", "srpt", "all"), default="fifo",
                    help="serving: which admitted requests each launch steps")
    ap.add_argument("--workload", choices=tuple(WORKLOADS), default="big320",
                    help="headline 320^3 grid (default); the others for profiling")
    ap.add_argument("--only", default="", help="comma list of side measurements to run (profiling): "
                    "slab,paper_beam,lasing168,lasing_density,paper_lasing,batched,serving")
    ap.add_argument("--tuning", default="", help="fixed tile_x,block,zchunk,graph_steps[,merge,parallel] (skip the autotuner)")
    ap.add_argument("--batch-tuning", default="",
                    help="fixed batch tuning tile_x,block,zchunk,graph_steps,merge,parallel,cache_mb (profiling)")
    ap.add_argument("--batch-steps", type=int, default=300, help="batched: timed steps")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched: skip the members-one-after-another baseline (profiling)")
    ap.add_argument("--skip-plain", action="store_true",
                    help="skip the headline measurement and print only the side measurements (profiling)")
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
    copy_gbs = copy_bandwidth()
    if args.skip_plain:
        out, value = {}, None
    else:
        out, value = headline(args, copy_gbs)
    only = set(q for q in args.only.split(",") if q)
    want = (lambda q: not args.no_extras and (not only or q in only))
    if want("slab"):
        log("slab 80x80x224 ...")
        out["slab_80x80x224"] = measure_side(args, "slab", 2000, 200, 200, copy_gbs)
    if want("paper_beam"):
        log("paper beam box ...")
        out["paper_beam_200"] = measure_side(args, "paper_beam", 400, 50, 100, copy_gbs)
    if want("lasing168"):
        log("lasing 168^3 ...")
        out["lasing_168"] = measure_side(args, "lasing168", 1000, 100, 50, copy_gbs)
    if want("lasing_density"):
        log("lasing 168^3, density matrix ...")
        out["lasing_density_168"] = measure_lasing_density(args)
    if want("paper_lasing"):
        log("paper lasing box ...")
        out["paper_lasing_200"] = measure_side(args, "paper_lasing", 300, 100, 50, copy_gbs)
    if want("batched"):
        log("batched ...")
        out["batched"] = measure_batched(args)
    if want("serving") and value is not None:
        log("serving ...")
        out["serving"] = measure_serving(args, value)
    print(json.dumps(out), flush=True)


def headline(args, copy_gbs):
    """The headline JSON fields: the plain stepper on the --workload grid, and the
    CPU oracle on its bounded sample."""
    plain = measure_plain(args)
    value = plain["ncell"] * args.steps / plain["wall"]
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
                   "cells": plain["ncell"], "tuning": plain["tuning"]},
        "roofline": _roofline(plain["kernels"], plain["dominant"], args.workload, plain["tuning"], plain["cfg"], copy_gbs),
        "kernels": plain["kernels"],
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = measure_cpu(args.workload, args.cpu_seconds)
    return out, value


if __name__ == "__main__":
    main()
