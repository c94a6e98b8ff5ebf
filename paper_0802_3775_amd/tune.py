"""Autotuner for the launch configuration of a plan.

A tuning is {tile_x, block, zchunk, graph_steps, max_blocks, merge, parallel}:
the xy tile of a workgroup (tile_x x block/tile_x columns), the number of
z-planes each tile marches, the number of steps captured in one hipGraph, an
optional cap on resident workgroups, how tile classes are folded into launches
and whether a step's launches are parallel graph branches.  Fields are bit-identical for every tuning (each cell's
arithmetic does not depend on the tiling), so the tuner is free to pick the
fastest.  It times candidate tunings through the library's fdtd_tune (scratch plans of
the same description bound in turn to one scratch arena), keeps the fastest,
and caches the choice per shape bin in a JSON file.
"""
import itertools
import json
import os
import time

CACHE_VERSION = 8


def _cache_path():
    base = os.environ.get("FDTD_TUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_0802_3775_amd", "tune.json")


def shape_key(cfg):
    """Shape bin: grid extents, boundary/CPML layout, gain model and flux presence."""
    g = cfg["grid"]
    gain = max(int(m.get("gain") or 0) for m in cfg["materials"])  # gain model (0 none)
    nflux = sum(1 for f in cfg.get("flux", []) if len(f.get("freqs", ())) > 0)
    return "v%d|n=%s|per=%s|pml=%s,%s|gain=%d|flux=%d" % (
        CACHE_VERSION, tuple(g["n"]), tuple(g.get("periodic", (1, 1, 1))), tuple(g.get("pml_lo", (0, 0, 0))),
        tuple(g.get("pml_hi", (0, 0, 0))), int(gain), nflux)


def candidates(cfg, quick=False):
    nx, ny, nz = cfg["grid"]["n"]
    # the usual winners first (the search stops at its time budget): wide tiles
    # and the chunk lengths that won on grids of 1-42 M cells
    tiles = [(64, 256), (32, 256), (16, 256), (32, 128), (16, 128)]
    if quick:
        tiles = [(64, 256), (32, 256), (16, 256)]
    chunks = [8, 16, 48, 4, 32, 64, 2, 1]
    out = []
    for (tx, b), z in itertools.product(tiles, chunks):
        if tx > 16 and tx > 2 * nx:
            continue
        if z > nz:
            continue
        out.append({"tile_x": tx, "block": b, "zchunk": z, "max_blocks": 0, "merge": 1, "parallel": 0})
    return out


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time_candidates(cfg, tunes, steps, warm):
    """Milliseconds per step of each tuning, timed by the library's fdtd_tune on
    scratch plans of cfg's description (one scratch arena for all); infinity for
    a tuning the library rejects."""
    from . import fdtd
    plan = fdtd.Plan(cfg, max_steps=warm + steps, bind=False)
    try:
        return [float("inf") if ms is None else ms for ms in plan.tune(tunes, steps, warmup=warm)]
    finally:
        plan.close()


def _time_candidate(cfg, tune, steps, warm):
    return _time_candidates(cfg, [tune], steps, warm)[0]


def autotune(cfg, budget_s=20.0, quick=False, use_cache=True, graph_steps=(50, 200), verbose=False):
    """Return the fastest tuning for this configuration's shape (cached)."""
    key = shape_key(cfg)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return dict(cache[key]["tuning"])
    ncell = cfg["grid"]["n"][0] * cfg["grid"]["n"][1] * cfg["grid"]["n"][2]
    # steps per trial: about 2e8 cell-updates, at least 20 (fewer left the
    # choice between shapes within a few percent of each other to noise)
    steps = int(max(20, min(200, 2e8 / max(ncell, 1))))
    t_end = time.perf_counter() + budget_s
    best, best_ms = None, float("inf")
    results = []
    cands = [dict(c, graph_steps=min(graph_steps)) for c in candidates(cfg, quick=quick)]
    for q0 in range(0, len(cands), 6):  # a few candidates per library call, budget checked between
        if time.perf_counter() > t_end and best is not None:
            break
        group = cands[q0:q0 + 6]
        for tune, ms in zip(group, _time_candidates(dict(cfg, steps=steps + 4), group, steps, 4)):
            results.append((ms, tune))
            if verbose:
                print("tune %s: %.2f us/step" % (tune, ms * 1e3), flush=True)
            if ms < best_ms:
                best, best_ms = tune, ms
    # launch grouping: classes folded into fewer launches, or launches as
    # parallel graph branches, for the three fastest shapes (the grouping and
    # the shape interact: on boxes with CPML on every face the all-in-one
    # launch favours wider tiles than the per-class launches do)
    results.sort(key=lambda r: r[0])
    groupings = [dict(t, merge=merge, parallel=par) for _, t in results[:3]
                 for merge, par in ((0, 0), (0, 1), (1, 1), (2, 0))]
    for tune, ms in zip(groupings, _time_candidates(dict(cfg, steps=steps + 4), groupings, steps, 4)):
        if verbose:
            print("tune %s: %.2f us/step" % (tune, ms * 1e3), flush=True)
        if ms < best_ms:
            best, best_ms = tune, ms
    # graph length: longer graphs amortise launches; keep the faster
    for gsteps in graph_steps:
        if gsteps == best["graph_steps"]:
            continue
        n = max(steps, gsteps)
        tune = dict(best, graph_steps=gsteps)
        ms = _time_candidate(dict(cfg, steps=n + 4), tune, n, 4)
        if verbose:
            print("tune %s: %.2f us/step" % (tune, ms * 1e3), flush=True)
        if ms < best_ms:
            best, best_ms = tune, ms
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": best, "us_per_step": best_ms * 1e3, "trials": len(results)}
        _save_cache(cache)
    return dict(best)


def common_tuning(cfgs, budget_s=30.0, verbose=False):
    """One tuning for a batch (members share tile_x and block): tune the largest
    member, keep its tile shape for all."""
    big = max(cfgs, key=lambda c: c["grid"]["n"][0] * c["grid"]["n"][1] * c["grid"]["n"][2])
    return autotune(big, budget_s=budget_s, verbose=verbose)


def _cells(c):
    n = c["grid"]["n"]
    return n[0] * n[1] * n[2]


def _time_batch(cfgs, tune, steps, warm):
    import torch
    from . import fdtd
    plans = [fdtd.Plan(dict(c, steps=steps + warm), max_steps=steps + warm, tuning=tune) for c in cfgs]
    b = None
    try:
        b = fdtd.Batch(plans)
        b.step(warm)
        torch.cuda.synchronize()
        return b.time_steps(steps) / steps
    finally:
        if b is not None:
            b.close()
        for p in plans:
            p.close()


def tune_batch(cfgs, budget_s=20.0, sample=8, use_cache=True, verbose=False):
    """One tuning for a batch of uneven realizations, timed on the batch itself:
    a sample of members spread over the size range is stepped as a Batch for
    every candidate tile shape (members share tile_x and block, and a tile wider
    than a member's grid wastes lanes, so the largest member's own best is not
    the batch's), then for member-group sizes and class groupings."""
    members = sorted(cfgs, key=_cells)
    if len(members) > sample:
        idx = [round(q * (len(members) - 1) / (sample - 1)) for q in range(sample)]
        members = [members[q] for q in sorted(set(idx))]
    key = "batch|" + "|".join(sorted(shape_key(c) for c in members))
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return dict(cache[key]["tuning"])
    total = sum(_cells(c) for c in members)
    steps = int(max(8, min(100, 2e8 / max(total, 1))))
    t0 = time.perf_counter()
    best, best_ms = None, float("inf")

    def trial(tune):
        nonlocal best, best_ms
        ms = _time_batch(members, tune, steps, 4)
        if verbose:
            print("batch tune %s: %.2f us/step" % (tune, ms * 1e3), flush=True)
        if ms < best_ms:
            best, best_ms = tune, ms

    # tile shapes within 60% of the budget, then member groups that fit the
    # 256 MB Infinity Cache (the sample's state already exceeds it; above it a
    # group streams from HBM) whatever the time, then the class grouping
    for cand in candidates(members[-1]):
        if time.perf_counter() - t0 > 0.6 * budget_s and best is not None:
            break
        trial(dict(cand, graph_steps=50))
    base = dict(best)
    for mb in (192, 224, 256):
        trial(dict(base, cache_mb=mb))
    base = dict(best)
    for merge, par in ((0, 0), (2, 0)):
        if time.perf_counter() - t0 > budget_s:
            break
        trial(dict(base, merge=merge, parallel=par))
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": best, "us_per_step": best_ms * 1e3}
        _save_cache(cache)
    return dict(best)
