"""Continuous-batching solve server for disorder-realization requests.

Requests (linear transmission runs or lasing runs of given size, resolution,
disorder and seed) arrive over time.  The server admits them in arrival order
while their HBM footprint fits the budget, keeps every admitted request's
fields resident in its own device arena, and steps admitted requests together
in batched launches of up to `chunk` steps.  At every launch boundary it
retires finished requests (results copied to the host), frees their arenas,
and admits waiting requests into the freed memory, so new work joins while
older work is still running.  Each request keeps its own step counter, source
timing and DFT phase, so its result is bit-identical to a run of the same
request alone.

Which admitted requests a launch steps: with policy "fifo" (the default), the
oldest admitted request, joined by the smallest others as long as their
remaining work (cells x remaining steps, lasing cells weighted by their higher
per-cell cost) together stays within `ride_frac` of its own -- first come first
served, the order that minimises the largest latency on one device, with small
requests progressing alongside instead of waiting behind it; with policy
"srpt", the group whose remaining work is within `group_factor` of the
smallest -- the shortest-remaining-work-first order, which minimises mean
latency when requests are small and starves the large ones when they are not;
with policy "all", every admitted request.  Requests outside the group stay resident and continue when
their turn comes.

The scheduling policy (Server) is independent of the device: a Backend does
the work.  GpuBackend drives libfdtd; tests drive the same policy with a host
test double.
"""
import math
import time

from . import workloads as W

# Launch shape of served requests: one block size and tile width for all (batch
# members share them); CPML on all faces (lasing boxes) folds every tile into
# the all-axes kernel, the z-CPML slabs keep interior tiles in the lighter one.
SERVE_TUNING = {"block": 256, "tile_x": 32, "zchunk": 8, "graph_steps": 50, "max_blocks": 0, "merge": 1,
                "parallel": 0, "stores": 0}
SERVE_TUNING_LASING = dict(SERVE_TUNING, zchunk=4, merge=2)
# per-cell cost of a lasing request relative to a linear one (gain state, CPML on all faces)
LASING_COST = 3.0


def request_config(req):
    """Workload dict of a request: linear slab (crystal n^3 cubic cells at `res`,
    vacuum margins, z-CPML, pulse, transmission flux) or lasing box (n^3 cells,
    CPML on all faces, gain voids at pump 1e10 s^-1; req["model"] = "density"
    fills them with the density-matrix dye instead of the Lorentz medium)."""
    n, res = int(req["n"]), int(req["res"])
    if req["kind"] == "linear":
        cfg = W.slab(delta=req["delta"], seed=req["seed"], res=res, cells=(n, n, n), steps=req["steps"],
                     nf=req.get("nf", 100), decim=8, energy_interval=req.get("energy_interval", 100))
    else:
        cfg = W.lasing(pump=req.get("pump", 1e10), delta=req["delta"], seed=req["seed"], res=res,
                       cells=(n, n, n), steps=req["steps"], energy_interval=req.get("energy_interval", 100),
                       model=req.get("model", "lorentz"))
    cfg["name"] = "req%d_%s" % (req["id"], cfg["name"])
    return cfg


def request_cells(req):
    """Cells of the request's grid (crystal, margins and CPML)."""
    n = request_config(dict(req, steps=1))["grid"]["n"]
    return n[0] * n[1] * n[2]


class GpuBackend:
    """libfdtd plans and batches; one torch uint8 arena per request.  A group of
    one steps on the plain stepper; larger groups step as one batch per gain
    model (members of a batch share a gain model: density-matrix requests in one,
    linear and Lorentz requests in the other), kept for the whole run and given
    its new members in place when the group changes."""

    def __init__(self, tuning=None):
        import torch
        from . import fdtd
        self.fdtd = fdtd
        self.torch = torch
        self.tuning = tuning
        self._batch = {}
        self._members = {}

    def prepare(self, req):
        cfg = request_config(req)
        lasing = req["kind"] != "linear"
        tune = self.tuning or (SERVE_TUNING_LASING if lasing else SERVE_TUNING)
        plan = self.fdtd.Plan(cfg, max_steps=req["steps"], tuning=tune, bind=False)
        dm = any(int(m.get("gain") or 0) == 2 for m in cfg["materials"])
        return {"plan": plan, "cfg": cfg, "bytes": plan.required_bytes() + 256, "group": int(dm),
                "cells": plan.ncell, "cost": LASING_COST if lasing else 1.0}

    def footprint(self, h):
        return h["bytes"]

    def work(self, h, steps):
        return h["cells"] * h["cost"] * steps

    def bind(self, h):
        h["plan"].bind()

    def step(self, hs, n):
        groups = {}
        for h in hs:
            groups.setdefault(h["group"], []).append(h)
        for key, g in groups.items():
            if len(g) == 1:
                g[0]["plan"].step(n)   # a lone request runs on the plain stepper
                continue
            members = tuple(id(h["plan"]) for h in g)
            plans = [h["plan"] for h in g]
            if self._batch.get(key) is None:
                self._batch[key] = self.fdtd.Batch(plans)
            elif members != self._members.get(key):
                self._batch[key].set_members(plans)
            self._members[key] = members
            self._batch[key].step(n)

    def sync(self):
        self.torch.cuda.synchronize()

    def healthy(self, h):
        p = h["plan"]
        if p.cfg.get("energy_interval") and p.step_count > 0:
            w = p.energy()
            if len(w) and not math.isfinite(float(w[-1])):
                return False
        if p.nprobe and p.step_count > 0:
            v = p.probe(0)
            if len(v) and not math.isfinite(float(v[-1])):
                return False
        return True

    def result(self, h):
        p = h["plan"]
        out = {"probe": [p.probe(q) for q in range(p.nprobe)], "steps": p.step_count}
        if p.nf:
            out["flux"] = [p.flux(f) for f in range(len(p.nf))]
        if p.cfg.get("energy_interval"):
            out["energy"] = p.energy()
        return out

    def release(self, h):
        # a batch whose member list still names this plan is not stepped again
        # before set_members gives it the next group
        for key in list(self._members):
            if id(h["plan"]) in self._members[key]:
                self._members[key] = ()
        h["plan"].close()

    def close(self):
        for b in self._batch.values():
            if b is not None:
                b.close()
        self._batch, self._members = {}, {}


class Server:
    """Arrival-ordered admission by footprint; batched stepping in chunks."""

    def __init__(self, backend, budget_bytes, chunk=400, max_active=64, clock=None, sleep=None, policy="fifo",
                 group_factor=4.0, ride_frac=0.125):
        if policy not in ("srpt", "fifo", "all"):
            raise ValueError("policy must be 'srpt', 'fifo' or 'all'")
        self.policy = policy
        self.group_factor = float(group_factor)
        self.ride_frac = float(ride_frac)
        self.backend = backend
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.max_active = int(max_active)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.pending = []     # (req, handle) in arrival order
        self.active = []      # dicts: req, h, done
        self.used = 0
        self.results = {}
        self.failed = {}
        self.cancelled = set()
        self.log = []

    def cancel(self, rid):
        self.cancelled.add(rid)

    def _admit(self, now):
        while self.pending and self.pending[0][0]["arrival"] <= now and len(self.active) < self.max_active:
            req, h = self.pending[0]
            if req["id"] in self.cancelled:
                self.pending.pop(0)
                self.failed[req["id"]] = "cancelled before admission"
                continue
            need = self.backend.footprint(h)
            if need > self.budget:
                self.pending.pop(0)
                self.failed[req["id"]] = "footprint %d exceeds the budget %d" % (need, self.budget)
                continue
            if self.used + need > self.budget:
                break  # head of line waits for memory
            self.pending.pop(0)
            try:
                self.backend.bind(h)
            except Exception as e:  # allocation failure: report, keep serving others
                self.failed[req["id"]] = "bind failed: %s" % (e,)
                continue
            self.used += need
            self.active.append({"req": req, "h": h, "done": 0, "admitted": now})
            self.log.append(("admit", req["id"], now))

    def _retire(self, entry, now, ok=True, why=""):
        req = entry["req"]
        if ok:
            res = self.backend.result(entry["h"])
            res["latency"] = now - req["arrival"]
            res["admitted"] = entry["admitted"]
            self.results[req["id"]] = res
            self.log.append(("done", req["id"], now))
        else:
            self.failed[req["id"]] = why
            self.log.append(("fail", req["id"], now))
        self.backend.release(entry["h"])
        self.used -= self.backend.footprint(entry["h"])

    def _group(self):
        """The admitted requests the next launch steps (see the module notes)."""
        if self.policy == "all" or len(self.active) == 1 or not hasattr(self.backend, "work"):
            return list(self.active)
        w = [self.backend.work(e["h"], e["req"]["steps"] - e["done"]) for e in self.active]
        if self.policy == "fifo":
            head = min(range(len(self.active)), key=lambda q: (self.active[q]["req"]["arrival"],
                                                                self.active[q]["req"]["id"]))
            group, ride = [self.active[head]], 0.0
            for q in sorted((q for q in range(len(self.active)) if q != head), key=lambda q: w[q]):
                if ride + w[q] > self.ride_frac * w[head]:
                    break
                ride += w[q]
                group.append(self.active[q])
            return group
        wmin = min(w)
        return [e for e, x in zip(self.active, w) if x <= self.group_factor * wmin]

    def run(self, requests):
        """Serve the requests (each with an 'arrival' time in seconds relative to the
        start of run); returns wall time."""
        reqs = sorted(requests, key=lambda r: (r["arrival"], r["id"]))
        self.pending = [(r, self.backend.prepare(r)) for r in reqs]
        t0 = self.clock()
        while self.pending or self.active:
            now = self.clock() - t0
            self._admit(now)
            if not self.active:
                if self.pending:
                    wait = self.pending[0][0]["arrival"] - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                    elif self.used == 0:
                        # nothing running and the head request cannot be admitted
                        req, h = self.pending.pop(0)
                        self.failed[req["id"]] = "not admissible"
                continue
            for e in list(self.active):
                if e["req"]["id"] in self.cancelled:
                    self.active.remove(e)
                    self._retire(e, self.clock() - t0, ok=False, why="cancelled")
            if not self.active:
                continue
            group = self._group()
            n = min(self.chunk, min(e["req"]["steps"] - e["done"] for e in group))
            self.backend.step([e["h"] for e in group], n)
            self.backend.sync()
            now = self.clock() - t0
            for e in group:
                e["done"] += n
                if not self.backend.healthy(e["h"]):
                    self.active.remove(e)
                    self._retire(e, now, ok=False, why="non-finite field")
                elif e["done"] >= e["req"]["steps"]:
                    self.active.remove(e)
                    self._retire(e, now)
        return self.clock() - t0


def percentile(vals, q):
    v = sorted(vals)
    if not v:
        return float("nan")
    pos = (len(v) - 1) * q / 100.0
    lo, hi = int(math.floor(pos)), int(math.ceil(pos))
    return v[lo] + (v[hi] - v[lo]) * (pos - lo)


def summarize(requests, wall, results, failed):
    lat = [results[r["id"]]["latency"] for r in requests if r["id"] in results]
    return {"requests": len(requests), "completed": len(lat), "failed": len(failed),
            "wall_s": wall, "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "realizations_per_hour": 3600.0 * len(lat) / wall if wall > 0 else float("nan")}


def run_sequential(backend, requests, clock=None, sleep=None):
    """Baseline: one request at a time, in arrival order, each stepped alone."""
    srv = Server(backend, budget_bytes=1 << 62, chunk=1 << 30, max_active=1, clock=clock, sleep=sleep)
    wall = srv.run(requests)
    return srv, wall
