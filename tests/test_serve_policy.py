"""Serving policy on the CPU with a host test double in place of the GPU
backend: admission by footprint, continuous joining at launch boundaries,
cancellation, allocation failure, non-finite results, oversized requests."""
import math

import pytest

from paper_0802_3775_amd.serve import Server, run_sequential, summarize, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class MockBackend:
    """Each step of a batch costs `step_cost` seconds of fake time (a batch
    advances all members at once, as the device does)."""

    def __init__(self, clock, step_cost=1e-3, fail_bind=(), nan_after=None):
        self.clock = clock
        self.step_cost = step_cost
        self.fail_bind = set(fail_bind)
        self.nan_after = nan_after or {}
        self.live = {}
        self.batches = []

    def prepare(self, req):
        return {"id": req["id"], "mem": req["mem"], "done": 0}

    def footprint(self, h):
        return h["mem"]

    def bind(self, h):
        if h["id"] in self.fail_bind:
            raise MemoryError("injected allocation failure")
        self.live[h["id"]] = h

    def step(self, hs, n):
        self.batches.append(sorted(h["id"] for h in hs))
        for h in hs:
            h["done"] += n
        self.clock.t += n * self.step_cost

    def sync(self):
        pass

    def healthy(self, h):
        lim = self.nan_after.get(h["id"])
        return lim is None or h["done"] < lim

    def result(self, h):
        return {"steps": h["done"], "value": h["id"] * 1000 + h["done"]}

    def release(self, h):
        del self.live[h["id"]]


def _req(i, arrival, steps, mem):
    return {"id": i, "arrival": arrival, "steps": steps, "mem": mem}


def test_admission_by_footprint_and_continuous_join():
    clk = FakeClock()
    be = MockBackend(clk)
    srv = Server(be, budget_bytes=100, chunk=100, clock=clk, sleep=clk.sleep)
    reqs = [_req(0, 0.0, 400, 60), _req(1, 0.0, 200, 30), _req(2, 0.05, 200, 50), _req(3, 0.15, 100, 10)]
    srv.run(reqs)
    assert set(srv.results) == {0, 1, 2, 3} and not srv.failed
    assert all(srv.results[r["id"]]["steps"] == r["steps"] for r in reqs)
    # request 2 (50) does not fit beside 0 and 1 (90 of 100): it waits for request 1 to finish
    adm = {rid: t for ev, rid, t in srv.log if ev == "admit"}
    done = {rid: t for ev, rid, t in srv.log if ev == "done"}
    assert adm[2] >= done[1]
    # request 3 arrived while others ran and joined a running batch
    assert any(3 in b and len(b) > 1 for b in be.batches)
    assert be.live == {} and srv.used == 0


def test_head_of_line_and_oversized_request():
    clk = FakeClock()
    be = MockBackend(clk)
    srv = Server(be, budget_bytes=100, chunk=50, clock=clk, sleep=clk.sleep)
    reqs = [_req(0, 0.0, 100, 80), _req(1, 0.0, 100, 500), _req(2, 0.0, 100, 30)]
    srv.run(reqs)
    assert "exceeds" in srv.failed[1]
    assert set(srv.results) == {0, 2}


def test_cancellation_and_injected_failures():
    clk = FakeClock()
    be = MockBackend(clk, fail_bind={1}, nan_after={2: 150})
    srv = Server(be, budget_bytes=1000, chunk=50, clock=clk, sleep=clk.sleep)
    reqs = [_req(0, 0.0, 300, 10), _req(1, 0.0, 300, 10), _req(2, 0.0, 300, 10), _req(3, 0.0, 300, 10),
            _req(4, 0.2, 300, 10)]
    srv.cancel(3)
    srv.run(reqs)
    assert "bind failed" in srv.failed[1]
    assert srv.failed[2] == "non-finite field"
    assert "cancelled" in srv.failed[3]
    assert set(srv.results) == {0, 4}
    # the failure of request 2 did not stop its batch-mate
    assert srv.results[0]["steps"] == 300
    assert be.live == {}


def test_sequential_baseline_and_summary():
    clk = FakeClock()
    reqs = [_req(i, 0.01 * i, 200, 10) for i in range(6)]
    srv, wall = run_sequential(MockBackend(clk), reqs, clock=clk, sleep=clk.sleep)
    assert set(srv.results) == set(range(6))
    s1 = summarize(reqs, wall, srv.results, srv.failed)
    clk2 = FakeClock()
    srv2 = Server(MockBackend(clk2), budget_bytes=1000, chunk=100, clock=clk2, sleep=clk2.sleep)
    wall2 = srv2.run(reqs)
    s2 = summarize(reqs, wall2, srv2.results, srv2.failed)
    # batched serving finishes the same work sooner (each batched step covers all members)
    assert s2["wall_s"] < s1["wall_s"] and s2["p99_s"] < s1["p99_s"]
    for r in reqs:
        assert srv.results[r["id"]]["value"] == srv2.results[r["id"]]["value"]


class SizedBackend(MockBackend):
    """Steps cost time in proportion to the cells they advance (a device that
    is busy with every member of a launch), and each request has a size."""

    def prepare(self, req):
        return {"id": req["id"], "mem": req["mem"], "done": 0, "cells": req["cells"]}

    def work(self, h, steps):
        return h["cells"] * steps

    def step(self, hs, n):
        self.batches.append(sorted(h["id"] for h in hs))
        for h in hs:
            h["done"] += n
        self.clock.t += n * self.step_cost * sum(h["cells"] for h in hs)


def _sized(i, arrival, steps, cells):
    return {"id": i, "arrival": arrival, "steps": steps, "mem": 10, "cells": cells}


def test_shortest_remaining_work_first_groups_similar_requests():
    """With policy srpt a launch steps the admitted requests whose remaining work
    is within group_factor of the smallest: a small request that arrives while a
    large one runs is served ahead of it, similar requests share launches, and
    every request still completes with all its steps."""
    reqs = [_sized(0, 0.0, 1000, 100), _sized(1, 0.01, 1000, 5), _sized(2, 0.01, 1000, 6), _sized(3, 0.02, 500, 100)]
    out = {}
    for policy in ("srpt", "all"):
        clk = FakeClock()
        be = SizedBackend(clk, step_cost=1e-6)
        srv = Server(be, budget_bytes=1000, chunk=100, clock=clk, sleep=clk.sleep, policy=policy)
        srv.run(reqs)
        assert set(srv.results) == {0, 1, 2, 3} and not srv.failed
        assert all(srv.results[r["id"]]["steps"] == r["steps"] for r in reqs)
        done = {rid: t for ev, rid, t in srv.log if ev == "done"}
        out[policy] = (be.batches, done, summarize(reqs, srv.clock(), srv.results, srv.failed))
    batches, done, s_srpt = out["srpt"]
    # the two small requests ran together, apart from the large ones, and finished first
    assert [1, 2] in batches and not any(1 in b and 0 in b for b in batches)
    assert max(done[1], done[2]) < min(done[0], done[3])
    # and their latency beats stepping every admitted request at once
    _, done_all, s_all = out["all"]
    assert max(done[1], done[2]) < max(done_all[1], done_all[2])
    assert s_srpt["p50_s"] < s_all["p50_s"]


def test_fifo_with_small_riders():
    """With policy fifo the oldest admitted request is stepped first, and small
    requests ride along while their remaining work together stays within
    ride_frac of its remaining work: the large requests finish in arrival order,
    the oldest no later than its own work plus the riders' (on a device that is
    busy with every member of a launch), and a request too large to ride waits
    its turn."""
    reqs = [_sized(0, 0.0, 1000, 100), _sized(1, 0.01, 1000, 5), _sized(2, 0.01, 1000, 6),
            _sized(3, 0.02, 1000, 100)]
    clk = FakeClock()
    be = SizedBackend(clk, step_cost=1e-6)
    srv = Server(be, budget_bytes=1000, chunk=100, clock=clk, sleep=clk.sleep, policy="fifo", ride_frac=0.25)
    srv.run(reqs)
    assert set(srv.results) == {0, 1, 2, 3} and not srv.failed
    assert all(srv.results[r["id"]]["steps"] == r["steps"] for r in reqs)
    done = {rid: t for ev, rid, t in srv.log if ev == "done"}
    # both small requests rode with the head once admitted
    assert any(b == [0, 1, 2] for b in be.batches)
    # first come, first served among the large ones; 3 never shared a launch with 0
    assert done[0] < done[3]
    assert not any(3 in b and 0 in b for b in be.batches)
    # the head took at most its own work plus the riders' (1000 steps x (100 + 5 + 6) cells)
    assert done[0] <= 1000 * 1e-6 * (100 + 5 + 6) + 1e-9
    # a rider too large for the share (20 x 1000 > 0.125 x 100 x 1000) waits its turn
    clk2 = FakeClock()
    be2 = SizedBackend(clk2, step_cost=1e-6)
    big = [_sized(0, 0.0, 1000, 100), _sized(1, 0.01, 1000, 20)]
    srv2 = Server(be2, budget_bytes=1000, chunk=100, clock=clk2, sleep=clk2.sleep, policy="fifo", ride_frac=0.125)
    srv2.run(big)
    assert set(srv2.results) == {0, 1}
    assert not any(0 in b and 1 in b for b in be2.batches)


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile([5], 99) == 5
    assert math.isnan(percentile([], 50))
