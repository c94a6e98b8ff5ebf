"""Continuous-batching server on the GPU: requests that join while others run
(linear, Lorentz lasing and density-matrix lasing, the last in a batch of their
own) produce exactly the results they produce when run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _trace():
    return [
        # long enough (several 10 ms) that the later arrivals join while it runs
        {"id": 0, "arrival": 0.00, "kind": "linear", "n": 1, "res": 10, "delta": 0.05, "seed": 501, "steps": 8000, "nf": 12},
        {"id": 1, "arrival": 0.00, "kind": "lasing", "n": 1, "res": 8, "delta": 0.08, "seed": 502, "steps": 400},
        {"id": 2, "arrival": 0.02, "kind": "linear", "n": 2, "res": 8, "delta": 0.00, "seed": 503, "steps": 400, "nf": 8},
        {"id": 3, "arrival": 0.05, "kind": "linear", "n": 1, "res": 12, "delta": 0.10, "seed": 504, "steps": 800, "nf": 10},
        {"id": 4, "arrival": 0.08, "kind": "lasing", "n": 1, "res": 10, "delta": 0.03, "seed": 505, "steps": 400},
        # density-matrix dye: a batch of their own beside the others
        {"id": 5, "arrival": 0.00, "kind": "lasing", "model": "density", "n": 1, "res": 8, "delta": 0.05,
         "seed": 506, "steps": 600},
        {"id": 6, "arrival": 0.03, "kind": "lasing", "model": "density", "n": 1, "res": 10, "delta": 0.02,
         "seed": 507, "steps": 400},
    ]


def _alone(req, tuning):
    import torch
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd.serve import request_config
    plan = fdtd.Plan(request_config(req), max_steps=req["steps"], tuning=tuning)
    plan.step(req["steps"])
    torch.cuda.synchronize()
    out = {"probe": [plan.probe(q) for q in range(plan.nprobe)]}
    if plan.nf:
        out["flux"] = [plan.flux(f) for f in range(len(plan.nf))]
    out["energy"] = plan.energy()
    plan.close()
    return out


def test_mix_equals_alone_bitwise():
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd.serve import GpuBackend, Server, summarize
    tuning = fdtd.default_tuning()
    backend = GpuBackend(tuning)
    srv = Server(backend, budget_bytes=8 << 30, chunk=200)
    reqs = _trace()
    wall = srv.run(reqs)
    assert not srv.failed, srv.failed
    # requests really overlapped on the device
    adm = {rid: t for ev, rid, t in srv.log if ev == "admit"}
    done = {rid: t for ev, rid, t in srv.log if ev == "done"}
    assert any(adm[b] < done[a] and adm[a] < adm[b] for a in adm for b in adm if a != b)
    for req in reqs:
        ref = _alone(req, tuning)
        got = srv.results[req["id"]]
        for a, b in zip(got["probe"], ref["probe"]):
            assert np.array_equal(a, b)
        for (Ta, Sa), (Tb, Sb) in zip(got.get("flux", []), ref.get("flux", [])):
            assert np.array_equal(Ta, Tb) and np.array_equal(Sa, Sb)
        assert np.array_equal(got["energy"], ref["energy"])
    s = summarize(reqs, wall, srv.results, srv.failed)
    assert s["completed"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0


def test_budget_forces_queueing():
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd.serve import GpuBackend, Server
    backend = GpuBackend(fdtd.default_tuning())
    reqs = _trace()[:3]
    sizes = [backend.footprint(backend.prepare(r)) for r in reqs]
    srv = Server(backend, budget_bytes=max(sizes) + min(sizes) // 2, chunk=200)
    srv.run(reqs)
    assert not srv.failed and len(srv.results) == 3
    # never more than one large request resident at a time
    admits = [t for ev, _, t in srv.log if ev == "admit"]
    assert len(admits) == 3


def test_served_requests_match_the_oracle():
    """Requests served in the mix (a linear slab and a Lorentz lasing box joining
    while others run) against the oracle's runs of the same request
    configurations: probe, T(t), spectra and energy."""
    from gpu_common import rel_l2, run_oracle
    from paper_0802_3775_amd import fdtd
    from paper_0802_3775_amd.serve import GpuBackend, Server, request_config
    backend = GpuBackend(fdtd.default_tuning())
    srv = Server(backend, budget_bytes=8 << 30, chunk=200)
    reqs = _trace()
    srv.run(reqs)
    assert not srv.failed, srv.failed
    for rid, tol in ((3, 1e-4), (4, 1e-3)):
        req = reqs[rid]
        orc = run_oracle(request_config(req), req["steps"])
        got = srv.results[rid]
        perr = rel_l2(got["probe"][0], orc.probe(0))
        werr = rel_l2(got["energy"], orc.energy())
        print("request", rid, req["kind"], "probe", perr, "energy", werr, flush=True)
        assert perr <= tol and werr <= tol
        for f, (T, S) in enumerate(got.get("flux", [])):
            To, So = orc.flux(f)
            assert rel_l2(T, To) <= 1e-3 and rel_l2(S, So) <= 1e-3
