"""The batch entry point that allocates no device memory
(fdtd_batch_create_static: launch tables in the library's static per-GPU array)
against the allocating one (fdtd_batch_create), through the C ABI: bit-identical
fields, probes, flux and energy on two calls in a row, the second with fewer
and smaller members; tables beyond the static maximum are refused; a static
batch whose tables a later one replaced refuses to step."""
import ctypes as C

import numpy as np
import pytest

from paper_0802_3775_amd import workloads as W

pytestmark = pytest.mark.gpu

TUNE = {"block": 128, "tile_x": 16, "zchunk": 8, "graph_steps": 20}


def _cfgs(steps, big=True):
    out = [W.slab(delta=0.05, seed=31, res=10, cells=(2, 2, 3), steps=steps, nf=12, decim=4, energy_interval=10),
           W.lasing(res=8, cells=(2, 2, 2), pml=4, steps=steps, pump=1e13, noise=1e-3, n_init=(0.3, 0.1, 0.5, 0.1),
                    energy_interval=5)]
    if big:
        out.append(W.slab(delta=0.10, seed=32, res=12, cells=(2, 2, 2), steps=steps, nf=8, decim=3,
                          energy_interval=7))
    else:
        out = out[:1]
        out[0] = W.slab(delta=0.02, seed=33, res=8, cells=(1, 1, 2), steps=steps, nf=6, decim=2, energy_interval=9)
    return out


def _state(plan):
    out = [plan.fields()] + [plan.probe(p) for p in range(plan.nprobe)]
    out += [a for f in range(len(plan.nf)) for a in plan.flux(f)]
    if plan.cfg.get("energy_interval"):
        out.append(plan.energy())
    if any(m.get("gain") for m in plan.cfg["materials"]):
        out += [plan.populations(), plan.polarization()]
    return out


def _run(cfgs, steps, static):
    import torch
    from paper_0802_3775_amd import fdtd as F
    plans = [F.Plan(c, max_steps=steps, tuning=TUNE) for c in cfgs]
    b = F.Batch(plans, static=static)
    b.step(7)      # eager launches
    b.step(steps - 7)  # graph replay
    torch.cuda.synchronize()
    out = [_state(p) for p in plans]
    b.close()
    for p in plans:
        p.close()
    return out


@pytest.mark.parametrize("big", [True, False])
def test_static_batch_equals_allocating_batch(big):
    steps = 67
    want = _run(_cfgs(steps, big), steps, static=False)
    got = _run(_cfgs(steps, big), steps, static=True)
    for a, b in zip(got, want):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_static_tables_limit_and_replacement():
    import torch
    from paper_0802_3775_amd import fdtd as F
    steps = 10
    # one z-plane per tile: a 1 x 1 x 400000 column has 400,000 tiles of 48 bytes,
    # beyond the 16 MiB of the static array (refused before anything is written)
    cfg = W.homogeneous_box(n=(1, 1, 400000), periodic=(1, 1, 1), res=10, steps=steps)
    big = F.Plan(cfg, max_steps=steps, tuning=dict(TUNE, zchunk=1))
    arr = (C.c_void_p * 1)(big.h.value)
    h = C.c_void_p()
    assert F.lib().fdtd_batch_create_static(arr, 1, None, C.byref(h)) == -2
    assert b"static maximum" in F.lib().fdtd_last_error()
    big.close()
    p1 = F.Plan(_cfgs(steps, False)[0], max_steps=steps, tuning=TUNE)
    p2 = F.Plan(_cfgs(steps, False)[0], max_steps=steps, tuning=TUNE)
    first = F.Batch([p1], static=True)
    second = F.Batch([p2], static=True)   # takes over the tables
    with pytest.raises(F.FdtdError) as e:
        first.step(1)
    assert e.value.code == -4
    second.step(steps)
    torch.cuda.synchronize()
    assert p1.step_count == 0 and p2.step_count == steps
    first.close()
    second.close()
    p1.close()
    p2.close()
