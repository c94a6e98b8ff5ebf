"""GPU parity at the workloads' full sizes and lengths, against stored oracle runs.

The FP64 oracle needs minutes to hours for these runs, so tests/golden/
make_oracle_runs.py ran it once on the CPU and stored every field component at a
seeded sample of cells at a few checkpoints, the transmitted power T(t), the flux
spectra, the probe and energy records, and for the lasing box the populations
and polarization at sampled gain cells.  The GPU runs here at full size, in the
launch configuration the autotuner picks, and is compared with those samples
(field relative L2 over the sampled cells; every T(t), probe and spectrum value).

Tolerances: linear runs fields <= 1e-4, T(t) and spectra <= 1e-3; lasing runs
fields <= 1e-3 (and the density matrix <= 1e-3); populations: the change from the initial state agrees with the
oracle's to 1e-3 of its size and 1e-6 absolute (the oracle evolves all four
levels; the GPU stores n1..n3 and takes n0 = 1 - (n1 + n2 + n3), so the sum is 1
by construction and the oracle's separately evolved N0 is the evidence).
"""
import importlib.util
import os

import numpy as np
import pytest

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixtures():
    spec = importlib.util.spec_from_file_location("make_oracle_runs", os.path.join(HERE, "golden", "make_oracle_runs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


FX = _fixtures()


def _say(*a):
    print(*a, flush=True)


def _sampled_rel(fields, fx, idx):
    g = fields.reshape(6, -1)[:, idx].astype(np.float64)
    o = fx.astype(np.float64)
    return max(rel_l2(g[:3], o[:3]), rel_l2(g[3:], o[3:]))


def _tuned(cfg, **extra):
    from paper_0802_3775_amd import tune
    t = tune.autotune(dict(cfg, steps=200), budget_s=3.0, quick=True, use_cache=False)
    t.update(extra)
    return t


def _run_checkpoints(name, tol_fields, tuning_extra=None, fields=True):
    """Step the GPU through the fixture's checkpoints; returns (plan, fixture).
    fields=False: the run ends empty (the pulse has left through the CPML and the
    oracle's field norm is rounding residue), so only the diagnostics compare."""
    import torch
    from paper_0802_3775_amd import fdtd as F
    build, _ = FX.RUNS[name]
    cfg = build()
    fx = FX.load(name)
    tuning = _tuned(cfg, **(tuning_extra or {}))
    _say(name, cfg["grid"]["n"], "checkpoints", list(fx["checkpoints"]), "tuning", tuning)
    plan = F.Plan(cfg, max_steps=cfg["steps"], tuning=tuning)
    done = 0
    for cp in fx["checkpoints"]:
        plan.step(int(cp) - done)
        done = int(cp)
        torch.cuda.synchronize()
        if not fields:
            _say("  step", cp, "oracle field norms", fx["norm_%d" % cp], "(not compared)")
            continue
        err = _sampled_rel(plan.fields(), fx["f_%d" % cp], fx["idx"])
        _say("  step", cp, "sampled field rel L2", err)
        assert err <= tol_fields, (name, cp, err)
        if "gain_idx" in fx:
            _check_populations(plan, fx, cp)
    return plan, fx


def _check_populations(plan, fx, cp):
    gi = fx["gain_idx"]
    # FP64: each level the exact sum of its stored pair, n0 = 1 - (n1 + n2 + n3)
    g = plan.populations().reshape(4, -1)[:, gi]
    dg = g - fx["pop_init"]
    do = fx["pop_%d" % cp] - fx["pop_init"]
    scale = np.abs(do).max()
    err = np.abs(dg - do).max()
    _say("  populations: max change %.3e, max |dN_gpu - dN_oracle| %.3e" % (scale, err))
    assert scale > 0
    assert err <= 1e-3 * scale and err <= 1e-6
    assert rel_l2(plan.polarization().reshape(3, -1)[:, gi], fx["pol_%d" % cp]) <= 1e-3
    if "dens_%d" % cp in fx:
        derr = rel_l2(plan.density().reshape(15, -1)[:, gi], fx["dens_%d" % cp])
        _say("  density matrix at sampled gain cells: rel L2 %.3e" % derr)
        assert derr <= 1e-3


def test_slab_full_size_full_length_with_transmission():
    """The slab for femtosecond-pulse transmission (80x80x224, delta 0.05a, 30 fs
    pulse, two flux planes with 100 frequencies every 8 steps, probe, energy) for
    its full 20,000 steps, and the empty slab for the transmission ratio."""
    plan, fx = _run_checkpoints("slab_d05_full", 1e-4)
    probe_err = rel_l2(plan.probe(0), fx["probe0"])
    _say("probe", probe_err)
    assert probe_err <= 1e-4
    assert rel_l2(plan.energy(), fx["energy"]) <= 1e-4
    spec = []
    for f in range(2):
        T, S = plan.flux(f)
        _say("flux", f, rel_l2(T, fx["T%d" % f]), rel_l2(S, fx["S%d" % f]))
        assert rel_l2(T, fx["T%d" % f]) <= 1e-3
        assert rel_l2(S, fx["S%d" % f]) <= 1e-3
        spec.append(S)
    plan.close()
    empty, efx = _run_checkpoints("slab_empty_full", 1e-4, fields=False)
    assert max(efx["norm_20000"]) < 1e-5 * max(fx["norm_20000"])
    Se = empty.flux(0)[1]
    assert rel_l2(empty.flux(0)[0], efx["T0"]) <= 1e-3
    assert rel_l2(Se, efx["S0"]) <= 1e-3
    # the transmission ratio over the pulse's band: the bins where the empty
    # run's spectrum is at least 1e-6 of its peak (outside it the 30 fs pulse
    # carries 1e-14 of its peak power, the rounding floor of either run, while
    # the slab's still-ringing field leaks power there, so the ratio would be
    # leakage over rounding noise)
    band = efx["S0"] >= 1e-6 * efx["S0"].max()
    tr_g, tr_o = spec[0][band] / Se[band], fx["S0"][band] / efx["S0"][band]
    _say("transmission over %d bins" % band.sum(), rel_l2(tr_g, tr_o))
    assert band.sum() >= 20
    assert rel_l2(tr_g, tr_o) <= 1e-3
    empty.close()


@pytest.mark.parametrize("name", ["slab_d00_4k", "slab_d02_4k", "slab_d10_4k"])
def test_slab_full_size_other_disorder_strengths(name):
    plan, fx = _run_checkpoints(name, 1e-4)
    for f in range(2):
        T, S = plan.flux(f)
        assert rel_l2(T, fx["T%d" % f]) <= 1e-3
        assert rel_l2(S, fx["S%d" % f]) <= 1e-3
    assert rel_l2(plan.probe(0), fx["probe0"]) <= 1e-4
    plan.close()


def test_lasing_box_168_at_pump_1e10():
    """The Maxwell-Bloch lasing box (6^3 cells at 24 cells/a, 168^3 with CPML on
    all faces, Lorentz gain voids at 1e24 m^-3, pump 1e10 s^-1, seeded noise) for
    2000 steps: fields, populations and polarization at three checkpoints."""
    plan, fx = _run_checkpoints("lasing168_p1e10", 1e-3)
    assert rel_l2(plan.probe(0), fx["probe0"]) <= 1e-3
    assert rel_l2(plan.energy(), fx["energy"]) <= 1e-3
    plan.close()


def test_lasing_box_168_at_pump_1e7():
    """The same box at the weakest pump of the workload's range, 1e7 s^-1, for
    2000 steps: each step moves the populations by ~3e-10, below half an FP32
    ulp of the ground level, so only the (hi, lo) pairs keep the change, and the
    FP64 readout of the pairs shows it: population changes against the oracle's
    at two checkpoints, with fields, polarization, probe and energy."""
    plan, fx = _run_checkpoints("lasing168_p1e7", 1e-3)
    assert rel_l2(plan.probe(0), fx["probe0"]) <= 1e-3
    assert rel_l2(plan.energy(), fx["energy"]) <= 1e-3
    plan.close()


def test_density_lasing_box_168():
    """The same 168^3 box with the density-matrix dye in the voids (inverted
    start, pump 1e10 s^-1, seeded noise) for 600 steps in the autotuned launch
    shape: fields, the 15 state values, populations and polarization at sampled
    gain cells at two checkpoints; probe and energy."""
    plan, fx = _run_checkpoints("lasing_density168", 1e-3)
    assert rel_l2(plan.probe(0), fx["probe0"]) <= 1e-3
    assert rel_l2(plan.energy(), fx["energy"]) <= 1e-3
    plan.close()


def test_paper_beam_box_200():
    """The paper's linear box (200^3: 8^3 cells of the inverted opal at 16
    cells/a, gamma 0.05, the TEM00 beam, CPML on all faces) for 3,000 steps, as
    the pulse crosses it, in the autotuned launch shape: fields at 1,000 and 3,000
    steps, the probe and T(t) at the output plane."""
    plan, fx = _run_checkpoints("paper_beam_3k", 1e-4)
    probe_err = rel_l2(plan.probe(0), fx["probe0"])
    T_err = rel_l2(plan.flux(0)[0], fx["T0"])
    _say("probe", probe_err, "T(t)", T_err, "peak T", float(np.abs(fx["T0"]).max()))
    assert probe_err <= 1e-4
    assert T_err <= 1e-3
    plan.close()


def test_paper_lasing_box_200():
    """The paper's lasing box (200^3: 8^3 cells of the eps-12 inverted opal at 16
    cells/a, gamma 0.1, the density-matrix dye in the voids, inverted start, pump
    1e10 s^-1, seeded noise) for 400 steps in the autotuned launch shape: fields,
    the 15 state values, populations and polarization at sampled gain cells at two
    checkpoints; probe and energy."""
    plan, fx = _run_checkpoints("paper_lasing_400", 1e-3)
    assert rel_l2(plan.probe(0), fx["probe0"]) <= 1e-3
    assert rel_l2(plan.energy(), fx["energy"]) <= 1e-3
    plan.close()


def test_largest_grid_with_nontemporal_stores():
    """The 320x320x408 grid (2.1 GB of step state) from random fields for 30 steps
    with the field stores forced non-temporal (the form the automatic choice takes
    above four times the Infinity Cache) in the autotuned launch shape."""
    plan, _ = _run_checkpoints("big320_random", 1e-4, tuning_extra={"stores": 2})
    plan.close()
