"""GPU parity of the density-matrix gain medium (section "Sample and numerical
approach": ground level plus three degenerate upper levels, one per field
component) against the FP64 oracle, through the C ABI.

Tolerances: the kernels hold the state in FP32 (populations as FP32 pairs), the
oracle in FP64.  Before the lasing onset (the oracle's energy below 1% of its
maximum) fields and density agree to relative L2 1e-3 (linear growth of rounding
through the coupled dynamics); smooth driven runs without noise to 1e-4.
Every tile class with gain (plain, z-CPML, all-axes CPML) is exercised."""
import numpy as np
import pytest

from gpu_common import emission_peak_bin, field_rel_l2, rel_l2
from oracle import oracle as O
from paper_0802_3775_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _smooth_field(n, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(m) for m in n[::-1]], indexing="ij")
    out = []
    for c in range(3):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        out.append(0.6 * np.cos(2 * np.pi * (k[0] * x / n[0] + k[1] * y / n[1] + k[2] * z / n[2]) + ph))
    return out


def _periodic_gain_box(n=(16, 16, 16), steps=600, noise=0.0, pump=0.0):
    dm = W.density_material(noise=noise, pump=pump, t1=50e-15, t2=10e-15, dipole=8e-29,
                            n_init=(0.4, 0.3, 0.2, 0.1))
    mp = np.zeros(n[::-1], dtype=np.uint8)
    mp[:, :, n[0] // 2:] = 1  # half gain, half background
    return {
        "name": "dm_box", "grid": W._grid(n, (1, 1, 1), 16, seed=5),
        "materials": [{"eps": 2.25}, dm], "map": mp, "sources": [], "probes": [(0, 3, 5, 7)],
        "flux": [], "energy_interval": 20, "steps": steps,
    }


def _both(cfg, steps, chunks, tuning=None, init=None):
    import torch
    from paper_0802_3775_amd import fdtd as F
    orc = O.OracleSim(cfg, max_steps=steps)
    plan = F.Plan(cfg, max_steps=steps, tuning=tuning)
    if init is not None:
        for c, a in enumerate(init):
            orc.set_field(c, a)
            plan.write_field(c, a.astype(np.float32))
    out = []
    done = 0
    for ch in chunks:
        orc.step(ch)
        plan.step(ch)
        torch.cuda.synchronize()
        done += ch
        out.append((done, field_rel_l2(plan.fields(), orc.fields()), plan.density(), orc.density()))
    return orc, plan, out


def test_density_box_smooth_parity():
    """Periodic box, half of it gain, a smooth initial field and no noise: the
    coupled field-matter dynamics (plain gain class)."""
    n = (16, 16, 16)
    cfg = _periodic_gain_box(n, steps=600)
    _say("density box", n)
    orc, plan, out = _both(cfg, 600, [200, 200, 200], tuning={"block": 128, "zchunk": 4, "graph_steps": 0},
                           init=_smooth_field(n, 3))
    gain = orc.map == 1
    for done, ferr, dg, do in out:
        derr = rel_l2(dg[:, gain], do[:, gain])
        _say("step", done, "fields", ferr, "density", derr)
        assert ferr <= 1e-4 and derr <= 1e-4
    assert rel_l2(plan.probe(0), orc.probe(0)) <= 1e-4
    assert rel_l2(plan.polarization()[:, gain], orc.polarization()[:, gain]) <= 1e-4
    # the density matrix stays one: positive with unit trace
    d = out[-1][2][:, gain].astype(np.float64)
    p = d[0:3]
    assert np.all(p >= -1e-6) and np.all(p.sum(axis=0) <= 1.0 + 1e-6)
    plan.close()


@pytest.mark.parametrize("merge", [0, 2])
def test_density_lasing_box_parity(merge):
    """The density-matrix lasing box (crystal flush with a 6-layer CPML on all
    faces, inverted dye in the voids, noise): fields, density and the probe agree
    through the onset; the populations keep their unit sum."""
    steps = 1500
    cfg = W.lasing(model="density", res=10, cells=(2, 2, 2), pml=6, steps=steps, noise=1e-3, pump=1e12,
                   energy_interval=10)
    _say("density lasing", cfg["grid"]["n"], "merge", merge)
    orc, plan, out = _both(cfg, steps, [300] * 5,
                           tuning={"block": 128, "zchunk": 8, "graph_steps": 50, "merge": merge})
    w = orc.energy()
    onset = int(np.argmax(w >= 0.01 * w.max())) * 10
    gain = orc.map == 1
    for done, ferr, dg, do in out:
        derr = rel_l2(dg[:, gain], do[:, gain])
        _say("step", done, "onset", onset, "fields", ferr, "density", derr)
        # the noise is the same counter-based draw on both sides, so the runs stay
        # together past the onset as well; the bound is the one stated up to it
        assert ferr <= 1e-3 and derr <= 1e-3
    assert onset < steps  # the run reaches the onset
    # emission peak of the probe from the onset on: the same bin within one
    qg, fg = emission_peak_bin(plan.probe(0), plan.dt, onset)
    qo, fo = emission_peak_bin(orc.probe(0), orc.dt, onset)
    _say("emission peak", fg, fo)
    assert abs(qg - qo) <= 1
    # rho_00 is not stored on the GPU (1 - the upper populations, so the trace is
    # 1 by construction); the oracle propagates the full 4x4 matrix, so its rho_00
    # is evolved separately: the changes of all four populations agree
    pops = plan.populations().astype(np.float64)[:, gain]
    pops[0] = 1.0 - pops[1:].sum(axis=0)
    opops = orc.populations()[:, gain]
    init = np.array(cfg["materials"][1]["n_init"])[:, None]
    dg, do = pops - init, opops - init
    _say("populations: max change %.3e, max |dN_gpu - dN_oracle| %.3e" % (np.abs(do).max(), np.abs(dg - do).max()))
    assert np.abs(dg - do).max() <= 1e-3 * np.abs(do).max()
    assert np.all(pops >= -1e-4)
    assert plan.energy()[-1] > 10 * plan.energy()[1]  # it lases
    plan.close()


def test_density_slab_zcpml_class():
    """Slab layout (periodic x, y; z-CPML) with dye voids: the z-CPML gain class,
    separate launches per class."""
    steps = 600
    cfg = W.slab(delta=0.05, seed=21, res=12, cells=(2, 2, 2), steps=steps, nf=0, energy_interval=50)
    cfg["materials"] = [cfg["materials"][0], W.density_material(noise=0.0, t1=50e-15, t2=10e-15, dipole=8e-29),
                        {"eps": 1.0}]
    cfg["opal"] = dict(cfg["opal"], mat_out=2)  # margins and CPML stay vacuum
    _say("density slab", cfg["grid"]["n"])
    orc, plan, out = _both(cfg, steps, [300, 300], tuning={"block": 256, "zchunk": 8, "graph_steps": 0, "merge": 0})
    gain = orc.map == 1
    assert gain.any()
    for done, ferr, dg, do in out:
        derr = rel_l2(dg[:, gain], do[:, gain])
        _say("step", done, "fields", ferr, "density", derr)
        assert ferr <= 1e-4 and derr <= 1e-3
    plan.close()


@pytest.mark.parametrize("cache_mb", [0, 1])
def test_density_batch_matches_plain_runs(cache_mb):
    """Two density-matrix lasing boxes stepped as a batch (cache_mb 1: each in a
    member group of its own, stepped through the call before the other) equal
    the same plans stepped alone, bit for bit."""
    import torch
    from paper_0802_3775_amd import fdtd as F
    cfgs = [W.lasing(model="density", res=8, cells=(2, 2, 2), pml=4, steps=200, noise=1e-3, seed=s)
            for s in (1, 2)]
    tune = {"block": 128, "zchunk": 8, "graph_steps": 0, "cache_mb": cache_mb}
    alone = []
    for c in cfgs:
        p = F.Plan(c, max_steps=200, tuning=tune)
        p.step(200)
        alone.append((p.fields(), p.density()))
        p.close()
    plans = [F.Plan(c, max_steps=200, tuning=tune) for c in cfgs]
    b = F.Batch(plans)
    b.step(200)
    torch.cuda.synchronize()
    for p, (f, d) in zip(plans, alone):
        assert np.array_equal(p.fields(), f) and np.array_equal(p.density(), d)
    b.close()
    for p in plans:
        p.close()


def test_paper_lasing_box_reduced_parity():
    """The paper's lasing run at reduced size (4^3 cells at 8 cells/a, eps-12 opal
    with uniform-radius disorder, dye spheres, CPML on all faces, noise-seeded)."""
    steps = 800
    cfg = W.paper_lasing(0.1, seed=5, res=8, cells=4, pml=6, box_um=2.4, steps=steps, noise=1e-3,
                         energy_interval=20)
    _say("paper lasing reduced", cfg["grid"]["n"])
    orc, plan, out = _both(cfg, steps, [400, 400], tuning={"block": 256, "tile_x": 32, "zchunk": 4,
                                                          "graph_steps": 50, "merge": 2})
    gain = orc.map == 1
    assert gain.any()
    for done, ferr, dg, do in out:
        derr = rel_l2(dg[:, gain], do[:, gain])
        _say("step", done, "fields", ferr, "density", derr)
        assert ferr <= 1e-3 and derr <= 1e-3
    assert rel_l2(plan.probe(0), orc.probe(0)) <= 1e-3
    assert rel_l2(plan.energy(), orc.energy()) <= 1e-3
    plan.close()


def test_paper_lasing_box_full_size():
    """The full 200^3 box (8 cells at 16 cells/a, gamma 0.1) in the benchmark's
    launch shape: the dye map bit-exact and 20 noise-driven steps against the
    oracle."""
    steps = 20
    cfg = W.paper_lasing(0.1, seed=5, steps=steps, noise=1e-3, energy_interval=10)
    _say("paper lasing 200^3", cfg["grid"]["n"])
    orc, plan, out = _both(cfg, steps, [steps], tuning={"block": 256, "tile_x": 32, "zchunk": 8,
                                                       "graph_steps": 0, "merge": 2})
    assert np.array_equal(plan.material_map(), orc.map)
    gain = orc.map == 1
    done, ferr, dg, do = out[-1]
    derr = rel_l2(dg[:, gain], do[:, gain])
    _say("step", done, "fields", ferr, "density", derr)
    assert ferr <= 1e-4 and derr <= 1e-4
    plan.close()


def test_density_pec_walls_and_ragged_shape():
    """Gain cells on PEC walls (tangential E held at zero inside the coupled
    update), a ragged 19 x 13 x 11 box, x and y PEC, z periodic."""
    n = (19, 13, 11)
    dm = W.density_material(noise=1e-3, pump=1e12, t1=50e-15, t2=10e-15, dipole=8e-29,
                            n_init=(0.2, 0.3, 0.3, 0.2))
    rng = np.random.default_rng(9)
    mp = (rng.random(n[::-1]) < 0.6).astype(np.uint8)  # scattered gain cells, walls included
    cfg = {"name": "dm_pec", "grid": W._grid(n, (0, 0, 1), 12, seed=3), "materials": [{"eps": 4.0}, dm],
           "map": mp, "sources": [], "probes": [(1, 0, 5, 5), (2, 7, 0, 3), (0, 9, 6, 4)], "flux": [],
           "energy_interval": 10,
           "steps": 400}
    _say("density pec", n)
    orc, plan, out = _both(cfg, 400, [200, 200], tuning={"block": 64, "tile_x": 16, "zchunk": 3, "graph_steps": 0},
                           init=[a * 0.3 for a in _smooth_field(n, 4)])
    gain = orc.map == 1
    for done, ferr, dg, do in out:
        derr = rel_l2(dg[:, gain], do[:, gain])
        _say("step", done, "fields", ferr, "density", derr)
        assert ferr <= 1e-4 and derr <= 1e-4
    E = plan.fields()
    assert np.all(E[1][:, :, 0] == 0) and np.all(E[2][:, :, 0] == 0)  # Ey, Ez on the x = 0 wall
    assert np.all(E[0][:, 0, :] == 0) and np.all(E[2][:, 0, :] == 0)  # Ex, Ez on the y = 0 wall
    for p in range(2):  # on the walls: exactly zero on both sides
        assert not np.any(orc.probe(p)) and not np.any(plan.probe(p))
    assert rel_l2(plan.probe(2), orc.probe(2)) <= 1e-4
    plan.close()
