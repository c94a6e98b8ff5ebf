"""Writes the oracle fixtures of the full-size GPU parity tests.

The FP64 oracle takes minutes to hours for the full-size workloads (the slab
for femtosecond-pulse transmission at 80x80x224 for its full 20,000 steps, the
168^3 lasing boxes, the paper's 200^3 beam and lasing boxes, the 320^3 grid),
too long to run beside the GPU inside the test suite.  This script runs them on the CPU once and stores what the tests
compare: every field component at a seeded sample of cells at a few
checkpoints, the transmitted power T(t), the flux spectra, the probe and energy
records, and for gain runs the populations and polarization (and for the
density-matrix medium its 15 state values) at sampled gain cells.  It calls only the oracle and the seeded input generators; nothing here
comes from the GPU path.

    python tests/golden/make_oracle_runs.py [name ...]

Each run writes tests/golden/oracle_<name>.npz.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_0802_3775_amd import workloads as W  # noqa: E402

NSAMP = 4096      # sampled cells per field checkpoint
NGAIN = 2048      # sampled gain cells for populations / polarization
SAMPLE_SEED = 2024


def _pec_clean(fields, periodic):
    """Zero the E components that sit on PEC walls (tangential at index 0)."""
    for c, axes in ((0, (1, 2)), (1, (0, 2)), (2, (0, 1))):
        for a in axes:
            if not periodic[a]:
                sl = [slice(None)] * 3
                sl[2 - a] = 0
                fields[c][tuple(sl)] = 0.0
    return fields


def big_random_cfg():
    """The largest serving grid (10^3 cubic cells at 32 cells/a, 320x320x408,
    z-CPML) from seeded random fields: the grid whose state (2.1 GB) exceeds
    four times the Infinity Cache, where the step kernel stores non-temporally."""
    cfg = W.slab(delta=0.05, seed=4242, res=32, cells=(10, 10, 10), steps=30, nf=0)
    cfg["init_fields"] = _pec_clean(W.random_fields(cfg["grid"]["n"], seed=77), cfg["grid"]["periodic"])
    return cfg


# name -> (config builder, field checkpoints)
RUNS = {
    # the slab for femtosecond-pulse transmission at its full size and length
    "slab_d05_full": (lambda: W.slab(delta=0.05, seed=13, steps=20000, nf=100, decim=8, energy_interval=100),
                      (5000, 10000, 20000)),
    "slab_empty_full": (lambda: W.slab(delta=0.05, seed=13, steps=20000, nf=100, decim=8, empty=True),
                        (20000,)),
    "slab_d00_4k": (lambda: W.slab(delta=0.0, seed=11, steps=4000, nf=100, decim=8), (4000,)),
    "slab_d02_4k": (lambda: W.slab(delta=0.02, seed=12, steps=4000, nf=100, decim=8), (4000,)),
    "slab_d10_4k": (lambda: W.slab(delta=0.10, seed=14, steps=4000, nf=100, decim=8), (4000,)),
    # the Maxwell-Bloch lasing box (Lorentz medium), pump 1e10 s^-1, seeded noise
    "lasing168_p1e10": (lambda: W.lasing(pump=1e10, steps=2000, energy_interval=100), (500, 1000, 2000)),
    # ... at the weakest pump of the workload's range, 1e7 s^-1: per step the
    # populations move ~1e-9, below half an FP32 ulp of the larger levels
    "lasing168_p1e7": (lambda: W.lasing(pump=1e7, steps=2000, energy_interval=100), (1000, 2000)),
    # the same box with the density-matrix dye (inverted start, pump 1e10 s^-1, seeded noise)
    "lasing_density168": (lambda: W.lasing(pump=1e10, steps=600, energy_interval=100, model="density"),
                          (200, 600)),
    # the paper's linear box (200^3, 8^3 cells at 16 cells/a, gamma 0.05, TEM00
    # beam, CPML on all faces) until the pulse has crossed it
    "paper_beam_3k": (lambda: W.paper_beam(0.05, seed=9, steps=3000), (1000, 3000)),
    # the paper's lasing box (200^3, 8^3 cells of inverted opal at 16 cells/a,
    # gamma 0.1, density-matrix dye in the voids, pump 1e10 s^-1, seeded noise)
    "paper_lasing_400": (lambda: W.paper_lasing(0.1, steps=400, energy_interval=100), (100, 400)),
    "big320_random": (big_random_cfg, (30,)),
}


def sample_cells(ncell, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ncell, size=min(n, ncell), replace=False)).astype(np.int64)


def run(name):
    from oracle import oracle as O
    build, checkpoints = RUNS[name]
    cfg = build()
    steps = cfg["steps"]
    assert checkpoints[-1] == steps
    t0 = time.time()
    sim = O.OracleSim(cfg, max_steps=steps)
    ncell = sim.ncell
    out = {"checkpoints": np.array(checkpoints, dtype=np.int64),
           "idx": sample_cells(ncell, NSAMP, SAMPLE_SEED)}
    gain = None
    mats = cfg["materials"]
    if any(m.get("gain") for m in mats):
        gm = np.array([1 if m.get("gain") else 0 for m in mats], dtype=bool)[sim.map.reshape(-1)]
        gcells = np.nonzero(gm)[0]
        rng = np.random.default_rng(SAMPLE_SEED + 1)
        gain = np.sort(rng.choice(gcells, size=min(NGAIN, len(gcells)), replace=False)).astype(np.int64)
        out["gain_idx"] = gain
        out["pop_init"] = sim.populations().reshape(4, -1)[:, gain]
    dm = any(m.get("gain") == 2 for m in mats)
    done = 0
    for cp in checkpoints:
        sim.step(cp - done)
        done = cp
        f = sim.fields().reshape(6, -1)
        out["f_%d" % cp] = f[:, out["idx"]].astype(np.float32)
        out["norm_%d" % cp] = np.array([np.linalg.norm(f[:3]), np.linalg.norm(f[3:])])
        if gain is not None:
            out["pop_%d" % cp] = sim.populations().reshape(4, -1)[:, gain]
            out["pol_%d" % cp] = sim.polarization().reshape(3, -1)[:, gain].astype(np.float32)
            if dm:
                out["dens_%d" % cp] = sim.density().reshape(15, -1)[:, gain]
        print("%s: step %d (%.0f s)" % (name, cp, time.time() - t0), flush=True)
    for p in range(sim.nprobe):
        out["probe%d" % p] = sim.probe(p).astype(np.float32)
    for fl in range(sim.nflux):
        T, S = sim.flux(fl)
        out["T%d" % fl] = T.astype(np.float32)
        out["S%d" % fl] = S
    if cfg.get("energy_interval"):
        out["energy"] = sim.energy()
    out["oracle_threads"] = np.array(O.threads())
    out["oracle_seconds"] = np.array(time.time() - t0)
    path = os.path.join(HERE, "oracle_%s.npz" % name)
    np.savez_compressed(path, **out)
    print("%s: wrote %s (%.0f KB, %.0f s)" % (name, path, os.path.getsize(path) / 1024, time.time() - t0), flush=True)


def load(name):
    """The stored fixture of run name (a dict of arrays)."""
    with np.load(os.path.join(HERE, "oracle_%s.npz" % name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(RUNS)):
        run(nm)
