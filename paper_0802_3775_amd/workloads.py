"""Seeded synthetic workloads: plain configuration dicts shared by the GPU
library's tests and benchmark and by the CPU oracle.

This module only lays out inputs (grid sizes, seeds, material parameters,
source and probe placement, random initial fields).  It holds none of the
method's arithmetic: coefficients, time steps, CPML profiles, waveforms and
geometry all live on each side of the comparison separately.

Paper context (arXiv:0802.3775, section "Sample and numerical approach"):
inverted opal with eps_r = 12 (here 11.9), lattice constant a = 480 nm, air
spheres at fcc sites, r0 = a/(2 sqrt 2) (here 0.35 a), 200^3 grids, 10^5 steps;
a Rhodamine-like gain medium (n = 1.3) fills the spheres for the lasing runs.

Config dict schema::

    {"grid": {"n": (nx, ny, nz), "periodic": (px, py, pz), "pml_lo": (..), "pml_hi": (..),
              "cpml": {"m", "sigma_max", "kappa_max", "alpha_max"},
              "res": cells per a, "courant": dt/dx, "a_meters": .., "seed": .., "realization": ..},
     "materials": [{"eps": .., "gain": 0/1, "n_total", "tau32", "tau21", "tau10", "pump",
                    "f_a", "df_a", "noise", "n_init"}, ...],
     "opal": {"cells", "origin", "r0", "disorder": none|uniform|gauss, "strength",
              "mat_bg", "mat_void", "mat_out"} or None,
     "map": optional uint8 [nz, ny, nx],
     "sources": [{"kind": dipole|plane|beam, "comp", "i", "j", "k", "f0",
                  "width_kind": fwhm_power|fwhm_intensity|sigma_t, "width", "delay", "amp",
                  "x0", "y0", "waist" (beam: axis and waist, units of a)}],
     "probes": [(comp, i, j, k)], "flux": [{"k", "freqs", "decim"}],
     "energy_interval": int, "steps": int, "init_fields": {comp: array}}
"""
import numpy as np

A_METERS = 480e-9                      # lattice constant, paper value
PULSE_30FS_A_OVER_C = 18.737028625     # 30 fs in units of a/c at a = 480 nm
ALPHA_MAX = 0.3141592653589793         # CPML alpha_max = 2 pi * 0.05 (c/a)
CPML = {"m": 3.0, "sigma_max": -1.0, "kappa_max": 1.0, "alpha_max": ALPHA_MAX}
EPS_BG = 11.9
EPS_DYE = 1.69                         # n = 1.3 dye in the voids
PML = 12

FLUX_FREQS = tuple(float(f) for f in np.linspace(0.6, 1.0, 100))


def gain_material(pump=1e10, noise=1e-6, n_total=1e24, n_init=(1.0, 0.0, 0.0, 0.0),
                  tau32=1e-13, tau21=1e-9, tau10=1e-13, f_a=0.75, df_a=0.02, eps=EPS_DYE):
    return {"eps": eps, "gain": 1, "n_total": n_total, "tau32": tau32, "tau21": tau21,
            "tau10": tau10, "pump": pump, "f_a": f_a, "df_a": df_a, "noise": noise,
            "n_init": tuple(n_init)}


def density_material(pump=0.0, noise=1e-6, n_total=5e25, n_init=(0.0, 1 / 3, 1 / 3, 1 / 3), t1=1e-9,
                     t2=10e-15, f_a=0.7749, dipole=0.0, eps=EPS_DYE):
    """The paper's density-matrix dye (section "Sample and numerical approach"):
    484 THz (0.7749 c/a at a = 480 nm), T1 = 1 ns, T2 = 10 fs, n = 1.3 host, and
    the lasing section's N_a = 5e25 m^-3 of molecules, inverted at the start and
    spread evenly over the three upper levels (the reading of "inversion N_a")."""
    return {"eps": eps, "gain": 2, "n_total": n_total, "f_a": f_a, "t1": t1, "t2": t2, "pump": pump,
            "dipole": dipole, "noise": noise, "n_init": tuple(n_init)}


def _grid(n, periodic, res, pml=(0, 0, 0), seed=0, realization=0, courant=0.5):
    lo = tuple(p if not per else 0 for p, per in zip(pml, periodic))
    return {"n": tuple(int(v) for v in n), "periodic": tuple(int(v) for v in periodic),
            "pml_lo": lo, "pml_hi": lo, "cpml": dict(CPML), "res": int(res),
            "courant": courant, "a_meters": A_METERS, "seed": int(seed),
            "realization": int(realization)}


def periodic_cell(res=32, seed=1, steps=2000, cells=1):
    """One cubic fcc cell of the inverted opal, periodic box, Ez dipole at a seeded
    random cell (centre 0.8 c/a, power-spectrum FWHM 0.3 c/a), Ez probe at a second
    seeded cell."""
    n = cells * res
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, 3)
    prb = src
    while np.array_equal(prb, src):
        prb = rng.integers(0, n, 3)
    return {
        "name": "periodic_cell_%d" % n,
        "grid": _grid((n, n, n), (1, 1, 1), res, seed=seed),
        "materials": [{"eps": EPS_BG}, {"eps": 1.0}],
        "opal": {"cells": (cells,) * 3, "origin": (0, 0, 0), "r0": 0.35, "disorder": "none",
                 "strength": 0.0, "mat_bg": 0, "mat_void": 1, "mat_out": 1},
        "sources": [{"kind": "dipole", "comp": 2, "i": int(src[0]), "j": int(src[1]),
                     "k": int(src[2]), "f0": 0.8, "width_kind": "fwhm_power", "width": 0.3,
                     "delay": 6.0, "amp": 1.0}],
        "probes": [(2, int(prb[0]), int(prb[1]), int(prb[2]))],
        "flux": [],
        "energy_interval": 0,
        "steps": steps,
    }


def slab(delta=0.05, seed=11, res=20, cells=(4, 4, 8), steps=20000, nf=100, decim=8,
         energy_interval=0, empty=False, realization=0, margin_cells=None, pml=PML):
    """Disordered inverted-opal slab for pulse transmission: periodic x, y; along z
    CPML | vacuum margin (1 a) | crystal | vacuum margin | CPML.  Ey plane-wave pulse
    (30 fs intensity FWHM, 0.8 c/a) launched from the middle of the front margin;
    transmission plane in the middle of the back margin; reflection plane between
    the source and the front CPML; Ey probe at a seeded point inside the crystal."""
    nx, ny = cells[0] * res, cells[1] * res
    margin = res if margin_cells is None else margin_cells
    ncz = cells[2] * res
    nz = 2 * pml + 2 * margin + ncz
    z0 = pml + margin
    k_src = pml + margin // 2
    k_tr = z0 + ncz + margin // 2
    k_ref = pml + max(1, margin // 4)
    rng = np.random.default_rng(seed + 7919)
    pi_, pj_, pk_ = rng.integers(0, nx), rng.integers(0, ny), z0 + rng.integers(0, ncz)
    freqs = tuple(float(f) for f in np.linspace(0.6, 1.0, nf)) if nf > 0 else ()
    return {
        "name": "slab_%dx%dx%d_R%d_d%.3f%s" % (cells + (res, delta, "_empty" if empty else "")),
        "grid": _grid((nx, ny, nz), (1, 1, 0), res, pml=(0, 0, pml), seed=seed,
                      realization=realization),
        "materials": [{"eps": EPS_BG}, {"eps": 1.0}],
        "opal": None if empty else {
            "cells": tuple(cells), "origin": (0, 0, z0), "r0": 0.35,
            "disorder": "gauss" if delta > 0 else "none", "strength": float(delta),
            "mat_bg": 0, "mat_void": 1, "mat_out": 1},
        "map": np.ones((nz, ny, nx), dtype=np.uint8) if empty else None,
        "sources": [{"kind": "plane", "comp": 1, "k": int(k_src), "f0": 0.8,
                     "width_kind": "fwhm_intensity", "width": PULSE_30FS_A_OVER_C,
                     "delay": 5.0, "amp": 1.0}],
        "probes": [(1, int(pi_), int(pj_), int(pk_))],
        "flux": ([{"k": int(k_tr), "freqs": freqs, "decim": decim},
                  {"k": int(k_ref), "freqs": freqs, "decim": decim}] if nf > 0 else []),
        "energy_interval": energy_interval,
        "steps": steps,
        "layout": {"z0": z0, "k_src": k_src, "k_tr": k_tr, "k_ref": k_ref},
    }


C_OVER_A_THZ = 299792458.0 / A_METERS / 1e12   # 1 c/a in THz (624.57 at a = 480 nm)


def paper_beam(gamma=0.0, seed=31, res=16, cells=8, margin=None, pml=PML, steps=58000, realization=0,
               eps=12.0, waist_um=2.0, f_thz=484.0, nf=0, box_um=6.0):
    """The paper's linear workload: a box of (cells a + 2 margins + 2 CPML) per
    axis (6 um = 200 cells at 16 cells/a for the defaults: 8 cubic cells of
    inverted opal, 36-cell margins, 12-cell CPML on all faces), eps 12 background,
    air spheres r0 = a/(2 sqrt 2) with uniform-radius disorder r0 (1 + gamma xi);
    a linearly polarised (Ey) single-cycle TEM00 beam (waist 2 um, 484 THz,
    intensity FWHM one period) launched along z ([100]) from the middle of the
    front margin, axis at the box centre; an Ey probe at a seeded low-symmetry
    point inside the crystal; T(t) through the middle of the back margin."""
    if margin is None:  # fill a box of box_um (6 um: 200 cells at 16 cells/a)
        margin = max(1, (int(round(box_um * 1e-6 / A_METERS * res)) - 2 * pml - cells * res) // 2)
    n = cells * res + 2 * margin + 2 * pml
    z0 = pml + margin
    k_src = pml + margin // 2
    k_tr = z0 + cells * res + margin // 2
    f0 = f_thz / C_OVER_A_THZ
    rng = np.random.default_rng(seed + 104729)
    lo, hi = z0 + 1, z0 + cells * res - 1
    pi_, pj_, pk_ = (int(v) for v in rng.integers(lo, hi, size=3))
    centre = 0.5 * n / res
    return {
        "name": "beam_%d^3_R%d_g%.3f" % (n, res, gamma),
        "grid": _grid((n, n, n), (0, 0, 0), res, pml=(pml, pml, pml), seed=seed, realization=realization),
        "materials": [{"eps": float(eps)}, {"eps": 1.0}],
        "opal": {"cells": (cells, cells, cells), "origin": (z0, z0, z0), "r0": 1.0 / (2.0 * np.sqrt(2.0)),
                 "disorder": "uniform" if gamma > 0 else "none", "strength": float(gamma),
                 "mat_bg": 0, "mat_void": 1, "mat_out": 1},
        "map": None,
        "sources": [{"kind": "beam", "comp": 1, "k": int(k_src), "f0": f0, "width_kind": "fwhm_intensity",
                     "width": 1.0 / f0, "delay": 5.0, "amp": 1.0,
                     "x0": centre, "y0": centre, "waist": waist_um * 1e-6 / A_METERS}],
        "probes": [(1, pi_, pj_, pk_)],
        "flux": [{"k": int(k_tr), "freqs": tuple(float(f) for f in np.linspace(0.6, 1.0, nf)) if nf else (),
                  "decim": 8}],
        "energy_interval": 0,
        "steps": steps,
        "layout": {"z0": z0, "k_src": k_src, "k_tr": k_tr, "f0": f0},
    }


def paper_diffusion(gamma=0.0, seed=31, res=16, cells=8, pml=PML, realization=0, f_thz=484.0, fwhm_fs=100.0,
                    window_ps=2.5, box_um=6.0):
    """The paper's dynamic-diffusion run (section "Dynamical diffusion and
    localization"): the box and beam of paper_beam, but a 100 fs Gaussian pulse
    (intensity FWHM) inside the gap near its upper edge -- read as the 484 THz at
    which the paper finds the localized state, just below the 490 THz band-edge
    mode it attributes to the pulse's high-frequency tail -- and T(t) recorded at
    the back margin for window_ps after launch (steps from the Courant-0.5 dt)."""
    steps = int(round(window_ps * 1e-12 / (A_METERS / 299792458.0) / (0.5 / res)))
    cfg = paper_beam(gamma, seed=seed, res=res, cells=cells, pml=pml, steps=steps, realization=realization,
                     f_thz=f_thz, box_um=box_um)
    cfg["name"] = cfg["name"].replace("beam", "diffusion")
    fwhm = fwhm_fs * 1e-15 / (A_METERS / 299792458.0)  # a/c
    cfg["sources"][0] = dict(cfg["sources"][0], width=fwhm, delay=5.0)
    return cfg


def paper_lasing(gamma=0.0, seed=37, res=16, cells=8, pml=PML, steps=59960, realization=0, pump=1e10,
                 noise=1e-6, energy_interval=100, box_um=6.0, **dye):
    """The paper's lasing run (lasing section): the box of paper_beam (6 um,
    200^3 at 16 cells/a, 8 cubic cells of eps-12 inverted opal with uniform-radius
    disorder gamma, CPML on all faces) with the spheres filled by the
    density-matrix dye of density_material (N_a = 5e25 m^-3 inverted at the
    start, pumped), no launched pulse: the emission starts from the noise.  An Ez
    probe at a seeded cell inside the crystal records the oscillation; the
    energy every energy_interval steps.  3 ps is 59,960 steps at Courant 0.5."""
    cfg = paper_beam(gamma, seed=seed, res=res, cells=cells, pml=pml, steps=steps, realization=realization,
                     box_um=box_um)
    cfg["name"] = cfg["name"].replace("beam", "lasing")
    cfg["materials"] = [cfg["materials"][0], density_material(pump=pump, noise=noise, **dye), {"eps": 1.0}]
    cfg["opal"] = dict(cfg["opal"], mat_out=2)  # margins and CPML stay vacuum, the dye fills the spheres
    cfg["sources"] = []
    cfg["probes"] = [(2,) + tuple(cfg["probes"][0][1:])]
    cfg["flux"] = []
    cfg["energy_interval"] = energy_interval
    return cfg


def ensemble(count=64, seed0=1000, steps=10000, max_cells=1_400_000, n_range=(4, 6),
             res_range=(16, 24)):
    """Uneven disorder realizations: delta ~ U[0, 0.12] a, n^3 cubic cells with
    n in {4, 5, 6} and res in {16..24}, redrawn while (n res)^3 exceeds max_cells;
    slab layout (vacuum margins, z-CPML), same pulse in physical time."""
    if (n_range[0] * res_range[0]) ** 3 > max_cells:
        raise ValueError("no (n, res) pair fits max_cells")
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        delta = float(rng.uniform(0.0, 0.12))
        while True:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            res = int(rng.integers(res_range[0], res_range[1] + 1))
            if (n * res) ** 3 <= max_cells:
                break
        c = slab(delta=delta, seed=seed0 + i, res=res, cells=(n, n, n), steps=steps)
        c["name"] = "ens%02d_n%d_R%d_d%.3f" % (i, n, res, delta)
        out.append(c)
    return out


def lasing(pump=1e10, delta=0.05, seed=7, res=24, cells=(6, 6, 6), steps=100000, noise=1e-6,
           n_init=None, energy_interval=100, pml=PML, tau21=1e-9, model="lorentz", **gain_kw):
    """Maxwell-Bloch lasing box: the crystal flush with a CPML on all six faces, gain
    medium in the voids, vacuum in the PML, seeded noise, Ez probe at a seeded cell
    inside the crystal, energy every energy_interval steps.  model: "lorentz"
    (Lorentz polarization + rate equations; n_init defaults to the ground state) or
    "density" (the density-matrix medium of density_material; n_init defaults to
    its inverted start)."""
    n = [c * res + 2 * pml for c in cells]
    rng = np.random.default_rng(seed + 104729)
    p = [int(pml + rng.integers(0, c * res)) for c in cells]
    if model == "density":
        gm = density_material(pump=pump, noise=noise, **gain_kw, **({"n_init": n_init} if n_init else {}))
    else:
        gm = gain_material(pump=pump, noise=noise, n_init=n_init or (1.0, 0.0, 0.0, 0.0), tau21=tau21, **gain_kw)
    return {
        "name": "lasing%s_%dx%dx%d_R%d_P%.0e" % ((("_dm" if model == "density" else ""),) + tuple(cells) + (res, pump)),
        "grid": _grid(n, (0, 0, 0), res, pml=(pml, pml, pml), seed=seed),
        "materials": [{"eps": EPS_BG}, gm, {"eps": 1.0}],
        "opal": {"cells": tuple(cells), "origin": (pml, pml, pml), "r0": 0.35,
                 "disorder": "gauss" if delta > 0 else "none", "strength": float(delta),
                 "mat_bg": 0, "mat_void": 1, "mat_out": 2},
        "sources": [],
        "probes": [(2, p[0], p[1], p[2])],
        "flux": [],
        "energy_interval": energy_interval,
        "steps": steps,
    }


def serving_trace(count=200, seed=42, rho=0.9, capacity_per_s=1.0, linear_frac=0.7,
                  n_range=(4, 10), res_range=(16, 32), cell_range=(1_000_000, 33_000_000),
                  linear_steps=10000, lasing_steps=20000):
    """Poisson stream of mixed requests: (arrival_s, kind, n, res, delta, seed, steps).
    Arrival rate = rho * capacity_per_s requests per second."""
    rng = np.random.default_rng(seed)
    pairs = [(n, r) for n in range(n_range[0], n_range[1] + 1)
             for r in range(res_range[0], res_range[1] + 1)
             if cell_range[0] <= (n * r) ** 3 <= cell_range[1]]
    t = 0.0
    reqs = []
    for q in range(count):
        t += float(rng.exponential(1.0 / (rho * capacity_per_s)))
        n, r = pairs[int(rng.integers(0, len(pairs)))]
        kind = "linear" if rng.uniform() < linear_frac else "lasing"
        reqs.append({"id": q, "arrival": t, "kind": kind, "n": n, "res": r,
                     "delta": float(rng.uniform(0.0, 0.12)), "seed": int(seed * 1000 + q),
                     "steps": linear_steps if kind == "linear" else lasing_steps})
    return reqs


def homogeneous_box(n=(8, 8, 8), periodic=(1, 1, 1), res=16, eps=1.0, pml=(0, 0, 0), seed=0,
                    materials=None, steps=100):
    """Uniform medium (material 0 everywhere), no sources: for closed-form checks."""
    nx, ny, nz = n
    return {
        "name": "box_%dx%dx%d" % n,
        "grid": _grid(n, periodic, res, pml=pml, seed=seed),
        "materials": materials if materials is not None else [{"eps": eps}],
        "opal": None,
        "map": np.zeros((nz, ny, nx), dtype=np.uint8),
        "sources": [], "probes": [], "flux": [], "energy_interval": 0, "steps": steps,
    }


def random_map(n, nmat, seed):
    nx, ny, nz = n
    return np.random.default_rng(seed).integers(0, nmat, (nz, ny, nx)).astype(np.uint8)


def random_fields(n, seed, scale=1.0):
    """Six random field arrays (Ex..Hz), [nz, ny, nx], normal with std `scale`."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return {c: scale * rng.standard_normal((nz, ny, nx)) for c in range(6)}
