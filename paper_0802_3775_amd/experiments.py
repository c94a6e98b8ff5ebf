"""Runs of the paper's experiments with the stepper.

* diffusion (section "Diffusion constant and decay times"): the dynamic-diffusion
  pulse through the 200^3 box for a set of disorder strengths and realizations,
  T(t) at the output face, the trailing edge fitted by exp(-t/tau0),
  D = L^2 / (pi^2 tau0), and the quadratic D(gamma) fit of Eq. (1);
* spectra (section "Wide-band excitation and gap filling"): the single-cycle
  beam, the field spectrum at a point inside the crystal, averaged over
  realizations, and the depth of its band-gap dip per gamma;
* lasing (the lasing section): the pumped density-matrix dye in the spheres,
  noise-seeded; emission peak, onset and stored energy density per gamma.

    python -m paper_0802_3775_amd.experiments diffusion --gammas 0 0.05 0.1 0.15 --realizations 2
    python -m paper_0802_3775_amd.experiments spectra --gammas 0 0.02 0.05 0.1 --realizations 2
    python -m paper_0802_3775_amd.experiments lasing --gammas 0 0.1
"""
import argparse
import json
import math
import sys

import numpy as np

from . import analysis as A
from . import workloads as W


def diffusion_run(gamma, realization=0, tuning=None, **kw):
    """One run: T(t) (W per a^2 units of the stepper, at t_{n+1/2}) and its tail fit."""
    import torch
    from . import fdtd
    cfg = W.paper_diffusion(gamma, realization=realization, **kw)
    steps = cfg["steps"]
    plan = fdtd.Plan(cfg, max_steps=steps, tuning=tuning)
    plan.step(steps)
    torch.cuda.synchronize()
    T, _ = plan.flux(0)
    dt = plan.dt
    plan.close()
    t = A.time_axis(len(T), dt)
    a = cfg["grid"]["a_meters"]
    L = cfg["opal"]["cells"][2] * a  # crystal thickness along the beam
    out = {"gamma": gamma, "realization": realization, "steps": steps, "L_m": L}
    try:
        tau0, amp, (i0, i1) = A.fit_tau0(t, T)
        tau_s = float(A.to_seconds(tau0, a))
        out.update(tau0_s=tau_s, D_m2_s=A.diffusion_constant(L, tau_s), window=(int(i0), int(i1)),
                   peak_step=int(np.argmax(T)))
    except ValueError as e:
        out.update(error=str(e))
    return out, T


def diffusion_sweep(gammas, realizations=1, tuning=None, **kw):
    runs = []
    for g in gammas:
        for r in range(realizations):
            res, _ = diffusion_run(g, realization=r, tuning=tuning, **kw)
            print(json.dumps(res), flush=True)
            runs.append(res)
    ok = [r for r in runs if "D_m2_s" in r]
    by_g = {}
    for r in ok:
        by_g.setdefault(r["gamma"], []).append(r["D_m2_s"])
    gam = sorted(by_g)
    D = [float(np.mean(by_g[g])) for g in gam]
    fit = None
    if len(gam) >= 3:
        (d0, d1, d2), zero = A.quadratic_fit(gam, D)
        fit = {"d0": d0, "d1": d1, "d2": d2, "gamma_zero": zero}
    return {"runs": runs, "gamma": gam, "D_mean_m2_s": D, "quadratic_fit": fit}


def spectrum_run(gamma, realization=0, tuning=None, steps=None):
    """The wide-band run of section "Wide-band excitation and gap filling": the
    single-cycle beam through the 200^3 box, the Ey probe inside the crystal, and
    its power spectrum (Hann window over the whole record) on 0.6-1.0 c/a."""
    import torch
    from . import fdtd
    cfg = W.paper_beam(gamma, realization=realization, **({"steps": steps} if steps else {}))
    n = cfg["steps"]
    plan = fdtd.Plan(cfg, max_steps=n, tuning=tuning)
    plan.step(n)
    torch.cuda.synchronize()
    probe = plan.probe(0).astype(np.float64)
    dt = plan.dt
    plan.close()
    f, P = A.field_spectrum(probe * np.hanning(len(probe)), dt)
    band = (f >= 0.6) & (f <= 1.0)
    return f[band], P[band]


def spectrum_sweep(gammas, realizations=1, tuning=None, steps=None, gap=(0.74, 0.84)):
    """Realization-averaged probe spectra per gamma, and how deep the band-gap dip
    is: the spectral power inside `gap` (c/a) against the power of the whole band,
    both from the averaged spectrum."""
    out = []
    for g in gammas:
        acc = None
        for r in range(realizations):
            f, P = spectrum_run(g, realization=r, tuning=tuning, steps=steps)
            acc = P if acc is None else acc + P
        P = acc / realizations
        inside = (f >= gap[0]) & (f <= gap[1])
        row = {"gamma": g, "realizations": realizations,
               "gap_fraction": float(P[inside].sum() / P.sum()),
               "min_freq_c_over_a": float(f[inside][np.argmin(P[inside])]),
               "min_over_median_db": float(10 * np.log10(P[inside].min() / np.median(P)))}
        print(json.dumps(row), flush=True)
        out.append(row)
    return out


EPS0 = 8.8541878128e-12
HBAR = 1.054571817e-34
C0 = 299792458.0


def dye_field_unit(material, a_m):
    """The field unit of the density-matrix medium, hbar c / (mu a) in V/m, with mu
    the material's dipole (or its radiative value from T1, as the library takes it)."""
    mu = material.get("dipole", 0.0)
    if not mu > 0:
        w = 2 * math.pi * material["f_a"] * C0 / a_m
        mu = math.sqrt(3 * math.pi * EPS0 * HBAR * C0 ** 3 / (w ** 3 * math.sqrt(material["eps"]) * material["t1"]))
    return HBAR * C0 / (mu * a_m)


def lasing_run(gamma, realization=0, tuning=None, steps=None):
    """The lasing run of the paper (section on lasing, Fig. 4b and 5): the 200^3 box
    with the density-matrix dye in the spheres, noise-seeded.  Returns the emission
    peak of the probe's spectrum over the second half of the record (argmax on
    0.6-0.9 c/a), the onset (energy first at 1% of its maximum) and the final
    field energy as a mean density over the crystal in fJ/um^3."""
    import torch
    from . import fdtd
    cfg = W.paper_lasing(gamma, realization=realization, **({"steps": steps} if steps else {}))
    n = cfg["steps"]
    plan = fdtd.Plan(cfg, max_steps=n, tuning=tuning)
    plan.step(n)
    torch.cuda.synchronize()
    probe = plan.probe(0).astype(np.float64)
    energy = plan.energy()
    dt = plan.dt
    plan.close()
    a = cfg["grid"]["a_meters"]
    half = probe[len(probe) // 2:]
    f, P = A.field_spectrum(half * np.hanning(len(half)), dt, pad=4)
    band = (f >= 0.6) & (f <= 0.9)
    fpk = float(f[band][np.argmax(P[band])])
    ke = cfg["energy_interval"]
    onset = int(np.argmax(energy >= 0.01 * energy.max())) * ke
    E0 = dye_field_unit(cfg["materials"][1], a)
    w_si = float(energy[-1]) * EPS0 * E0 ** 2 * a ** 3          # J
    vol = (cfg["opal"]["cells"][0] * a) ** 3
    return {"gamma": gamma, "realization": realization, "steps": n,
            "peak_c_over_a": fpk, "peak_thz": fpk * C0 / a / 1e12,
            "onset_ps": float(A.to_seconds(onset * dt, a) * 1e12),
            "energy_density_fJ_um3": w_si / vol * 1e15 / 1e18}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="?", choices=("diffusion", "spectra", "lasing"), default="diffusion")
    ap.add_argument("--gammas", type=float, nargs="+", default=[0.0, 0.05, 0.1, 0.15])
    ap.add_argument("--realizations", type=int, default=1)
    ap.add_argument("--window-ps", type=float, default=2.5)
    ap.add_argument("--f-thz", type=float, default=484.0)
    args = ap.parse_args(argv)
    tuning = {"tile_x": 32, "block": 256, "zchunk": 8, "graph_steps": 200, "max_blocks": 0, "merge": 2,
              "parallel": 0}
    if args.what == "spectra":
        spectrum_sweep(args.gammas, args.realizations, tuning=tuning)
        return
    if args.what == "lasing":
        for g in args.gammas:
            for r in range(args.realizations):
                print(json.dumps(lasing_run(g, realization=r, tuning=tuning)), flush=True)
        return
    res = diffusion_sweep(args.gammas, args.realizations, tuning=tuning, window_ps=args.window_ps,
                          f_thz=args.f_thz)
    print(json.dumps({k: v for k, v in res.items() if k != "runs"}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
