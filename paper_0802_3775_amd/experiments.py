"""Runs of the paper's experiments with the stepper.

* diffusion (section "Diffusion constant and decay times"): the dynamic-diffusion
  pulse through the 200^3 box for a set of disorder strengths and realizations,
  T(t) at the output face, the trailing edge fitted by exp(-t/tau0),
  D = L^2 / (pi^2 tau0), and the quadratic D(gamma) fit of Eq. (1);
* spectra (section "Wide-band excitation and gap filling"): the single-cycle
  beam, the field spectrum at a point inside the crystal, averaged over
  realizations, and the depth of its band-gap dip per gamma.

    python -m paper_0802_3775_amd.experiments diffusion --gammas 0 0.05 0.1 0.15 --realizations 2
    python -m paper_0802_3775_amd.experiments spectra --gammas 0 0.02 0.05 0.1 --realizations 2
"""
import argparse
import json
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="?", choices=("diffusion", "spectra"), default="diffusion")
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
    res = diffusion_sweep(args.gammas, args.realizations, tuning=tuning, window_ps=args.window_ps,
                          f_thz=args.f_thz)
    print(json.dumps({k: v for k, v in res.items() if k != "runs"}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
