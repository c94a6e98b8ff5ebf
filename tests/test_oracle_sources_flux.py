"""Pins of the oracle's sources, absorbing boundary and flux diagnostics (CPU only).

Paper: pulsed plane-wave excitation and the transmitted power T(t), the
Poynting flux through the output plane summed over that plane (section
"Dynamical diffusion and localization"); absorbing walls around the box
(section "Sample and numerical approach").  A 1x1xN periodic column is an
exact 1-D Yee line (x and y differences vanish), which gives closed forms.
"""
import math

import numpy as np
from scipy.signal import hilbert

from oracle import oracle as O
from paper_0802_3775_amd import workloads as W


def _column(Nz, res, src, pml=12, mats=None, mp=None, flux=None, probes=None, steps=0):
    cfg = W.homogeneous_box(n=(1, 1, Nz), periodic=(1, 1, 0), res=res, pml=(0, 0, pml),
                            materials=mats or [{"eps": 1.0}], steps=steps)
    if mp is not None:
        cfg["map"] = mp
    cfg["sources"] = [src]
    cfg["flux"] = flux or []
    cfg["probes"] = probes or []
    return cfg


def _half_crossings(x, y):
    half = y.max() / 2
    idx = np.where(y > half)[0]
    i0, i1 = idx[0], idx[-1]
    lo = x[i0 - 1] + (half - y[i0 - 1]) * (x[i0] - x[i0 - 1]) / (y[i0] - y[i0 - 1])
    hi = x[i1] + (half - y[i1]) * (x[i1 + 1] - x[i1]) / (y[i1 + 1] - y[i1])
    return lo, hi


def test_dipole_waveform_power_spectrum():
    """In a 1x1x1 periodic box every curl vanishes, so Ez accumulates the dipole
    current: Ez^{n+1} - Ez^n = -(dt/dx^2) s(t_{n+1/2}).  The recovered waveform has its
    power spectrum centred on 0.8 c/a with FWHM 0.3 c/a (the configured bandwidth)."""
    res = 32
    cfg = W.homogeneous_box(n=(1, 1, 1), res=res, steps=2000)
    cfg["sources"] = [dict(kind="dipole", comp=2, i=0, j=0, k=0, f0=0.8, width_kind="fwhm_power",
                           width=0.3, delay=6.0, amp=1.0)]
    cfg["probes"] = [(2, 0, 0, 0)]
    sim = O.OracleSim(cfg)
    sim.step(2000)
    p = sim.probe(0)
    dt, dx = sim.dt, 1.0 / res
    s = -np.diff(np.concatenate([[0.0], p])) * dx * dx / dt
    N = 1 << 20
    S = np.abs(np.fft.rfft(s, N)) ** 2
    f = np.fft.rfftfreq(N, dt)
    lo, hi = _half_crossings(f, S)
    assert abs(f[np.argmax(S)] - 0.8) < 2e-4
    assert abs((hi - lo) - 0.3) < 1e-4
    # H never moves in this box
    assert np.all(sim.field(3) == 0) and np.all(sim.field(5) == 0)


def test_plane_waveform_intensity_fwhm():
    """Sheet source in a 1x1x1 box: Ey^{n+1} - Ey^n = -(dt/dx) s(t_{n+1/2}); the
    intensity envelope |analytic signal|^2 has FWHM 30 fs = 18.737 a/c."""
    res = 20
    cfg = W.homogeneous_box(n=(1, 1, 1), res=res, steps=12000)
    cfg["sources"] = [dict(kind="plane", comp=1, k=0, f0=0.8, width_kind="fwhm_intensity",
                           width=W.PULSE_30FS_A_OVER_C, delay=5.0, amp=1.0)]
    cfg["probes"] = [(1, 0, 0, 0)]
    sim = O.OracleSim(cfg)
    sim.step(12000)
    dt, dx = sim.dt, 1.0 / res
    s = -np.diff(np.concatenate([[0.0], sim.probe(0)])) * dx / dt
    t = (np.arange(len(s)) + 0.5) * dt
    lo, hi = _half_crossings(t, np.abs(hilbert(s)) ** 2)
    assert abs((hi - lo) - W.PULSE_30FS_A_OVER_C) < 2e-3 * W.PULSE_30FS_A_OVER_C
    assert abs(0.5 * (lo + hi) - 5.0 * W.PULSE_30FS_A_OVER_C / (2 * math.sqrt(math.log(2)))) < 0.05


def test_sheet_source_radiates_half_each_way():
    """A current sheet K(t) in vacuum radiates E = -K/2 to each side (impedance 1), so
    the time-integrated Poynting flux through a plane on either side is
    (1/4) int K^2 dt per unit area; the discrete value converges at second order."""
    ratios = []
    for res in (20, 40, 80):
        Nz = 24 + 5 * res
        ks = Nz // 2
        L = int(1.25 * res)
        sig = 1.0
        src = dict(kind="plane", comp=1, k=ks, f0=0.8, width_kind="sigma_t", width=sig, delay=5.0, amp=1.0)
        steps = int(50 / (0.5 / res))
        cfg = _column(Nz, res, src, flux=[dict(k=ks + L, freqs=[0.8], decim=1),
                                          dict(k=ks - L, freqs=[0.8], decim=1)], steps=steps)
        sim = O.OracleSim(cfg)
        sim.step(steps)
        fwd, _ = sim.flux(0)
        bwd, _ = sim.flux(1)
        dt, dx = sim.dt, 1.0 / res
        # int sin^2(2 pi f0 t) exp(-t^2/sig^2) dt = (sqrt(pi) sig / 2)(1 - exp(-(2 pi f0 sig)^2))
        want = dx * dx * 0.25 * 0.5 * math.sqrt(math.pi) * sig * (1 - math.exp(-(2 * math.pi * 0.8 * sig) ** 2))
        ratios.append((fwd.sum() * dt / want, -bwd.sum() * dt / want))
    for a, b in ratios:
        assert abs(a - b) < 1e-12
    errs = [abs(a - 1) for a, _ in ratios]
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def _probe_run(Nz, res, ks, kp, steps, pml):
    src = dict(kind="plane", comp=1, k=ks, f0=0.8, width_kind="sigma_t", width=2.0, delay=5.0, amp=1.0)
    sim = O.OracleSim(_column(Nz, res, src, pml=pml, probes=[(1, 0, 0, kp)], steps=steps))
    sim.step(steps)
    return sim


def test_cpml_reflection_below_minus_60_db():
    """Reflection of the CFS-CPML (12 layers, m = 3, default sigma_max) at normal
    incidence, from the difference with a run whose far wall is out of reach within
    the window; [0.6, 1.0] c/a, resolution 20 cells/a."""
    res, pml = 20, 12
    steps = int(150 / (0.5 / res))
    short = _probe_run(pml + 100 + pml, res, pml + 20, pml + 40, steps, pml)
    far = _probe_run(pml + 100 + 4000, res, pml + 20, pml + 40, steps, pml)
    a, b = short.probe(0), far.probe(0)
    N = 1 << 16
    F = np.fft.rfftfreq(N, short.dt)
    R = np.abs(np.fft.rfft(a - b, N)) / np.abs(np.fft.rfft(b, N))
    sel = (F >= 0.6) & (F <= 1.0)
    assert 20 * np.log10(R[sel].max()) < -60.0
    # and the wall does reflect something (the absorber is finite, not a hole)
    assert np.max(np.abs(a - b)) > 0.0


def test_airy_slab_transmission_converges():
    """Homogeneous dielectric slab (n = 2, d = a/2) at normal incidence: the DFT-flux
    transmission ratio P_slab(f)/P_empty(f) approaches the Airy function
    T = 1/(1 + F sin^2(2 pi n d f)), F = 4R/(1-R)^2, R = ((n-1)/(n+1))^2, at second order."""
    n_idx, d = 2.0, 0.5
    errs = []
    freqs = list(np.linspace(0.6, 1.0, 41))
    for res in (40, 80):
        L = int(d * res)
        pml = 12
        Nz = pml + 2 * res + L + 2 * res + pml
        ks, k0 = pml + res // 2, pml + 2 * res
        kt = k0 + L + res
        mp = np.zeros((Nz, 1, 1), np.uint8)
        mp[k0:k0 + L] = 1
        mats = [{"eps": 1.0}, {"eps": n_idx ** 2}]
        steps = int(120 / (0.5 / res))
        src = dict(kind="plane", comp=1, k=ks, f0=0.8, width_kind="sigma_t", width=1.0, delay=5.0, amp=1.0)
        out = []
        for m in (mp, np.zeros_like(mp)):
            sim = O.OracleSim(_column(Nz, res, src, mats=mats, mp=m,
                                      flux=[dict(k=kt, freqs=freqs, decim=4)], steps=steps))
            sim.step(steps)
            out.append(sim.flux(0)[1])
        T = out[0] / out[1]
        R = ((n_idx - 1) / (n_idx + 1)) ** 2
        F = 4 * R / (1 - R) ** 2
        Ta = 1 / (1 + F * np.sin(2 * math.pi * n_idx * d * np.array(freqs)) ** 2)
        errs.append(np.abs(T - Ta).max())
        assert T.min() < 0.7 and T.max() > 0.99   # the fringes are resolved
    assert errs[-1] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def _beam_box(n, res, waist, x0, y0, kind="beam", comp=1, steps=1):
    cfg = W.homogeneous_box(n=(n, n, 6), periodic=(0, 0, 0), res=res, steps=steps)
    cfg["sources"] = [{"kind": kind, "comp": comp, "k": 3, "f0": 0.8, "width_kind": "sigma_t",
                       "width": 2.0, "delay": -0.25, "amp": 1.0, "x0": x0, "y0": y0, "waist": waist}]
    return cfg


def test_beam_weights_gaussian_integral_and_axis():
    """TEM00 sheet (section "Wide-band excitation and gap filling": a linearly
    polarised TEM00 beam of given waist launched along [100]).  After one step from
    rest E = -(dt/dx) dxJ w(i, j) on the source plane, so the ratio to a uniform
    sheet's field is the transverse weight w.  Checks: w = 1 exactly on the beam
    axis at the driven component's own Yee position (Ey sits at (i, j + 1/2)), the
    sampled Gaussian sums to pi waist^2 / dx^2 (Poisson summation: exact to
    rounding once the box holds the tails), and w is mirror-symmetric about the
    axis."""
    res, n = 4, 48
    dx = 1.0 / res
    waist = 3.0 * dx
    x0, y0 = 24 * dx, 20.5 * dx            # Ey of cell (24, 20) sits on the axis
    beam = O.OracleSim(_beam_box(n, res, waist, x0, y0), max_steps=1)
    beam.step(1)
    plane = O.OracleSim(_beam_box(n, res, waist, x0, y0, kind="plane"), max_steps=1)
    plane.step(1)
    eb, ep = beam.fields()[1][3], plane.fields()[1][3]      # Ey on the source plane [y][x]
    assert np.all(ep[1:-1, 1:-1] != 0.0)
    w = np.zeros_like(eb)
    w[1:-1, 1:-1] = eb[1:-1, 1:-1] / ep[1:-1, 1:-1]
    assert w[20, 24] == 1.0
    assert abs(w.sum() - math.pi * waist ** 2 / dx ** 2) <= 1e-12 * w.sum()
    assert np.allclose(w[20, 24 - 5:24], w[20, 24 + 5:24:-1], rtol=0, atol=1e-15)   # x mirror about i = 24
    assert np.allclose(w[20 - 5:20, 24], w[20 + 5:20:-1, 24], rtol=0, atol=1e-15)   # y mirror about j = 20


def test_beam_with_infinite_waist_is_the_plane_sheet():
    """A waist far larger than the box makes every weight exp(-tiny) = 1 in FP64:
    the beam run equals the uniform-sheet run bit for bit after many steps (CPML
    and PEC walls included), for every driven component."""
    for comp in (0, 1, 2):
        cfgs = []
        for kind in ("beam", "plane"):
            c = W.homogeneous_box(n=(10, 12, 30), periodic=(0, 0, 0), res=8, pml=(4, 4, 4), steps=60)
            c["sources"] = [{"kind": kind, "comp": comp, "k": 9, "f0": 0.8, "width_kind": "fwhm_intensity",
                             "width": 1.25, "delay": 5.0, "amp": 1.0, "x0": 0.7, "y0": 0.6, "waist": 1e30}]
            cfgs.append(c)
        a = O.OracleSim(cfgs[0], max_steps=60)
        a.step(60)
        b = O.OracleSim(cfgs[1], max_steps=60)
        b.step(60)
        fa, fb = a.fields(), b.fields()
        assert np.abs(fb).max() > 0
        assert np.array_equal(fa, fb), comp
