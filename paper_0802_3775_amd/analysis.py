"""Host analysis of the stepper's diagnostics (section "Diffusion constant and
decay times" and the spectra of section "Wide-band excitation and gap filling").

* tail_window / fit_tau0: the trailing edge of the transmitted power T(t) fitted
  by a single exponential exp(-t/tau0) (least squares on log T over the window).
* diffusion_constant: D = L^2 / (pi^2 tau0) for a sample of thickness L.
* quadratic_fit: D(gamma) ~ d0 + d1 gamma + d2 gamma^2 (the paper's form).
* decay_time_distribution: g(tau) >= 0 minimising the squared difference between
  the trailing edge and sum_tau g(tau) exp(-t/tau) over a dictionary of decay
  times (non-negative least squares).
* field_spectrum: power spectrum of a probe record (the "electromagnetic
  oscillation spectrum" at a point inside the sample).

Times are in units of a/c unless a_meters is given (then seconds); the step
kernels produce T(t) at t_{n+1/2} = (n + 1/2) dt.  Everything here runs on the
host in FP64 and reads only the library's outputs.
"""
import math

import numpy as np
from scipy.optimize import nnls

C0 = 299792458.0


def time_axis(n, dt, half_step=True):
    """t_n (or t_{n+1/2}) for n = 0 .. n-1 in the units of dt."""
    return (np.arange(n, dtype=np.float64) + (0.5 if half_step else 0.0)) * dt


def tail_window(T, hi=0.1, lo=1e-5):
    """Indices [i0, i1) of the trailing edge: after the peak of T, from the first
    sample at or below hi * max(T) to the last sample still above lo * max(T)
    (the reading of "trailing edge" used here; the paper gives no thresholds)."""
    T = np.asarray(T, dtype=np.float64)
    if T.size == 0 or not np.isfinite(T).all():
        raise ValueError("T must be a non-empty finite record")
    ip = int(np.argmax(T))
    tmax = T[ip]
    if not tmax > 0:
        raise ValueError("T has no positive peak")
    after = np.arange(ip, T.size)
    below = after[T[ip:] <= hi * tmax]
    if below.size == 0:
        raise ValueError("T never falls to %g of its peak" % hi)
    i0 = int(below[0])
    above = np.nonzero(T[i0:] > lo * tmax)[0]
    if above.size < 2:
        raise ValueError("trailing edge shorter than two samples above %g of the peak" % lo)
    i1 = i0 + int(above[-1]) + 1
    return i0, i1


def fit_tau0(t, T, window=None):
    """Leading decay time tau0 of the trailing edge: least-squares line through
    (t, log T) over the window (samples with T <= 0 are skipped).  Returns
    (tau0, amplitude at t[i0], window)."""
    t = np.asarray(t, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    i0, i1 = window if window is not None else tail_window(T)
    tt, yy = t[i0:i1], T[i0:i1]
    keep = yy > 0
    tt, yy = tt[keep], np.log(yy[keep])
    if tt.size < 2:
        raise ValueError("not enough positive samples in the window")
    A = np.stack([np.ones_like(tt), tt - tt[0]], axis=1)
    coef, *_ = np.linalg.lstsq(A, yy, rcond=None)
    slope = coef[1]
    if not slope < 0:
        raise ValueError("the trailing edge does not decay")
    return -1.0 / slope, math.exp(coef[0]), (i0, i1)


def diffusion_constant(L, tau0):
    """D = L^2 / (pi^2 tau0) (consistent units: L in m and tau0 in s give m^2/s)."""
    if not (L > 0 and tau0 > 0):
        raise ValueError("L and tau0 must be positive")
    return L * L / (math.pi ** 2 * tau0)


def to_seconds(t_a_over_c, a_meters):
    """Convert times in a/c to seconds for a lattice constant a_meters."""
    return np.asarray(t_a_over_c, dtype=np.float64) * a_meters / C0


def quadratic_fit(gamma, D):
    """Least-squares D(gamma) = d0 + d1 gamma + d2 gamma^2; returns (d0, d1, d2)
    and the smallest positive root of the fitted polynomial (gamma where D = 0;
    nan when there is none)."""
    g = np.asarray(gamma, dtype=np.float64)
    d = np.asarray(D, dtype=np.float64)
    if g.size < 3:
        raise ValueError("a quadratic fit needs at least three points")
    d2, d1, d0 = np.polyfit(g, d, 2)
    roots = np.roots([d2, d1, d0])
    pos = sorted(r.real for r in roots if abs(r.imag) < 1e-12 and r.real > 0)
    return (d0, d1, d2), (pos[0] if pos else float("nan"))


def decay_time_distribution(t, T, taus, window=None):
    """g(tau) >= 0 on the given decay times minimising
    || T(t) - sum_j g_j exp(-(t - t_0) / tau_j) ||^2 over the trailing edge
    (t_0: first time of the window).  Each dictionary column is scaled to unit
    norm for the solve and g is returned in the original scale, with the
    relative residual of the fit."""
    t = np.asarray(t, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    taus = np.asarray(taus, dtype=np.float64)
    if np.any(taus <= 0):
        raise ValueError("decay times must be positive")
    i0, i1 = window if window is not None else tail_window(T)
    tt = t[i0:i1] - t[i0]
    A = np.exp(-tt[:, None] / taus[None, :])
    scale = np.linalg.norm(A, axis=0)
    g_s, res = nnls(A / scale[None, :], T[i0:i1])
    rel = res / max(np.linalg.norm(T[i0:i1]), 1e-300)
    return g_s / scale, rel


def field_spectrum(signal, dt, pad=1):
    """Power spectrum |FFT|^2 of a real record sampled every dt; returns
    (frequencies in 1/(units of dt), power).  pad > 1 zero-pads to pad times the
    length (finer bins, same resolution 1/(n dt))."""
    x = np.asarray(signal, dtype=np.float64)
    n = x.size * max(1, int(pad))
    X = np.fft.rfft(x, n=n)
    f = np.fft.rfftfreq(n, d=dt)
    return f, (X.real ** 2 + X.imag ** 2)
