"""Host analysis of T(t) and probe records (section "Diffusion constant and
decay times"): each function is pinned to a closed form on synthetic records
(CPU only)."""
import math

import numpy as np
import pytest

from paper_0802_3775_amd import analysis as A


def _pulse_then_tail(t, t_peak, rise, tau, amp=1.0):
    """A smooth rise to a peak at t_peak followed by an exact exponential tail."""
    return np.where(t < t_peak, amp * np.exp(-((t - t_peak) / rise) ** 2), amp * np.exp(-(t - t_peak) / tau))


def test_fit_tau0_recovers_single_exponential():
    dt = 0.03125
    t = A.time_axis(40000, dt)
    for tau in (37.5, 120.0, 410.0):
        T = _pulse_then_tail(t, 200.0, 20.0, tau, amp=3.7)
        tau0, amp, (i0, i1) = A.fit_tau0(t, T)
        assert abs(tau0 - tau) <= 1e-9 * tau
        # the window starts where T first falls to 10% of the peak
        assert T[i0] <= 0.1 * T.max() < T[i0 - 1]
        assert T[i1 - 1] > 1e-5 * T.max()


def test_fit_ignores_the_rise_and_rejects_growth():
    t = A.time_axis(2000, 0.1)
    with pytest.raises(ValueError):
        A.fit_tau0(t, np.exp(t / 50.0))          # no trailing edge
    with pytest.raises(ValueError):
        A.tail_window(np.zeros(10))


def test_diffusion_constant_closed_form_and_units():
    # L = 4 um, tau0 = 1 ps: D = 16e-12 / (pi^2 1e-12) m^2/s
    assert A.diffusion_constant(4e-6, 1e-12) == pytest.approx(16.0 / math.pi ** 2, rel=1e-15)
    # a/c to seconds at a = 480 nm
    assert A.to_seconds(1.0, 480e-9) == pytest.approx(480e-9 / 299792458.0, rel=1e-15)


def test_quadratic_fit_recovers_coefficients_and_zero():
    g = np.linspace(0.0, 0.15, 7)
    D = 14.0 - 19.0 * g - 204.0 * g ** 2
    (d0, d1, d2), g0 = A.quadratic_fit(g, D)
    assert (d0, d1, d2) == pytest.approx((14.0, -19.0, -204.0), rel=1e-10)
    # positive root of 14 - 19 g - 204 g^2
    want = (-19.0 + math.sqrt(19.0 ** 2 + 4 * 204.0 * 14.0)) / (2 * 204.0)
    assert g0 == pytest.approx(want, rel=1e-10)


def test_decay_distribution_recovers_two_components():
    """A tail that is an exact sum of two exponentials whose times are on the
    dictionary is fitted with weight only on those two (to 1e-8 of the total)."""
    taus = np.geomspace(5.0, 2000.0, 40)
    t1, t2 = taus[8], taus[27]
    t = A.time_axis(60000, 0.05)
    tail = lambda tt: 2.0 * np.exp(-tt / t1) + 0.7 * np.exp(-tt / t2)
    t_peak = 100.0
    T = np.where(t < t_peak, tail(0.0) * np.exp(-((t - t_peak) / 10.0) ** 2), tail(t - t_peak))
    g, rel = A.decay_time_distribution(t, T, taus)
    i0, _ = A.tail_window(T)
    # weights are referred to the window start: g_j = w_j exp(-(t_i0 - t_peak)/tau_j)
    dt0 = t[i0] - t_peak
    w = g * np.exp(dt0 / taus)
    assert rel < 1e-10
    assert w[8] == pytest.approx(2.0, rel=1e-6)
    assert w[27] == pytest.approx(0.7, rel=1e-6)
    others = np.delete(w, [8, 27])
    assert others.sum() <= 1e-8 * w.sum()


def test_field_spectrum_peaks_at_the_tone():
    dt = 0.03125
    n = 16384
    f0 = 0.775
    t = np.arange(n) * dt
    f, P = A.field_spectrum(np.sin(2 * math.pi * f0 * t) * np.hanning(n), dt, pad=4)
    assert abs(f[np.argmax(P)] - f0) <= 0.5 / (4 * n * dt) + 1e-12
    # Parseval: sum of |X|^2 over the full spectrum equals n_fft * sum x^2
    x = np.sin(2 * math.pi * f0 * t)
    X = np.fft.fft(x)
    assert np.sum(np.abs(X) ** 2) == pytest.approx(n * np.sum(x ** 2), rel=1e-12)
