"""Closed-form pins of the oracle's Yee core (CPU only).

Paper, section "Sample and numerical approach": the method is Yee FDTD
(the paper cites Taflove's textbook).  These tests check the oracle against
the discrete dispersion relation of the Yee scheme, the exact mode solution of
a PEC cavity, the continuum cavity frequencies, and the exact discrete energy
invariant of a lossless box.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0802_3775_amd import workloads as W


def _positions(n, dx):
    """Coordinates of each Yee component's samples, arrays [nz, ny, nx]."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    half = {0: (0.5, 0, 0), 1: (0, 0.5, 0), 2: (0, 0, 0.5)}
    return {c: ((i + half[c][0]) * dx, (j + half[c][1]) * dx, (k + half[c][2]) * dx) for c in range(3)}


def _standing_wave_prediction(K, eps, dt, n):
    """E^n / E^0 for a discrete eigenmode started with H^{-1/2} = 0.

    Leapfrog on one mode: e_{n+1} - 2 e_n + e_{n-1} = -4 sin^2(theta/2) e_n with
    sin(theta/2) = (dt/2)|K|/sqrt(eps) (discrete dispersion), e_0 = 1, e_1 = 1 - 4 sin^2(theta/2):
    e_n = cos((n + 1/2) theta) / cos(theta / 2).
    """
    s = dt * np.linalg.norm(K) / (2.0 * math.sqrt(eps))
    theta = 2.0 * math.asin(s)
    return math.cos((n + 0.5) * theta) / math.cos(theta / 2.0), theta


def _discrete_K(kvec, dx):
    return np.array([2.0 / dx * math.sin(kd * dx / 2.0) for kd in kvec])


@pytest.mark.parametrize("eps", [1.0, 2.5])
def test_periodic_standing_wave_dispersion(eps):
    n = (12, 10, 8)
    res = 16
    dx = 1.0 / res
    cfg = W.homogeneous_box(n=n, res=res, eps=eps, steps=700)
    sim = O.OracleSim(cfg)
    dt = sim.dt
    m = (1, 2, -1)
    kvec = [2 * math.pi * m[d] / (n[d] * dx) for d in range(3)]
    K = _discrete_K(kvec, dx)
    E0 = np.cross(K, [0.3, -0.5, 0.8])
    E0 /= np.linalg.norm(E0)
    assert abs(np.dot(K, E0)) < 1e-12 * np.linalg.norm(K)
    pos = _positions(n, dx)
    init = [E0[c] * np.cos(kvec[0] * pos[c][0] + kvec[1] * pos[c][1] + kvec[2] * pos[c][2]) for c in range(3)]
    for c in range(3):
        sim.set_field(c, init[c])
    done = 0
    for target in (1, 2, 57, 700):
        sim.step(target - done)
        done = target
        ratio, theta = _standing_wave_prediction(K, eps, dt, done)
        for c in range(3):
            err = np.max(np.abs(sim.field(c) - ratio * init[c]))
            assert err < 1e-11, (c, done, err)
    # the measured frequency is the discrete one, not the continuum one
    f_cont = np.linalg.norm(kvec) / (2 * math.pi * math.sqrt(eps))
    f_disc = theta / (2 * math.pi * dt)
    assert abs(f_disc - f_cont) / f_cont > 1e-4


def _pec_mode(n, res, m, pol):
    dx = 1.0 / res
    L = [n[d] * dx for d in range(3)]
    kvec = [m[d] * math.pi / L[d] for d in range(3)]
    K = _discrete_K(kvec, dx)
    E0 = np.cross(K, pol)
    E0 /= np.linalg.norm(E0)
    pos = _positions(n, dx)
    f = []
    for c in range(3):
        x, y, z = pos[c]
        tx = np.cos(kvec[0] * x) if c == 0 else np.sin(kvec[0] * x)
        ty = np.cos(kvec[1] * y) if c == 1 else np.sin(kvec[1] * y)
        tz = np.cos(kvec[2] * z) if c == 2 else np.sin(kvec[2] * z)
        f.append(E0[c] * tx * ty * tz)
    return f, K, kvec


def test_pec_cavity_mode_exact():
    n = (10, 12, 14)
    res = 10
    cfg = W.homogeneous_box(n=n, periodic=(0, 0, 0), res=res, eps=1.0, steps=900)
    sim = O.OracleSim(cfg)
    init, K, _ = _pec_mode(n, res, (1, 2, 3), [0.2, 0.7, -0.4])
    for c in range(3):
        sim.set_field(c, init[c])
    sim.step(900)
    ratio, _ = _standing_wave_prediction(K, 1.0, sim.dt, 900)
    for c in range(3):
        assert np.max(np.abs(sim.field(c) - ratio * init[c])) < 1e-11
    # the walls stay field-free: tangential E at index 0 on every axis
    ex, ey, ez = (sim.field(c) for c in range(3))
    assert np.all(ex[:, 0, :] == 0) and np.all(ex[0, :, :] == 0)
    assert np.all(ey[:, :, 0] == 0) and np.all(ey[0, :, :] == 0)
    assert np.all(ez[:, :, 0] == 0) and np.all(ez[:, 0, :] == 0)


def test_pec_cavity_frequency_converges_to_continuum():
    # continuum TE/TM mode of a cube of side L: f = (1/(2L)) sqrt(m^2 + n^2 + p^2)
    m = (1, 1, 2)
    L = 1.0
    f_cont = math.sqrt(sum(v * v for v in m)) / (2 * L)
    errs = []
    for res in (8, 16, 32):
        dx = 1.0 / res
        dt = 0.5 * dx
        K = _discrete_K([m[d] * math.pi / L for d in range(3)], dx)
        _, theta = _standing_wave_prediction(K, 1.0, dt, 0)
        errs.append(abs(theta / (2 * math.pi * dt) - f_cont) / f_cont)
    # second-order convergence in dx (at fixed Courant number)
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    # and the oracle rings at the discrete frequency of this mode at res 8
    n = (8, 8, 16)
    cfg = W.homogeneous_box(n=n, periodic=(0, 0, 0), res=8, eps=1.0, steps=400)
    sim = O.OracleSim(cfg)
    init, K, _ = _pec_mode(n, 8, (1, 1, 4), [1.0, -0.3, 0.2])   # same physical mode, L_z = 2
    for c in range(3):
        sim.set_field(c, init[c])
    sim.step(400)
    ratio, _ = _standing_wave_prediction(K, 1.0, sim.dt, 400)
    assert np.max(np.abs(sim.field(0) - ratio * init[0])) < 1e-11


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0), (1, 0, 1)])
def test_discrete_energy_invariant(periodic):
    """W^n = 1/2 sum (eps |E^n|^2 + H^{n-1/2}.H^{n+1/2}) dx^3 is exactly conserved by
    the Yee scheme in a closed lossless box, for any permittivity map (curl-H is the
    adjoint of curl-E on the staggered grid)."""
    n = (9, 8, 7)
    cfg = W.homogeneous_box(n=n, periodic=periodic, res=12, steps=600,
                            materials=[{"eps": 1.0}, {"eps": 2.5}, {"eps": 11.9}])
    cfg["map"] = W.random_map(n, 3, seed=5)
    cfg["energy_interval"] = 1
    sim = O.OracleSim(cfg)
    f = W.random_fields(n, seed=9)
    # tangential E on PEC walls is zero by definition
    for c, axes in ((0, (1, 2)), (1, (0, 2)), (2, (0, 1))):
        for a in axes:
            if not periodic[a]:
                sl = [slice(None)] * 3
                sl[2 - a] = 0
                f[c][tuple(sl)] = 0.0
    for c in range(6):
        sim.set_field(c, f[c])
    sim.step(600)
    w = sim.energy()
    assert len(w) == 600
    assert np.max(np.abs(w - w[0])) / abs(w[0]) < 1e-12
    # a plainly wrong scheme would not conserve it: flip the sign of H and the
    # energy identity must still hold (it is quadratic), but a drift of the fields
    # themselves shows the evolution is non-trivial
    assert np.max(np.abs(sim.field(0) - f[0])) > 1e-2
