"""Pins of the oracle's density-matrix gain model (section "Sample and numerical
approach": a ground level coupled to three degenerate upper levels, one per
field component, with decay time T1, dephasing time T2 and a pump).

Each test holds the oracle to something it does not compute itself: closed
forms of free precession and relaxation, an adaptive library ODE solution of
the continuum density-matrix equations (second-order convergence of the
splitting), the spectrum of rho under unitary steps, and the energy that the
coupled field-matter system conserves.  CPU only."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import oracle as O

A_M = 480e-9
T_UNIT = A_M / 299792458.0  # seconds per a/c


def material(**kw):
    # explicit dipole (8e-29 C m, the radiative value for T1 = 1 ns): the tests vary T1
    m = {"eps": 1.69, "gain": 2, "n_total": 5e25, "f_a": 0.7749, "t1": 1.0, "t2": 1.0, "pump": 0.0,
         "noise": 0.0, "n_init": (1.0, 0.0, 0.0, 0.0), "dipole": 8e-29}
    m.update(kw)
    return m


def pure(v):
    v = np.asarray(v, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    return np.outer(v, v.conj())


def hamiltonian(w0, E):
    H = np.zeros((4, 4), dtype=np.complex128)
    for k in range(3):
        H[k + 1, k + 1] = w0
        H[0, k + 1] = H[k + 1, 0] = -E[k]
    return H


def rhs_factory(w0, g1, g2, gp, efield):
    """Continuum equations written from the model's definition."""
    def rhs(t, y):
        r = y.view(np.complex128).reshape(4, 4)
        H = hamiltonian(w0, efield(t))
        d = -1j * (H @ r - r @ H)
        for k in range(1, 4):
            d[k, k] += -g1 * r[k, k] + gp / 3.0 * r[0, 0]
        d[0, 0] += g1 * (r[1, 1] + r[2, 2] + r[3, 3]) - gp * r[0, 0]
        off = ~np.eye(4, dtype=bool)
        d[off] += -g2 * r[off]
        return d.reshape(-1).view(np.float64)
    return rhs


def test_free_precession_is_exact():
    """E = 0 and no relaxation: rho_0k turns by exp(i w0 dt) per step exactly
    (prewarped Cayley step); populations and upper coherences stay put."""
    m = material(t1=1e3, t2=1e3)
    dt, dx = 0.5 / 24, 1.0 / 24
    w0 = 2 * math.pi * m["f_a"]
    r0 = pure([1.0, 0.5 + 0.5j, 1j, -0.7])
    n = 5000
    r = O.bloch_evolve(m, dt, dx, A_M, np.zeros((n, 3)), r0)
    ph = np.exp(1j * w0 * n * dt)
    decay = math.exp(-n * dt * T_UNIT / 1e3)
    for k in range(1, 4):
        assert abs(r[0, k] - r0[0, k] * ph * decay) <= 1e-12
    assert np.allclose(r[1:, 1:], r0[1:, 1:] * np.where(np.eye(3, dtype=bool), 1.0, decay), atol=1e-12, rtol=0)


def test_relaxation_and_pump_closed_forms():
    """E = 0: upper total e(t) = e_inf + (e0 - e_inf) exp(-(P + 1/T1) t), each level's
    excess over e/3 decays as exp(-t/T1), every coherence as exp(-t/T2) (the
    ground-upper ones also turning at w0)."""
    m = material(t1=20e-15, t2=5e-15, pump=1e13)
    dt, dx = 0.5 / 24, 1.0 / 24
    w0 = 2 * math.pi * m["f_a"]
    g1, g2, gp = T_UNIT / 20e-15, T_UNIT / 5e-15, 1e13 * T_UNIT
    r0 = 0.5 * pure([0.3, 1.0, 0.2j, 0.5]) + 0.5 * np.diag([0.1, 0.6, 0.1, 0.2])
    n = 3000
    r, hist = O.bloch_evolve(m, dt, dx, A_M, np.zeros((n, 3)), r0, history=True)
    t = (np.arange(n) + 1) * dt
    e0 = np.trace(r0[1:, 1:]).real
    einf = gp / (gp + g1)
    e = einf + (e0 - einf) * np.exp(-(gp + g1) * t)
    for k in range(1, 4):
        want = e / 3 + (r0[k, k].real - e0 / 3) * np.exp(-g1 * t)
        assert np.max(np.abs(hist[:, k, k].real - want)) <= 1e-12
        want0k = r0[0, k] * np.exp((1j * w0 - g2) * t)
        assert np.max(np.abs(hist[:, 0, k] - want0k)) <= 1e-12
    assert np.max(np.abs(hist[:, 1, 2] - r0[1, 2] * np.exp(-g2 * t))) <= 1e-12
    assert np.max(np.abs(np.trace(hist, axis1=1, axis2=2) - 1.0)) <= 1e-12


@pytest.mark.parametrize("relax", [False, True])
def test_splitting_converges_to_the_continuum_at_second_order(relax):
    """A driven atom (oscillating field along a tilted direction, strong enough to
    move population) against scipy's adaptive solution of the continuum
    equations: the error at t = 12 a/c falls by ~4 per halving of dt."""
    if relax:
        m = material(t1=40e-15, t2=8e-15, pump=2e13)
        g1, g2, gp = T_UNIT / 40e-15, T_UNIT / 8e-15, 2e13 * T_UNIT
    else:
        m = material(t1=1e3, t2=1e3)
        g1 = g2 = T_UNIT / 1e3
        gp = 0.0
    w0 = 2 * math.pi * m["f_a"]
    u = np.array([0.6, -0.48, 0.64])
    efield = lambda t: 1.5 * math.cos(0.9 * w0 * t) * u + np.array([0.0, 0.3, 0.0])
    r0 = np.diag([0.7, 0.1, 0.1, 0.1]).astype(np.complex128)
    T = 12.0
    sol = solve_ivp(rhs_factory(w0, g1, g2, gp, efield), (0.0, T), r0.reshape(-1).view(np.float64),
                    method="DOP853", rtol=1e-12, atol=1e-14)
    exact = sol.y[:, -1].view(np.complex128).reshape(4, 4)
    errs = []
    for n in (600, 1200, 2400):
        dt = T / n
        emid = np.array([efield((q + 0.5) * dt) for q in range(n)])
        r = O.bloch_evolve(m, dt, dt * 2, A_M, emid, r0)
        errs.append(np.max(np.abs(r - exact)))
    assert errs[0] < 5e-3
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_unitary_steps_keep_the_spectrum_and_relaxation_keeps_a_density_matrix():
    rng = np.random.default_rng(3)
    dt, dx = 0.5 / 24, 1.0 / 24
    emid = rng.normal(scale=0.8, size=(2000, 3))
    v = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    r0 = v @ v.conj().T
    r0 /= np.trace(r0).real
    r = O.bloch_evolve(material(t1=1e3, t2=1e3), dt, dx, A_M, emid, r0)
    assert np.allclose(np.linalg.eigvalsh(r), np.linalg.eigvalsh(r0), atol=1e-12, rtol=0)
    r = O.bloch_evolve(material(t1=30e-15, t2=6e-15, pump=5e13), dt, dx, A_M, emid, r0)
    assert np.max(np.abs(r - r.conj().T)) <= 1e-15
    assert abs(np.trace(r) - 1.0) <= 1e-12
    assert np.linalg.eigvalsh(r).min() >= -1e-13


def test_coherent_step_matches_the_propagator_for_a_constant_field():
    """One field direction, no relaxation: after n steps the state equals
    exp(-i H_c t) rho0 exp(+i H_c t) for the Hamiltonian whose Cayley map the step
    is, up to rounding: the Cayley phase 2 atan(lambda dt/2) per eigenvalue
    lambda of the prewarped Hamiltonian."""
    m = material(t1=1e3, t2=1e3)
    dt, dx = 0.5 / 24, 1.0 / 24
    w0 = 2 * math.pi * m["f_a"]
    wp = (2 / dt) * math.tan(w0 * dt / 2)
    E = np.array([0.4, -1.1, 0.7])
    Hp = hamiltonian(wp, E)
    lam, U = np.linalg.eigh(Hp)
    Hc = (U * (2 / dt * np.arctan(lam * dt / 2))) @ U.conj().T
    r0 = pure([1.0, 0.2, 0.0, 0.3j])
    n = 3000
    r = O.bloch_evolve(m, dt, dx, A_M, np.tile(E, (n, 1)), r0)
    Ut = expm(-1j * Hc * n * dt)
    assert np.max(np.abs(r - Ut @ r0 @ Ut.conj().T)) <= 1e-11


def _one_cell(m, res, E0, steps):
    g = {"n": (1, 1, 1), "periodic": (1, 1, 1), "res": res, "courant": 0.5, "a_meters": A_M}
    sim = O.OracleSim({"grid": g, "materials": [m]}, max_steps=steps)
    for c in range(3):
        sim.set_field(c, np.full((1, 1, 1), E0[c]))
    return sim


def test_coupled_cell_conserves_field_plus_matter_energy():
    """A single periodic cell (curl = 0): eps E^2 / 2 + kappa w0 (rho_11 + rho_22 +
    rho_33) is constant for the continuum system; the scheme keeps it to O(dt^2)."""
    m = material(t1=1e3, t2=1e3, n_init=(0.6, 0.3, 0.1, 0.0))
    drift = []
    for res in (24, 48, 96):
        dt = 0.5 / res
        n = int(round(10.0 / dt))
        w0, _, kappa, *_ = O.bloch_constants(m, dt, 1.0 / res, A_M)
        sim = _one_cell(m, res, (0.5, 0.2, -0.3), n)
        W = []
        for _ in range(n):
            E = np.array([sim.field(c)[0, 0, 0] for c in range(3)])
            rho = sim.populations()[:, 0, 0, 0]
            W.append(0.5 * m["eps"] * E @ E + kappa * w0 * rho[1:].sum())
            sim.step(1)
        W = np.array(W)
        drift.append(np.max(np.abs(W - W[0])) / W[0])
    assert drift[0] < 2e-3
    assert 3.5 < drift[0] / drift[1] < 4.5 and 3.5 < drift[1] / drift[2] < 4.5, drift


def test_inverted_cell_gives_energy_to_the_field_and_ground_cell_takes_it():
    m_inv = material(t1=1e3, t2=1e3, n_init=(0.0, 1.0, 0.0, 0.0))
    m_gnd = material(t1=1e3, t2=1e3, n_init=(1.0, 0.0, 0.0, 0.0))
    n = 400
    out = []
    for m in (m_inv, m_gnd):
        sim = _one_cell(m, 24, (0.05, 0.0, 0.0), n)
        sim.step(n)
        out.append((sim.field(0)[0, 0, 0], sim.populations()[1, 0, 0, 0]))
    (e_inv, p_inv), (e_gnd, p_gnd) = out
    # the field amplitude along x is bounded by energy exchange: the inverted atom
    # has lost upper population, the ground one gained some
    assert p_inv < 1.0 - 1e-6 and p_gnd > 1e-6


def _rotation_box(N=12, M=6, src=None, steps=0):
    """Periodic N x N x M box of uniform permittivity 1 (so only the matter can
    break a symmetry) with density-matrix cells forming a plus sign around cell
    (c, c, kc) that a 90-degree turn about that cell's centre maps onto itself."""
    c, kc = N // 2, M // 2
    dye = material(eps=1.0, t1=1e3, t2=1e3, n_init=(0.4, 0.2, 0.2, 0.2))
    mp = np.zeros((M, N, N), np.uint8)
    for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
        mp[kc, c + dj, c + di] = 1
    grid = {"n": (N, N, M), "periodic": (1, 1, 1), "pml_lo": (0, 0, 0), "pml_hi": (0, 0, 0), "res": 16,
            "courant": 0.5, "a_meters": A_M, "seed": 3, "realization": 0}
    cfg = {"name": "rot", "grid": grid, "materials": [{"eps": 1.0}, dye], "map": mp, "sources": [src],
           "probes": [], "flux": [], "energy_interval": 0, "steps": steps}
    return cfg, c, kc


def test_density_matrix_sits_at_the_cell_centre_rotation_isotropy():
    """The density matrix lives at the cell centre (the placement of section
    "Sample and numerical approach"): a gain cell couples to the
    average of the four edges of each field component around its centre and
    hands its polarization change back to them.  Turning the whole setup by 90
    degrees about z through a gain cell's centre, (x, y) -> (2c+1-y, x), maps
    the Yee lattice onto itself (Ex edges onto Ey edges), so the run of the
    turned source must give the turned density matrix: upper levels 1, 2, 3
    transform as the vector (x, y, z) -> (-y, x, z).  Coupling each cell to the
    three edges at its lower corner instead breaks this at first order."""
    steps = 300
    wave = {"f0": 0.78, "width_kind": "fwhm_power", "width": 0.3, "delay": 5.0, "amp": 40.0}
    cfg_a, c_, kc_ = _rotation_box()
    # source A: Ex of cell (c+2, c+1); its image is Ey of cell (2c+1-(c+1), c+2) = (c, c+2)
    cfg_a["sources"] = [dict(wave, kind="dipole", comp=0, i=c_ + 2, j=c_ + 1, k=kc_)]
    cfg_b, _, _ = _rotation_box()
    cfg_b["sources"] = [dict(wave, kind="dipole", comp=1, i=c_, j=c_ + 2, k=kc_)]
    runs = []
    for cfg in (cfg_a, cfg_b):
        sim = O.OracleSim(cfg, max_steps=steps)
        sim.step(steps)
        runs.append((sim.density(), sim.fields()))
    (da, fa), (db, fb) = runs
    scale = np.abs(da[3:9]).max()
    assert scale > 1e-3  # the pulse reached the matter
    for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
        i, j = c_ + di, c_ + dj
        ib, jb = 2 * c_ + 1 - j - 1, i   # the turned cell: centre (i+1/2, j+1/2) -> (2c+1-j-1/2, i+1/2)
        a = da[:, kc_, j, i]
        b = db[:, kc_, jb, ib]
        # populations rho_11, rho_22, rho_33 -> (rho_22, rho_11, rho_33)
        assert np.allclose([b[0], b[1], b[2]], [a[1], a[0], a[2]], rtol=0, atol=1e-10 * scale)
        # ground-upper coherences (rho_01, rho_02, rho_03) -> (-rho_02, rho_01, rho_03), Re (3..5) and Im (6..8)
        for o in (3, 6):
            assert np.allclose([b[o], b[o + 1], b[o + 2]], [-a[o + 1], a[o], a[o + 2]], rtol=0, atol=1e-10 * scale)
    # and the fields: E'_y at the image of an Ex edge equals E_x there
    ex_a = fa[0, kc_]            # Ex(i, j) at (i+1/2, j) -> Ey(2c+1-j, i)
    ey_b = fb[1, kc_]
    N = ex_a.shape[0]
    for j in range(N):
        for i in range(N):
            assert abs(ey_b[i, (2 * c_ + 1 - j) % N] - ex_a[j, i]) <= 1e-10 * np.abs(ex_a).max()


def test_density_matrix_cells_conserve_field_plus_matter_energy_in_a_box():
    """Periodic 6^3 box filled with the dye (no relaxation, pump or noise) from
    random fields: the discrete field energy W^n (eps |E^n|^2 + H^{n-1/2} .
    H^{n+1/2}) / 2 plus the matter energy kappa w0 sum_k rho_kk of every cell,
    times dx^3, is constant to O(dt^2) -- the centre average and the hand-back
    to the edges are adjoint, so the exchange between field and matter balances
    cell by cell."""
    drift = []
    for res in (16, 32):
        m = material(t1=1e3, t2=1e3, n_init=(0.6, 0.3, 0.1, 0.0))
        n = (6, 6, 6)
        rng = np.random.default_rng(11)
        cfg = {"name": "dm_energy", "grid": {"n": n, "periodic": (1, 1, 1), "pml_lo": (0, 0, 0), "pml_hi": (0, 0, 0),
                                             "res": res, "courant": 0.5, "a_meters": A_M, "seed": 1,
                                             "realization": 0},
               "materials": [m], "map": np.zeros(n, np.uint8), "sources": [], "probes": [], "flux": [],
               "energy_interval": 1, "steps": 0}
        dt, dx = 0.5 / res, 1.0 / res
        steps = int(round(4.0 / dt))
        sim = O.OracleSim(cfg, max_steps=steps + 1)
        for c in range(3):
            sim.set_field(c, 0.3 * rng.standard_normal(n))
        w0, _, kappa, *_ = O.bloch_constants(m, dt, dx, A_M)
        tot = []
        for _ in range(steps):
            pops = sim.populations()
            matter = kappa * w0 * pops[1:].sum() * dx ** 3
            sim.step(1)
            tot.append(sim.energy()[-1] + matter)
        tot = np.array(tot)
        drift.append(np.max(np.abs(tot - tot[0])) / tot[0])
    assert drift[0] < 5e-3
    assert 3.0 < drift[0] / drift[1] < 5.0, drift
