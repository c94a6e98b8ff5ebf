"""Values the paper prints, held in tests/golden/ with their citations, against
the host analysis, the workload builders and the oracle's unit conversions
(CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_0802_3775_amd import analysis as A
from paper_0802_3775_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C0 = 299792458.0


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_eq1_quadratic_fit_and_its_zero():
    """Eq. (1): D = 14 - 19 gamma - 204 gamma^2 (m^2/s) vanishes near gamma = 0.2.
    The fit over gamma in [0, 0.15] (the paper's sweep range) returns the printed
    coefficients, and its zero rounds to the printed value."""
    g = _load("eq1_diffusion_fit.json")
    gam = np.linspace(0.0, 0.15, 7)
    D = g["d0"] + g["d1"] * gam + g["d2"] * gam ** 2
    (d0, d1, d2), zero = A.quadratic_fit(gam, D)
    assert (d0, d1, d2) == pytest.approx((g["d0"], g["d1"], g["d2"]), rel=1e-9)
    assert round(zero, 1) == g["gamma_zero_printed"]
    # D = L^2 / (pi^2 tau0) at the printed D(0) and crystal edge gives back D(0)
    p = _load("paper_parameters.json")
    tau0 = p["crystal_edge_m"] ** 2 / (math.pi ** 2 * g["d0"])
    assert A.diffusion_constant(p["crystal_edge_m"], tau0) == pytest.approx(g["d0"], rel=1e-12)


def test_paper_box_and_beam_from_the_printed_parameters():
    p = _load("paper_parameters.json")
    cfg = W.paper_beam(0.05, steps=1)
    n = cfg["grid"]["n"]
    res = cfg["grid"]["res"]
    assert n == (p["grid_cells_per_axis"],) * 3
    assert n[0] / res * p["a_m"] == pytest.approx(p["box_m"], rel=1e-12)       # 6 um box
    assert abs(cfg["opal"]["cells"][0] * p["a_m"] - p["crystal_edge_m"]) <= p["a_m"] / 2  # 4 um crystal
    f0 = cfg["layout"]["f0"]
    assert f0 * C0 / p["a_m"] == pytest.approx(p["f_thz"] * 1e12, rel=1e-3)   # 484 THz in c/a
    assert C0 / (p["f_thz"] * 1e12) * 1e9 == pytest.approx(p["lambda0_nm_printed"], abs=1.0)  # ~620 nm
    assert cfg["sources"][0]["waist"] * p["a_m"] == pytest.approx(p["waist_m"], rel=1e-12)
    # the run length and the spectral resolution it gives (~0.4 THz)
    assert 1.0 / p["run_time_s"] / 1e12 == pytest.approx(p["spectral_resolution_thz_printed"], abs=0.06)


def test_dye_parameters_and_their_normalised_rates():
    """T1 = 1 ns, T2 = 10 fs ("gain bandwidth of order 1/T2 = 100 THz"), n = 1.3,
    N_a = 5e25 m^-3: the density-matrix material carries them, and the oracle's
    normalised dephasing rate is 1/T2 in units of c/a."""
    p = _load("paper_parameters.json")
    m = W.density_material()
    assert m["t1"] == p["t1_s"] and m["t2"] == p["t2_s"]
    assert m["eps"] == pytest.approx(p["host_index"] ** 2, rel=1e-12)
    assert m["n_total"] == p["inversion_m3"]
    assert m["f_a"] * C0 / p["a_m"] == pytest.approx(p["f_thz"] * 1e12, rel=1e-3)
    dt = 0.5 / 16
    w0, wp, kappa, g1, g2, gp = O.bloch_constants(m, dt, 1.0 / 16, p["a_m"])
    t_unit = p["a_m"] / C0
    assert g2 / t_unit == pytest.approx(p["gain_bandwidth_hz_printed"], rel=1e-12)
    assert g1 / t_unit == pytest.approx(1.0 / p["t1_s"], rel=1e-12)
    assert w0 == pytest.approx(2 * math.pi * m["f_a"], rel=1e-15)


def test_diffusion_run_pulse_and_window():
    """The dynamic-diffusion run: a 100 fs pulse (intensity FWHM) in the paper's
    box and beam, T(t) at the back margin, 2.5 ps at Courant 0.5."""
    p = _load("paper_parameters.json")
    cfg = W.paper_diffusion(0.1)
    src = cfg["sources"][0]
    t_unit = p["a_m"] / C0
    assert src["width_kind"] == "fwhm_intensity"
    assert src["width"] * t_unit == pytest.approx(100e-15, rel=1e-12)
    assert cfg["steps"] * 0.5 / cfg["grid"]["res"] * t_unit == pytest.approx(2.5e-12, rel=1e-4)
    assert cfg["flux"][0]["k"] > cfg["layout"]["z0"] + cfg["opal"]["cells"][2] * cfg["grid"]["res"]
    assert cfg["grid"]["n"] == (p["grid_cells_per_axis"],) * 3
