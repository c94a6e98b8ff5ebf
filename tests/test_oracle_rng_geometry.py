"""Pins of the oracle's random numbers and inverted-opal geometry (CPU only).

Paper, section "Sample and numerical approach": air spheres at the fcc sites of
a cubic lattice in a dielectric background, r0 = a/(2 sqrt 2), disorder on the
radius r = r0 (1 + gamma xi) with xi uniform in [-1/2, 1/2].
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0802_3775_amd import workloads as W


def test_philox_known_answers():
    # Known-answer vectors published with the Philox4x32-10 reference
    # implementation (Salmon et al., SC'11): counter, key -> output.
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert [int(v) for v in O.philox(ctr, key)] == want


def test_box_muller_moments():
    # 4 x 20000 normals from consecutive counters: moments of N(0, 1).
    g = np.array([O.normals4([n, 5, 0, 2], [7, 3]) for n in range(20000)]).ravel()
    assert abs(g.mean()) < 0.02
    assert abs(g.var() - 1.0) < 0.03
    assert abs(np.mean(g ** 4) - 3.0) < 0.15
    # the two members of each Box-Muller pair are uncorrelated
    pairs = g.reshape(-1, 2)
    assert abs(np.mean(pairs[:, 0] * pairs[:, 1])) < 0.02


def _fcc_count(n, periodic):
    ext = [2 * c if p else 2 * c + 1 for c, p in zip(n, periodic)]
    return sum(1 for h, k, l in itertools.product(*[range(e) for e in ext]) if (h + k + l) % 2 == 0)


def test_sphere_sites_ordered():
    cfg = W.periodic_cell(res=16)
    sph = O.opal_spheres(cfg["grid"], cfg["opal"])
    # one cubic fcc cell, periodic: the 4 sites (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2)
    assert sph.shape == (4, 5)
    q = 2 * 16 * 65536  # quanta per a
    got = sorted(tuple(r) for r in (sph[:, 1:4] / (q / 2)).astype(int))
    assert got == sorted([(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])
    assert np.all(sph[:, 4] == round(0.35 * q))
    # slab: 4x4x8 periodic in x, y, closed in z
    cfg = W.slab(res=8, steps=1, nf=0)
    sph = O.opal_spheres(cfg["grid"], cfg["opal"])
    assert sph.shape[0] == _fcc_count((4, 4, 8), (1, 1, 0)) == 544


def test_gauss_jitter_statistics():
    cfg = W.lasing(res=8, cells=(6, 6, 6), delta=0.05, steps=1)
    sph = O.opal_spheres(cfg["grid"], cfg["opal"])
    cfg0 = W.lasing(res=8, cells=(6, 6, 6), delta=0.0, steps=1)
    sph0 = O.opal_spheres(cfg0["grid"], cfg0["opal"])
    assert np.array_equal(sph[:, 0], sph0[:, 0])
    q = 2 * 8 * 65536
    dc = (sph[:, 1:4] - sph0[:, 1:4]) / q
    dr = (sph[:, 4] - sph0[:, 4]) / q
    for v in (dc.ravel(), dr):
        assert abs(v.mean()) < 0.05 * 0.15
        assert abs(v.std() - 0.05) < 0.05 * 0.1
        assert np.abs(v).max() <= 4 * 0.05 + 1.0 / q


def test_uniform_radius_disorder():
    cfg = W.slab(res=8, steps=1, nf=0)
    cfg["opal"].update(disorder="uniform", strength=0.2, r0=1.0 / (2 * math.sqrt(2)))
    sph = O.opal_spheres(cfg["grid"], cfg["opal"])
    q = 2 * 8 * 65536
    r = sph[:, 4] / q
    r0 = 1.0 / (2 * math.sqrt(2))
    xi = (r / r0 - 1.0) / 0.2
    assert xi.min() >= -0.5 - 1e-6 and xi.max() <= 0.5 + 1e-6
    assert abs(xi.mean()) < 0.05 and abs(xi.var() - 1.0 / 12.0) < 0.02


@pytest.mark.parametrize("maker", [
    lambda: W.periodic_cell(res=24),
    lambda: W.slab(delta=0.1, res=10, cells=(2, 2, 3), steps=1, nf=0),
    lambda: W.lasing(delta=0.05, res=10, cells=(2, 2, 2), steps=1, pml=4),
    lambda: W.ensemble(count=1, steps=1, max_cells=36 ** 3, n_range=(2, 3), res_range=(8, 12))[0],
])
def test_gather_equals_scatter(maker):
    cfg = maker()
    a = O.voxelize(cfg["grid"], cfg["opal"], method="gather")
    b = O.voxelize(cfg["grid"], cfg["opal"], method="scatter")
    assert np.array_equal(a, b)
    assert set(np.unique(a)) <= {cfg["opal"]["mat_bg"], cfg["opal"]["mat_void"], cfg["opal"]["mat_out"]}


def test_ordered_map_cubic_symmetry():
    cfg = W.periodic_cell(res=20)
    m = O.voxelize(cfg["grid"], cfg["opal"])  # [z, y, x]
    # voxel centres (i + 1/2) dx; the fcc lattice is invariant under x -> L - x (i -> N-1-i)
    for ax in range(3):
        assert np.array_equal(m, np.flip(m, axis=ax))
    for perm in itertools.permutations(range(3)):
        assert np.array_equal(m, np.transpose(m, perm))


def test_void_fraction_closed_form():
    # r = 0.35 a < a/(2 sqrt 2): the 4 spheres per cubic cell do not overlap,
    # void fraction = 4 (4/3) pi r^3 = 0.71838...
    exact = 16.0 / 3.0 * math.pi * 0.35 ** 3
    errs = []
    for res in (16, 32, 64):
        cfg = W.periodic_cell(res=res)
        m = O.voxelize(cfg["grid"], cfg["opal"])
        frac = float(np.mean(m == 1))
        # surface-voxel bound: sphere area * half voxel diagonal / volume
        bound = 4 * 4 * math.pi * 0.35 ** 2 * (math.sqrt(3) / 2) / res
        errs.append(abs(frac - exact))
        assert abs(frac - exact) < bound
    assert errs[-1] < 2e-3


def test_crystal_region_and_outside_material():
    cfg = W.lasing(delta=0.0, res=8, cells=(2, 2, 2), steps=1, pml=5)
    m = O.voxelize(cfg["grid"], cfg["opal"])
    inner = m[5:-5, 5:-5, 5:-5]
    outer = m.copy()
    outer[5:-5, 5:-5, 5:-5] = 2
    assert np.all(outer == 2)       # outside the crystal: the PML vacuum material
    assert set(np.unique(inner)) == {0, 1}
