"""Host-side checks of libfdtd (no GPU needed): the shared library loads, exports
every function declared in include/fdtd.h, validates plans, and its host
geometry (Philox4x32-10 + Box-Muller sphere list) matches the oracle's bit for bit.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_0802_3775_amd import fdtd as F
from paper_0802_3775_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 30
    lib = F.lib()
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(F.SIGNATURES)


def test_version_string():
    assert b"gfx950" in F.lib().fdtd_version()


def _plan(g):
    h = C.c_void_p()
    code = F.lib().fdtd_plan_create(C.byref(F._grid(g)), C.byref(h))
    return code, h


def test_plan_validation():
    g = W.periodic_cell(res=8)["grid"]
    code, h = _plan(g)
    assert code == 0
    F.lib().fdtd_plan_destroy(h)
    bad = dict(g, courant=0.6)
    assert _plan(bad)[0] == -5  # EUNSTABLE: 3-D Yee limit 1/sqrt(3)
    assert b"courant" in F.lib().fdtd_last_error()
    assert _plan(dict(g, n=(0, 4, 4)))[0] == -1
    assert _plan(dict(g, pml_lo=(2, 0, 0)))[0] == -1  # CPML on a periodic axis


def test_add_calls_reject_out_of_range():
    cfg = W.slab(res=8, cells=(1, 1, 2), steps=10, nf=4)
    code, h = _plan(cfg["grid"])
    assert code == 0
    L = F.lib()
    assert L.fdtd_add_probe(h, 0, 99, 0, 0, None) == -1
    assert L.fdtd_add_probe(h, 7, 0, 0, 0, None) == -1
    fr = np.array([0.8])
    assert L.fdtd_add_flux_plane(h, 2, 0, F._ptr(fr, C.c_double), 1, 1, None) == -1  # k=0 on a PEC axis
    assert L.fdtd_add_flux_plane(h, 2, 5, F._ptr(fr, C.c_double), 1, 0, None) == -1  # decim 0
    assert L.fdtd_add_flux_plane(h, 3, 5, F._ptr(fr, C.c_double), 1, 1, None) == -1  # no such axis
    assert L.fdtd_add_flux_plane(h, 0, 5, F._ptr(fr, C.c_double), 1, 1, None) == -6  # x-normal: unsupported
    assert b"normal to z" in L.fdtd_last_error()
    assert L.fdtd_add_flux_plane(h, 2, 5, F._ptr(fr, C.c_double), 1, 1, None) == 0
    t = F.Tuning(100, 8, 0, 0)
    assert L.fdtd_set_tuning(h, C.byref(t)) == -1  # block not a multiple of 64
    # the tile's halo ring must fit one cell per thread: 2 (tx+2) + 2 block/tx <= block
    for block, tx, ok in ((64, 16, True), (64, 32, False), (128, 32, True), (128, 64, False), (256, 64, True)):
        t = F.Tuning(block, 4, 0, 0, tx, 1, 0)
        assert (L.fdtd_set_tuning(h, C.byref(t)) == 0) == ok, (block, tx)
    t = F.make_tuning({"stores": 3})
    assert L.fdtd_set_tuning(h, C.byref(t)) == -1  # no such store mode
    size = C.c_size_t()
    assert L.fdtd_set_tuning(h, C.byref(F.make_tuning({}))) == 0
    assert L.fdtd_required_bytes(h, 100, C.byref(size)) == 0 and size.value > 0
    L.fdtd_plan_destroy(h)


def test_tune_sizes_its_scratch_arena_on_the_host():
    """fdtd_tune with no scratch arena only sizes it: the largest arena any valid
    candidate needs for warmup + steps steps, equal to fdtd_required_bytes of a
    plan with that candidate; invalid candidates are skipped, the plan untouched."""
    cfg = W.slab(res=8, cells=(1, 1, 2), steps=10, nf=4)
    plan = F.Plan(cfg, max_steps=10, bind=False)
    L = F.lib()
    tunes = [{"tile_x": 16, "block": 128, "zchunk": 1}, {"tile_x": 64, "block": 128}, {"zchunk": 8}]
    arr = (F.Tuning * 3)(*[F.make_tuning(t) for t in tunes])
    need = C.c_size_t()
    assert L.fdtd_tune(plan.h, arr, 3, 2, 6, None, 0, C.byref(need), None, None) == 0
    sizes = []
    for t in (tunes[0], tunes[2]):
        p2 = F.Plan(cfg, max_steps=8, tuning=t, bind=False)
        sizes.append(p2.required_bytes())
        p2.close()
    assert need.value == max(sizes)
    assert plan.required_bytes() > 0 and plan.tuning == F.default_tuning()
    assert L.fdtd_tune(plan.h, arr, 0, 2, 6, None, 0, C.byref(need), None, None) == -1
    assert L.fdtd_tune(plan.h, arr, 3, 2, 0, None, 0, C.byref(need), None, None) == -1
    plan.close()


@pytest.mark.parametrize("maker", [
    lambda: W.periodic_cell(res=32),
    lambda: W.slab(delta=0.05, seed=12, res=20, steps=1),
    lambda: W.slab(delta=0.10, seed=14, res=20, steps=1),
    lambda: W.lasing(delta=0.05, steps=1),
    lambda: W.ensemble(count=3, steps=1)[2],
])
def test_sphere_list_matches_oracle_bit_for_bit(maker):
    cfg = maker()
    code, h = _plan(cfg["grid"])
    assert code == 0
    o = cfg["opal"]
    d = F.OpalDesc()
    d.cells[:] = list(o["cells"])
    d.origin[:] = list(o["origin"])
    d.r0 = o["r0"]
    d.disorder = F.DIS[o["disorder"]]
    d.strength = o["strength"]
    d.mat_bg, d.mat_void, d.mat_out = o["mat_bg"], o["mat_void"], o["mat_out"]
    mats = (F.Material * len(cfg["materials"]))(*[F._material(m) for m in cfg["materials"]])
    assert F.lib().fdtd_set_materials(h, mats, len(cfg["materials"])) == 0
    assert F.lib().fdtd_build_opal(h, C.byref(d)) == 0, F.lib().fdtd_last_error()
    n = C.c_int64()
    F.lib().fdtd_get_spheres(h, None, C.byref(n))
    got = np.zeros((n.value, 5), dtype=np.int64)
    F.lib().fdtd_get_spheres(h, F._ptr(got, C.c_int64), C.byref(n))
    F.lib().fdtd_plan_destroy(h)
    want = O.opal_spheres(cfg["grid"], cfg["opal"])
    assert np.array_equal(got, want)


def test_density_matrix_materials_validated():
    """gain = 2 materials: parameters checked at fdtd_set_materials, one gain model
    per plan, transitions too fast for dt rejected, 18 state floats per cell."""
    g = W.periodic_cell(res=8)["grid"]
    L = F.lib()

    def set_mats(mats):
        code, h = _plan(g)
        assert code == 0
        arr = (F.Material * len(mats))(*[F._material(m) for m in mats])
        r = L.fdtd_set_materials(h, arr, len(mats))
        return r, h

    dm = W.density_material()
    r, h = set_mats([{"eps": 11.9}, dm])
    assert r == 0
    t = F.Tuning(128, 4, 0, 0, 16, 1, 0)
    assert L.fdtd_set_tuning(h, C.byref(t)) == 0
    with_dm = C.c_size_t()
    assert L.fdtd_required_bytes(h, 10, C.byref(with_dm)) == 0
    L.fdtd_plan_destroy(h)
    r, h = set_mats([{"eps": 11.9}, W.gain_material()])
    assert L.fdtd_set_tuning(h, C.byref(t)) == 0
    with_lorentz = C.c_size_t()
    assert L.fdtd_required_bytes(h, 10, C.byref(with_lorentz)) == 0
    L.fdtd_plan_destroy(h)
    # 18 floats per cell instead of 6 populations and two P buffers (12)
    ncell = 8 * 8 * 8
    assert with_dm.value - with_lorentz.value >= 4 * ncell * (18 - 12) - 4096
    for bad in (dict(dm, t1=0.0), dict(dm, t2=-1.0), dict(dm, f_a=0.0), dict(dm, pump=-1.0)):
        r, h = set_mats([{"eps": 11.9}, bad])
        assert r == -1, bad
        L.fdtd_plan_destroy(h)
    r, h = set_mats([{"eps": 11.9}, dm, W.gain_material()])
    assert r == -6 and b"gain models" in L.fdtd_last_error()
    L.fdtd_plan_destroy(h)
    r, h = set_mats([{"eps": 11.9}, dict(dm, f_a=20.0)])  # w0 dt >= pi at 8 cells/a
    assert r == -5
    L.fdtd_plan_destroy(h)
