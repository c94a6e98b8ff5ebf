"""Thin ctypes binding of libfdtd (include/fdtd.h).

Argument marshalling only: every step of the method runs in the gfx950
kernels of libfdtd.so.  PyTorch supplies the device arena (one uint8 tensor per
plan) and the stream.  There is no CPU fallback: if the shared library is
missing this module raises at load time.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

BC_PERIODIC, BC_PEC = 0, 1
SRC = {"dipole": 0, "plane": 1, "beam": 2}
WIDTH = {"fwhm_power": 0, "fwhm_intensity": 1, "sigma_t": 2}
DIS = {"none": 0, "uniform": 1, "gauss": 2}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "EUNSTABLE", -6: "EUNSUPPORTED"}


class FdtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32 * 3),
                ("pml_lo", C.c_int32 * 3), ("pml_hi", C.c_int32 * 3),
                ("cpml_m", C.c_double), ("cpml_sigma_max", C.c_double),
                ("cpml_kappa_max", C.c_double), ("cpml_alpha_max", C.c_double),
                ("res", C.c_int32), ("courant", C.c_double), ("a_meters", C.c_double),
                ("seed", C.c_uint32), ("realization", C.c_uint32)]


class Material(C.Structure):
    _fields_ = [("eps", C.c_double), ("gain", C.c_int32), ("n_total", C.c_double),
                ("tau32", C.c_double), ("tau21", C.c_double), ("tau10", C.c_double),
                ("pump", C.c_double), ("f_a", C.c_double), ("df_a", C.c_double),
                ("noise", C.c_double), ("n_init", C.c_double * 4),
                ("t1", C.c_double), ("t2", C.c_double), ("dipole", C.c_double)]


class SourceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32), ("i", C.c_int32), ("j", C.c_int32),
                ("k", C.c_int32), ("f0", C.c_double), ("width_kind", C.c_int32),
                ("width", C.c_double), ("delay", C.c_double), ("amp", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("waist", C.c_double)]


class OpalDesc(C.Structure):
    _fields_ = [("cells", C.c_int32 * 3), ("origin", C.c_int32 * 3), ("r0", C.c_double),
                ("disorder", C.c_int32), ("strength", C.c_double),
                ("mat_bg", C.c_int32), ("mat_void", C.c_int32), ("mat_out", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("zchunk", C.c_int32), ("graph_steps", C.c_int32),
                ("max_blocks", C.c_int32), ("tile_x", C.c_int32), ("merge", C.c_int32),
                ("parallel", C.c_int32), ("stores", C.c_int32), ("cache_mb", C.c_int32)]


STORES = {"auto": 0, "ordinary": 1, "nontemporal": 2}
TUNING_KEYS = ("block", "zchunk", "graph_steps", "max_blocks", "tile_x", "merge", "parallel", "stores", "cache_mb")


def make_tuning(t):
    """Tuning struct from a tuning dict (missing keys take the defaults)."""
    d = dict(default_tuning())
    d.update(t or {})
    return Tuning(*[int(d[k]) for k in TUNING_KEYS])


# Every exported symbol of include/fdtd.h with its ctypes signature.
P = C.POINTER
VP = C.c_void_p
SIGNATURES = {
    "fdtd_last_error": ([], C.c_char_p),
    "fdtd_version": ([], C.c_char_p),
    "fdtd_plan_create": ([P(GridDesc), P(VP)], C.c_int),
    "fdtd_plan_destroy": ([VP], None),
    "fdtd_set_materials": ([VP, P(Material), C.c_int32], C.c_int),
    "fdtd_build_opal": ([VP, P(OpalDesc)], C.c_int),
    "fdtd_set_material_map": ([VP, P(C.c_uint8)], C.c_int),
    "fdtd_get_spheres": ([VP, P(C.c_int64), P(C.c_int64)], C.c_int),
    "fdtd_get_material_map": ([VP, P(C.c_uint8), VP], C.c_int),
    "fdtd_add_source": ([VP, P(SourceDesc), P(C.c_int32)], C.c_int),
    "fdtd_add_probe": ([VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(C.c_int32)], C.c_int),
    "fdtd_add_flux_plane": ([VP, C.c_int32, C.c_int32, P(C.c_double), C.c_int32, C.c_int32, P(C.c_int32)], C.c_int),
    "fdtd_set_energy_interval": ([VP, C.c_int32], C.c_int),
    "fdtd_set_tuning": ([VP, P(Tuning)], C.c_int),
    "fdtd_get_tuning": ([VP, P(Tuning)], C.c_int),
    "fdtd_required_bytes": ([VP, C.c_int64, P(C.c_size_t)], C.c_int),
    "fdtd_bind_arena": ([VP, VP, C.c_size_t, C.c_int64, VP], C.c_int),
    "fdtd_step": ([VP, C.c_int64, VP], C.c_int),
    "fdtd_step_count": ([VP], C.c_int64),
    "fdtd_cell_count": ([VP], C.c_int64),
    "fdtd_dt": ([VP], C.c_double),
    "fdtd_read_field": ([VP, C.c_int32, P(C.c_float), VP], C.c_int),
    "fdtd_write_field": ([VP, C.c_int32, P(C.c_float), VP], C.c_int),
    "fdtd_read_probe": ([VP, C.c_int32, P(C.c_float), P(C.c_int64), VP], C.c_int),
    "fdtd_read_flux": ([VP, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_int64), VP], C.c_int),
    "fdtd_read_populations": ([VP, P(C.c_double), VP], C.c_int),
    "fdtd_read_polarization": ([VP, P(C.c_float), VP], C.c_int),
    "fdtd_read_density": ([VP, P(C.c_float), VP], C.c_int),
    "fdtd_read_energy": ([VP, P(C.c_double), P(C.c_int64), VP], C.c_int),
    "fdtd_batch_create": ([P(VP), C.c_int32, P(Tuning), P(VP)], C.c_int),
    "fdtd_batch_create_static": ([P(VP), C.c_int32, P(Tuning), P(VP)], C.c_int),
    "fdtd_batch_step": ([VP, C.c_int64, VP], C.c_int),
    "fdtd_batch_set_members": ([VP, P(VP), C.c_int32, VP], C.c_int),
    "fdtd_batch_destroy": ([VP], None),
    "fdtd_time_steps": ([VP, C.c_int64, VP, P(C.c_double)], C.c_int),
    "fdtd_batch_time_steps": ([VP, C.c_int64, VP, P(C.c_double)], C.c_int),
    "fdtd_class_cells": ([VP, P(C.c_int64)], C.c_int),
    "fdtd_class_bytes": ([VP, P(C.c_double)], C.c_int),
    "fdtd_time_kernels": ([VP, C.c_int64, VP, P(C.c_double), P(C.c_int64)], C.c_int),
    "fdtd_batch_time_kernels": ([VP, C.c_int64, VP, P(C.c_double), P(C.c_int64)], C.c_int),
    "fdtd_tune": ([VP, P(Tuning), C.c_int32, C.c_int64, C.c_int64, VP, C.c_size_t, P(C.c_size_t), P(C.c_double),
                   VP], C.c_int),
}

_lib = None


def lib():
    """Load libfdtd.so (built in-tree by paper_0802_3775_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfdtd.so is not built (run python -m paper_0802_3775_amd.build); "
                               "there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise FdtdError(code, lib().fdtd_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _grid(g):
    d = GridDesc()
    d.nx, d.ny, d.nz = g["n"]
    per = g.get("periodic", (1, 1, 1))
    d.bc[:] = [BC_PERIODIC if p else BC_PEC for p in per]
    d.pml_lo[:] = list(g.get("pml_lo", (0, 0, 0)))
    d.pml_hi[:] = list(g.get("pml_hi", (0, 0, 0)))
    cp = g.get("cpml", {})
    d.cpml_m = cp.get("m", 3.0)
    d.cpml_sigma_max = cp.get("sigma_max", -1.0)
    d.cpml_kappa_max = cp.get("kappa_max", 1.0)
    d.cpml_alpha_max = cp.get("alpha_max", 0.0)
    d.res = g["res"]
    d.courant = g.get("courant", 0.5)
    d.a_meters = g.get("a_meters", 480e-9)
    d.seed = g.get("seed", 0)
    d.realization = g.get("realization", 0)
    return d


def _material(m):
    d = Material()
    d.eps = m["eps"]
    d.gain = int(m.get("gain") or 0)
    for f in ("n_total", "tau32", "tau21", "tau10", "pump", "f_a", "df_a", "noise", "t1", "t2", "dipole"):
        setattr(d, f, float(m.get(f, 0.0)))
    if d.gain:
        d.n_init[:] = list(m.get("n_init", (1.0, 0.0, 0.0, 0.0)))
    return d


def default_tuning(cfg=None):
    return {"block": 256, "zchunk": 4, "graph_steps": 64, "max_blocks": 0, "tile_x": 32, "merge": 1,
            "parallel": 0, "stores": 0, "cache_mb": 0}


class Plan:
    """One realization on the GPU, built from a workload config dict."""

    def __init__(self, cfg, max_steps=None, tuning=None, stream=None, bind=True):
        import torch
        self.cfg = cfg
        self.n = tuple(cfg["grid"]["n"])
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.h = C.c_void_p()
        g = _grid(cfg["grid"])
        _check(lib().fdtd_plan_create(C.byref(g), C.byref(self.h)))
        mats = cfg["materials"]
        arr = (Material * len(mats))(*[_material(m) for m in mats])
        _check(lib().fdtd_set_materials(self.h, arr, len(mats)))
        if cfg.get("map") is not None:
            mp = np.ascontiguousarray(cfg["map"], dtype=np.uint8)
            _check(lib().fdtd_set_material_map(self.h, _ptr(mp, C.c_uint8)))
        elif cfg.get("opal") is not None:
            o = cfg["opal"]
            d = OpalDesc()
            d.cells[:] = list(o["cells"])
            d.origin[:] = list(o.get("origin", (0, 0, 0)))
            d.r0 = o["r0"]
            d.disorder = DIS[o.get("disorder", "none")]
            d.strength = o.get("strength", 0.0)
            d.mat_bg, d.mat_void, d.mat_out = o.get("mat_bg", 0), o.get("mat_void", 1), o.get("mat_out", 1)
            _check(lib().fdtd_build_opal(self.h, C.byref(d)))
        for s in cfg.get("sources", []):
            d = SourceDesc()
            d.kind = SRC[s["kind"]]
            d.comp = s["comp"]
            d.i, d.j, d.k = s.get("i", 0), s.get("j", 0), s["k"]
            d.f0 = s["f0"]
            d.width_kind = WIDTH[s["width_kind"]]
            d.width = s["width"]
            d.delay = s["delay"]
            d.amp = s.get("amp", 1.0)
            d.x0, d.y0, d.waist = s.get("x0", 0.0), s.get("y0", 0.0), s.get("waist", 0.0)
            _check(lib().fdtd_add_source(self.h, C.byref(d), None))
        self.nprobe = 0
        for p in cfg.get("probes", []):
            _check(lib().fdtd_add_probe(self.h, *[int(v) for v in p], None))
            self.nprobe += 1
        self.nf = []
        for f in cfg.get("flux", []):
            fr = np.ascontiguousarray(f["freqs"], dtype=np.float64)
            _check(lib().fdtd_add_flux_plane(self.h, int(f.get("axis", 2)), int(f["k"]), _ptr(fr, C.c_double),
                                             len(fr), int(f.get("decim", 1)), None))
            self.nf.append(len(fr))
        if cfg.get("energy_interval"):
            _check(lib().fdtd_set_energy_interval(self.h, int(cfg["energy_interval"])))
        t = dict(default_tuning(cfg))
        t.update(tuning or {})
        tu = make_tuning(t)
        _check(lib().fdtd_set_tuning(self.h, C.byref(tu)))
        self.tuning = t
        self.max_steps = int(max_steps if max_steps is not None else cfg.get("steps", 0))
        self.arena = None
        if bind:
            self.bind(stream)

    def required_bytes(self):
        b = C.c_size_t()
        _check(lib().fdtd_required_bytes(self.h, self.max_steps, C.byref(b)))
        return b.value

    def bind(self, stream=None):
        import torch
        nbytes = self.required_bytes()
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        _check(lib().fdtd_bind_arena(self.h, C.c_void_p(aligned), nbytes, self.max_steps, _stream(stream)))
        for comp, a in (self.cfg.get("init_fields") or {}).items():
            self.write_field(comp, a, stream)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().fdtd_plan_destroy(self.h)
            self.h = C.c_void_p()
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, candidates, steps, warmup=4, stream=None):
        """Milliseconds per step of each candidate tuning (dicts), timed by
        fdtd_tune on scratch plans of this plan's description bound to one torch
        scratch arena; None for an invalid candidate."""
        import torch
        cand = (Tuning * len(candidates))(*[make_tuning(t) for t in candidates])
        need = C.c_size_t()
        _check(lib().fdtd_tune(self.h, cand, len(candidates), int(warmup), int(steps), None, 0, C.byref(need),
                               None, _stream(stream)))
        scratch = torch.empty(need.value + 256, dtype=torch.uint8, device="cuda")
        base = (scratch.data_ptr() + 255) & ~255
        ms = np.zeros(len(candidates), dtype=np.float64)
        try:
            _check(lib().fdtd_tune(self.h, cand, len(candidates), int(warmup), int(steps), C.c_void_p(base),
                                   need.value, None, _ptr(ms, C.c_double), _stream(stream)))
        finally:
            torch.cuda.synchronize()
            del scratch
        return [float(v) if v >= 0 else None for v in ms]

    # -------------------------------------------------------------- stepping
    def step(self, n, stream=None):
        _check(lib().fdtd_step(self.h, int(n), _stream(stream)))

    def time_steps(self, n, stream=None):
        ms = C.c_double()
        _check(lib().fdtd_time_steps(self.h, int(n), _stream(stream), C.byref(ms)))
        return ms.value

    CLASSES = ("step_plain", "step_cpml_z", "step_cpml", "step_gain", "step_cpml_z_gain",
               "step_cpml_gain", "dft", "dm_predict", "dm_correct", "dm_edges", "dm_diag")

    def class_cells(self):
        out = np.zeros(len(self.CLASSES), dtype=np.int64)
        _check(lib().fdtd_class_cells(self.h, _ptr(out, C.c_int64)))
        return out

    def class_bytes(self):
        out = np.zeros(len(self.CLASSES), dtype=np.float64)
        _check(lib().fdtd_class_bytes(self.h, _ptr(out, C.c_double)))
        return out

    def time_kernels(self, n, stream=None):
        """Per kernel class: (total ms, launches) over n eager steps."""
        ms = np.zeros(len(Plan.CLASSES), dtype=np.float64)
        cnt = np.zeros(len(Plan.CLASSES), dtype=np.int64)
        _check(lib().fdtd_time_kernels(self.h, int(n), _stream(stream), _ptr(ms, C.c_double),
                                       _ptr(cnt, C.c_int64)))
        return ms, cnt

    @property
    def step_count(self):
        return lib().fdtd_step_count(self.h)

    @property
    def dt(self):
        return lib().fdtd_dt(self.h)

    # -------------------------------------------------------------- readout
    def spheres(self):
        n = C.c_int64()
        _check(lib().fdtd_get_spheres(self.h, None, C.byref(n)))
        out = np.zeros((n.value, 5), dtype=np.int64)
        if n.value:
            _check(lib().fdtd_get_spheres(self.h, _ptr(out, C.c_int64), C.byref(n)))
        return out

    def material_map(self, stream=None):
        out = np.zeros(self.n[::-1], dtype=np.uint8)
        _check(lib().fdtd_get_material_map(self.h, _ptr(out, C.c_uint8), _stream(stream)))
        return out

    def field(self, comp, stream=None):
        out = np.zeros(self.n[::-1], dtype=np.float32)
        _check(lib().fdtd_read_field(self.h, int(comp), _ptr(out, C.c_float), _stream(stream)))
        return out

    def fields(self, stream=None):
        return np.stack([self.field(c, stream) for c in range(6)])

    def write_field(self, comp, arr, stream=None):
        a = np.ascontiguousarray(arr, dtype=np.float32).reshape(self.n[::-1])
        _check(lib().fdtd_write_field(self.h, int(comp), _ptr(a, C.c_float), _stream(stream)))

    def probe(self, pid, stream=None):
        out = np.zeros(max(self.max_steps, 1), dtype=np.float32)
        n = C.c_int64()
        _check(lib().fdtd_read_probe(self.h, int(pid), _ptr(out, C.c_float), C.byref(n), _stream(stream)))
        return out[: n.value]

    def flux(self, fid, stream=None):
        T = np.zeros(max(self.max_steps, 1), dtype=np.float64)
        spec = np.zeros(max(self.nf[fid], 1), dtype=np.float64)
        n = C.c_int64()
        _check(lib().fdtd_read_flux(self.h, int(fid), _ptr(T, C.c_double), _ptr(spec, C.c_double),
                                    C.byref(n), _stream(stream)))
        return T[: n.value], spec[: self.nf[fid]]

    def populations(self, stream=None):
        """n0..n3 of the gain cells (FP64: the exact sums of the stored pairs)."""
        out = np.zeros((4,) + self.n[::-1], dtype=np.float64)
        _check(lib().fdtd_read_populations(self.h, _ptr(out, C.c_double), _stream(stream)))
        return out

    def density(self, stream=None):
        """Density matrix of the density-matrix gain cells, 15 planes: rho_11..33,
        Re rho_01..03, Im rho_01..03, Re rho_12, 13, 23, Im rho_12, 13, 23."""
        out = np.zeros((15,) + self.n[::-1], dtype=np.float32)
        _check(lib().fdtd_read_density(self.h, _ptr(out, C.c_float), _stream(stream)))
        return out

    def polarization(self, stream=None):
        out = np.zeros((3,) + self.n[::-1], dtype=np.float32)
        _check(lib().fdtd_read_polarization(self.h, _ptr(out, C.c_float), _stream(stream)))
        return out

    def energy(self, stream=None):
        out = np.zeros(self.max_steps + 1, dtype=np.float64)
        n = C.c_int64()
        _check(lib().fdtd_read_energy(self.h, _ptr(out, C.c_double), C.byref(n), _stream(stream)))
        return out[: n.value]


class Batch:
    """Bound plans stepped together: one launch per tile class per step.
    tuning: the batch's launch settings (graph_steps, max_blocks, parallel,
    stores; block and tile_x must be the members'); None takes the first
    member's.  static: launch tables in the library's static per-GPU array
    (fdtd_batch_create_static: no device allocation)."""

    def __init__(self, plans, tuning=None, static=False):
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p.h.value for p in self.plans])
        self.h = C.c_void_p()
        t = None
        if tuning is not None:
            base = dict(self.plans[0].tuning)
            base.update(tuning)
            t = C.byref(make_tuning(base))
        create = lib().fdtd_batch_create_static if static else lib().fdtd_batch_create
        _check(create(arr, len(self.plans), t, C.byref(self.h)))

    def set_members(self, plans, stream=None):
        """Replace the members in place (tables rewritten, grown only if needed)."""
        plans = list(plans)
        arr = (C.c_void_p * len(plans))(*[p.h.value for p in plans])
        _check(lib().fdtd_batch_set_members(self.h, arr, len(plans), _stream(stream)))
        self.plans = plans

    def step(self, n, stream=None):
        _check(lib().fdtd_batch_step(self.h, int(n), _stream(stream)))

    def time_steps(self, n, stream=None):
        ms = C.c_double()
        _check(lib().fdtd_batch_time_steps(self.h, int(n), _stream(stream), C.byref(ms)))
        return ms.value

    def time_kernels(self, n, stream=None):
        """Per kernel class: (total ms, launches) over n eager batch steps."""
        ms = np.zeros(len(Plan.CLASSES), dtype=np.float64)
        cnt = np.zeros(len(Plan.CLASSES), dtype=np.int64)
        _check(lib().fdtd_batch_time_kernels(self.h, int(n), _stream(stream), _ptr(ms, C.c_double),
                                             _ptr(cnt, C.c_int64)))
        return ms, cnt

    def class_bytes(self):
        """Algorithmic bytes of one launch of each class over all members."""
        return np.sum([p.class_bytes() for p in self.plans], axis=0)

    def class_cells(self):
        return np.sum([p.class_cells() for p in self.plans], axis=0)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().fdtd_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
