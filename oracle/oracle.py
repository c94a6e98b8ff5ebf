"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The GPU library never imports this module, and
this module never imports the GPU library.

Configurations are the plain dicts built by ``paper_0802_3775_amd.workloads``
(the seeded input generators shared by both sides; they hold no arithmetic of
the method).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

DIS = {"none": 0, "uniform": 1, "gauss": 2}
SRC = {"dipole": 0, "plane": 1, "beam": 2}
WIDTH = {"fwhm_power": 0, "fwhm_intensity": 1, "sigma_t": 2}


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("pml_lo", C.c_int32 * 3), ("pml_hi", C.c_int32 * 3),
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


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32), ("i", C.c_int32), ("j", C.c_int32),
                ("k", C.c_int32), ("f0", C.c_double), ("width_kind", C.c_int32),
                ("width", C.c_double), ("delay", C.c_double), ("amp", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("waist", C.c_double)]


class Opal(C.Structure):
    _fields_ = [("cells", C.c_int32 * 3), ("origin", C.c_int32 * 3), ("r0", C.c_double),
                ("disorder", C.c_int32), ("strength", C.c_double),
                ("mat_bg", C.c_int32), ("mat_void", C.c_int32), ("mat_out", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_normals4.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_double)]
        L.orc_opal_count.argtypes = [P(Grid), P(Opal)]
        L.orc_opal_count.restype = C.c_int64
        L.orc_opal_spheres.argtypes = [P(Grid), P(Opal), P(C.c_int64)]
        for fn in (L.orc_voxelize_gather, L.orc_voxelize_scatter):
            fn.argtypes = [P(Grid), P(Opal), P(C.c_int64), C.c_int64, P(C.c_uint8)]
        L.orc_create.argtypes = [P(Grid), P(Material), C.c_int32, C.c_int64]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_material_map.argtypes = [C.c_void_p, P(C.c_uint8)]
        L.orc_add_source.argtypes = [C.c_void_p, P(Source)]
        L.orc_add_probe.argtypes = [C.c_void_p] + [C.c_int32] * 4
        L.orc_add_flux_plane.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), C.c_int32, C.c_int32]
        L.orc_set_energy_interval.argtypes = [C.c_void_p, C.c_int32]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_step_count.restype = C.c_int64
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
        L.orc_get_populations.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_get_polarization.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_get_density.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_bloch_evolve.argtypes = [P(Material), C.c_double, C.c_double, C.c_double, C.c_int64,
                                       P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_bloch_constants.argtypes = [P(Material), C.c_double, C.c_double, C.c_double, P(C.c_double)]
        L.orc_get_probe.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
        L.orc_get_probe.restype = C.c_int64
        L.orc_get_flux.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double)]
        L.orc_get_flux.restype = C.c_int64
        L.orc_get_energy.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_get_energy.restype = C.c_int64
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_dt.restype = C.c_double
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ------------------------------------------------------------------ structs

def make_grid(g):
    cp = g.get("cpml", {})
    s = Grid()
    s.nx, s.ny, s.nz = g["n"]
    s.periodic[:] = list(g.get("periodic", (1, 1, 1)))
    s.pml_lo[:] = list(g.get("pml_lo", (0, 0, 0)))
    s.pml_hi[:] = list(g.get("pml_hi", (0, 0, 0)))
    s.cpml_m = cp.get("m", 3.0)
    s.cpml_sigma_max = cp.get("sigma_max", -1.0)
    s.cpml_kappa_max = cp.get("kappa_max", 1.0)
    s.cpml_alpha_max = cp.get("alpha_max", 0.0)
    s.res = g["res"]
    s.courant = g.get("courant", 0.5)
    s.a_meters = g.get("a_meters", 480e-9)
    s.seed = g.get("seed", 0)
    s.realization = g.get("realization", 0)
    return s


def make_material(m):
    s = Material()
    s.eps = m["eps"]
    s.gain = int(m.get("gain") or 0)
    for f in ("n_total", "tau32", "tau21", "tau10", "pump", "f_a", "df_a", "noise", "t1", "t2", "dipole"):
        setattr(s, f, float(m.get(f, 0.0)))
    if s.gain:
        s.n_init[:] = list(m.get("n_init", (1.0, 0.0, 0.0, 0.0)))
    return s


def make_opal(o):
    s = Opal()
    s.cells[:] = list(o["cells"])
    s.origin[:] = list(o.get("origin", (0, 0, 0)))
    s.r0 = o["r0"]
    s.disorder = DIS[o.get("disorder", "none")]
    s.strength = o.get("strength", 0.0)
    s.mat_bg, s.mat_void, s.mat_out = o.get("mat_bg", 0), o.get("mat_void", 1), o.get("mat_out", 1)
    return s


def make_source(d):
    s = Source()
    s.kind = SRC[d["kind"]]
    s.comp = d["comp"]
    s.i, s.j, s.k = d.get("i", 0), d.get("j", 0), d["k"]
    s.f0 = d["f0"]
    s.width_kind = WIDTH[d["width_kind"]]
    s.width = d["width"]
    s.delay = d["delay"]
    s.amp = d.get("amp", 1.0)
    s.x0, s.y0, s.waist = d.get("x0", 0.0), d.get("y0", 0.0), d.get("waist", 0.0)
    return s


# ------------------------------------------------------------------ RNG / geometry

def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def normals4(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.float64)
    lib().orc_normals4(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_double))
    return out


def opal_spheres(grid, opal):
    g, o = make_grid(grid), make_opal(opal)
    n = lib().orc_opal_count(C.byref(g), C.byref(o))
    if n < 0:
        raise ValueError("invalid opal / grid combination")
    out = np.zeros((n, 5), dtype=np.int64)
    if lib().orc_opal_spheres(C.byref(g), C.byref(o), _ptr(out, C.c_int64)) != 0:
        raise ValueError("orc_opal_spheres failed")
    return out


def voxelize(grid, opal, spheres=None, method="gather"):
    g, o = make_grid(grid), make_opal(opal)
    if spheres is None:
        spheres = opal_spheres(grid, opal)
    sph = np.ascontiguousarray(spheres, dtype=np.int64)
    nx, ny, nz = grid["n"]
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    fn = lib().orc_voxelize_gather if method == "gather" else lib().orc_voxelize_scatter
    if fn(C.byref(g), C.byref(o), _ptr(sph, C.c_int64), sph.shape[0], _ptr(m, C.c_uint8)) != 0:
        raise ValueError("voxelize failed")
    return m


def threads():
    return int(lib().orc_threads())


# ------------------------------------------------------------------ simulation

class OracleSim:
    """FP64 reference run of one configuration dict."""

    def __init__(self, cfg, max_steps=None):
        self.cfg = cfg
        grid = cfg["grid"]
        self.n = tuple(grid["n"])
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        mats = cfg["materials"]
        arr = (Material * len(mats))(*[make_material(m) for m in mats])
        g = make_grid(grid)
        self.max_steps = int(max_steps if max_steps is not None else cfg.get("steps", 0))
        self.h = lib().orc_create(C.byref(g), arr, len(mats), self.max_steps)
        if not self.h:
            raise ValueError("orc_create rejected the configuration")
        if cfg.get("map") is not None:
            mp = np.ascontiguousarray(cfg["map"], dtype=np.uint8)
        elif cfg.get("opal") is not None:
            mp = voxelize(grid, cfg["opal"])
        else:
            mp = np.zeros(self.n[::-1], dtype=np.uint8)
        self.map = mp
        if lib().orc_set_material_map(self.h, _ptr(mp, C.c_uint8)) != 0:
            raise ValueError("material index out of range")
        for s in cfg.get("sources", []):
            src = make_source(s)
            if lib().orc_add_source(self.h, C.byref(src)) < 0:
                raise ValueError("bad source %r" % (s,))
        self.nprobe = 0
        for p in cfg.get("probes", []):
            if lib().orc_add_probe(self.h, *[int(v) for v in p]) < 0:
                raise ValueError("bad probe %r" % (p,))
            self.nprobe += 1
        self.nflux = 0
        self.nf = []
        for f in cfg.get("flux", []):
            fr = np.ascontiguousarray(f["freqs"], dtype=np.float64)
            if lib().orc_add_flux_plane(self.h, f["k"], _ptr(fr, C.c_double), len(fr), f.get("decim", 1)) < 0:
                raise ValueError("bad flux plane %r" % (f,))
            self.nflux += 1
            self.nf.append(len(fr))
        if cfg.get("energy_interval"):
            lib().orc_set_energy_interval(self.h, int(cfg["energy_interval"]))
        for comp, arr0 in (cfg.get("init_fields") or {}).items():
            self.set_field(comp, arr0)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    @property
    def dt(self):
        return lib().orc_dt(self.h)

    @property
    def step_count(self):
        return lib().orc_step_count(self.h)

    def step(self, n):
        if lib().orc_step(self.h, int(n)) != 0:
            raise ValueError("orc_step: beyond max_steps")

    def field(self, comp):
        out = np.zeros(self.n[::-1], dtype=np.float64)
        lib().orc_get_field(self.h, int(comp), _ptr(out, C.c_double))
        return out

    def fields(self):
        return np.stack([self.field(c) for c in range(6)])

    def set_field(self, comp, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.n[::-1])
        lib().orc_set_field(self.h, int(comp), _ptr(a, C.c_double))

    def populations(self):
        out = np.zeros((4,) + self.n[::-1], dtype=np.float64)
        if lib().orc_get_populations(self.h, _ptr(out, C.c_double)) != 0:
            raise ValueError("no gain material")
        return out

    def polarization(self):
        out = np.zeros((3,) + self.n[::-1], dtype=np.float64)
        if lib().orc_get_polarization(self.h, _ptr(out, C.c_double)) != 0:
            raise ValueError("no gain material")
        return out

    def density(self):
        """Density matrix of the density-matrix gain cells, 15 planes (see
        orc_get_density)."""
        out = np.zeros((15,) + self.n[::-1], dtype=np.float64)
        if lib().orc_get_density(self.h, _ptr(out, C.c_double)) != 0:
            raise ValueError("no density-matrix gain material")
        return out

    def probe(self, pid):
        out = np.zeros(max(self.max_steps, 1), dtype=np.float64)
        n = lib().orc_get_probe(self.h, int(pid), _ptr(out, C.c_double))
        return out[:n]

    def flux(self, fid):
        T = np.zeros(max(self.max_steps, 1), dtype=np.float64)
        spec = np.zeros(max(self.nf[fid], 1), dtype=np.float64)
        n = lib().orc_get_flux(self.h, int(fid), _ptr(T, C.c_double), _ptr(spec, C.c_double))
        return T[:n], spec[: self.nf[fid]]

    def energy(self):
        out = np.zeros(self.max_steps + 1, dtype=np.float64)
        n = lib().orc_get_energy(self.h, _ptr(out, C.c_double))
        return out[:max(n, 0)]


# ------------------------------------------------------------ matter alone

def bloch_evolve(material, dt, dx, a_meters, emid, rho0, history=False):
    """Density matrix of one gain-2 cell driven by the midpoint fields emid
    (n x 3), from the 4x4 complex rho0.  Returns the final rho, and the n x 4 x 4
    history when asked."""
    m = make_material(material)
    e = np.ascontiguousarray(emid, dtype=np.float64).reshape(-1, 3)
    n = e.shape[0]
    r = np.ascontiguousarray(np.asarray(rho0, dtype=np.complex128).reshape(4, 4)).view(np.float64).copy()
    hist = np.zeros((max(n, 1), 32), dtype=np.float64) if history else None
    rc = lib().orc_bloch_evolve(C.byref(m), float(dt), float(dx), float(a_meters), n, _ptr(e, C.c_double),
                                _ptr(r, C.c_double), _ptr(hist, C.c_double) if history else None)
    if rc != 0:
        raise ValueError("invalid density-matrix material")
    out = r.view(np.complex128).reshape(4, 4)
    if history:
        return out, hist[:n].view(np.complex128).reshape(n, 4, 4)
    return out


def bloch_constants(material, dt, dx, a_meters):
    """(w0, prewarped w', kappa, 1/T1, 1/T2, pump) in normalised units."""
    m = make_material(material)
    out = np.zeros(6, dtype=np.float64)
    if lib().orc_bloch_constants(C.byref(m), float(dt), float(dx), float(a_meters), _ptr(out, C.c_double)) != 0:
        raise ValueError("invalid density-matrix material")
    return tuple(out)
