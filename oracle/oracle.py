"""ctypes wrapper of the FP64 CPU oracle (oracle/frt_oracle.c).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It imports
nothing from the GPU package; both sides receive the same seeded inputs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "frt_oracle.c")
# FRT_ORACLE_LIB names another build of the same source (the sanitizer
# build of the CPU tests, say)
LIB = os.environ.get("FRT_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
MAX_BINS = 8
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, IEEE double (no fast-math);
    with sanitize=True an AddressSanitizer + UBSan build of the same source
    (into `out`)."""
    out = out or LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        opt = SANITIZE if sanitize else ["-O2"]
        subprocess.check_call(["gcc", "-std=c11", *opt, "-fno-fast-math", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", "-D_DEFAULT_SOURCE",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("n_bins", C.c_int), ("sigma", C.c_double * MAX_BINS),
                ("alpha_B", C.c_double), ("coll_ion", C.c_double),
                ("base_level", C.c_int), ("max_level", C.c_int), ("n_ray_min", C.c_double),
                ("flux_floor", C.c_double), ("max_dist", C.c_double), ("c_ray", C.c_double),
                ("n_chunks", C.c_int), ("chem_iterations", C.c_int), ("opacity_mode", C.c_int),
                ("he_chi", C.c_double), ("merge", C.c_int), ("merge_level", C.c_int),
                ("merge_exempt", C.c_double), ("temperature", C.c_int), ("heat_ev", C.c_double * MAX_BINS),
                ("hubble", C.c_double), ("cmb_z", C.c_double), ("t_reion", C.c_double),
                ("spectral_index", C.c_double)]


class Ledger(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed_HI", C.c_double), ("absorbed_sub", C.c_double),
                ("escaped", C.c_double), ("dropped", C.c_double), ("in_flight", C.c_double),
                ("crossings", C.c_longlong), ("rays_emitted", C.c_longlong), ("splits", C.c_longlong),
                ("n_escaped", C.c_longlong), ("n_dropped", C.c_longlong), ("n_in_flight", C.c_longlong),
                ("absorbed_front", C.c_double), ("merge_residual", C.c_double), ("merges", C.c_longlong),
                ("rays_merged", C.c_longlong), ("front_excess", C.c_double), ("heat_in", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_kappa.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_set_sources.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_double, dp, C.c_void_p, C.c_int]
        L.orc_flight_dump.restype = C.c_longlong
        L.orc_flight_dump.argtypes = [C.c_void_p, C.c_void_p, C.c_longlong]
        L.orc_merge_now.argtypes = [C.c_void_p, dp]
        L.orc_read.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_ledger_get.argtypes = [C.c_void_p, C.POINTER(Ledger)]
        L.orc_last_crossings.restype = C.c_longlong
        L.orc_last_crossings.argtypes = [C.c_void_p]
        L.orc_state_bytes.restype = C.c_longlong
        L.orc_state_bytes.argtypes = [C.c_void_p]
        L.orc_save.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_load.argtypes = [C.c_void_p, C.c_void_p]
        L.healpix_nest_center.argtypes = [C.c_int, C.c_longlong, dp]
        L.healpix_nest_pixel.restype = C.c_longlong
        L.healpix_nest_pixel.argtypes = [C.c_int, dp]
        L.shoemake_rotation.argtypes = [dp, dp]
        L.split_radius.restype = C.c_double
        L.split_radius.argtypes = [C.c_double, C.c_int, C.c_double]
        L.chemistry_be.restype = C.c_double
        L.chemistry_be.argtypes = [C.c_double] * 6
        L.chemistry_avg.restype = C.c_double
        L.chemistry_avg.argtypes = [C.c_double] * 6 + [C.POINTER(C.c_double)]
        L.orc_flight_radii.restype = C.c_longlong
        L.orc_flight_radii.argtypes = [C.c_void_p, C.c_void_p, C.c_longlong]
        L.orc_chemistry_field.argtypes = [C.c_longlong, dp, dp, dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_debug_transmit.restype = C.c_int
        L.orc_debug_transmit.argtypes = [C.c_void_p, dp, dp, dp, C.c_double, dp, dp, C.c_void_p]
        L.orc_rates.argtypes = [C.c_double, dp]
        L.orc_set_temperature.argtypes = [C.c_void_p, dp]
        L.orc_read_temperature.argtypes = [C.c_void_p, dp]
        L.temperature_update.restype = C.c_double
        L.temperature_update.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double]
        L.orc_set_density.restype = C.c_int
        L.orc_set_density.argtypes = [C.c_void_p, C.c_void_p]
        L.reion_heat_per_recombination.restype = C.c_double
        L.reion_heat_per_recombination.argtypes = [C.c_double]
        L.ionized_temperature_update.restype = C.c_double
        L.ionized_temperature_update.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double,
                                                 C.c_double]
        _lib = L
    return _lib


# ------------------------------------------------------------- primitives
def healpix_center(level: int, pix: int) -> np.ndarray:
    out = np.zeros(3)
    lib().healpix_nest_center(level, pix, out)
    return out


def healpix_centers(level: int) -> np.ndarray:
    n = 12 * 4 ** level
    return np.stack([healpix_center(level, p) for p in range(n)])


def healpix_pixel(level: int, v) -> int:
    return int(lib().healpix_nest_pixel(level, np.ascontiguousarray(v, dtype=np.float64)))


def rotation(u) -> np.ndarray:
    R = np.zeros(9)
    lib().shoemake_rotation(np.ascontiguousarray(u, dtype=np.float64), R)
    return R.reshape(3, 3)


def split_radius(dx: float, level: int, n_ray_min: float) -> float:
    return float(lib().split_radius(dx, level, n_ray_min))


def chemistry(x, gamma, nH, alpha, coll, dt) -> float:
    return float(lib().chemistry_be(x, gamma, nH, alpha, coll, dt))


def chemistry_field(x, gamma, nH, alpha, coll, dt) -> np.ndarray:
    """Backward-Euler update of whole fields (arrays of one shape)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(x.shape)
    n = np.ascontiguousarray(nH, dtype=np.float64).reshape(x.shape)
    out = np.empty_like(x)
    lib().orc_chemistry_field(x.size, x.reshape(-1), g.reshape(-1), n.reshape(-1), alpha, coll, dt, out.reshape(-1))
    return out


def chemistry_avg(x0, gamma, ne, alpha, coll, dt):
    """(<x>, x(dt)) of the time-averaged update at fixed n_e."""
    xe = C.c_double(0.0)
    xa = lib().chemistry_avg(x0, gamma, ne, alpha, coll, dt, C.byref(xe))
    return float(xa), float(xe.value)


def rates(T: float) -> dict:
    """The temperature-dependent rates of pure H at T (K): alpha_B, C_HI and
    alpha_A (cm^3/s) and the cooling coefficients (erg cm^3/s)."""
    out = np.zeros(7)
    lib().orc_rates(float(T), out)
    return dict(zip(("alpha_B", "coll_ion", "rec_cool", "ci_cool", "ce_cool", "ff_cool", "alpha_A"), out))


def reion_heat_per_recombination(spectral_index: float) -> float:
    """Photo-heating per recombination of ionized gas in photo-ionization
    equilibrium under a power law of this index cut at 4 Ryd, erg."""
    return float(lib().reion_heat_per_recombination(float(spectral_index)))


def ionized_temperature(T, nH, gamma, dt, spectral_index=1.5, hubble_s=0.0, cmb_z=-1.0) -> float:
    """One step of the ionized gas's temperature in the Generalized Opacity
    Mode at fixed n_H and Gamma."""
    P = Params()
    P.temperature, P.opacity_mode, P.spectral_index, P.hubble, P.cmb_z = 1, 1, spectral_index, hubble_s, cmb_z
    return float(lib().ionized_temperature_update(C.byref(P), float(T), float(nH), float(gamma), float(dt)))


# ------------------------------------------------------------- the solver
class Oracle:
    """One RT problem on the CPU: grid, sources, carried packets, ledger."""

    def __init__(self, shape, dx_cm, sigma_bins, alpha_B, n_H, kappa=None, x_HI0=None,
                 coll_ion=0.0, base_level=0, max_level=12, n_ray_min=1.0, flux_floor=0.0,
                 max_dist_cm=0.0, c_ray=np.inf, n_chunks=16, chem_iterations=0, opacity_mode=0, he_chi=0.0,
                 merge=False, merge_level=0, merge_exempt=0.0, temperature=False, heat_ev=None, hubble_s=0.0,
                 cmb_z=-1.0, T0=None, t_reion=2e4, spectral_index=1.5):
        nz, ny, nx = shape
        sig = list(sigma_bins)
        P = Params()
        P.nx, P.ny, P.nz, P.dx = nx, ny, nz, dx_cm
        P.n_bins = len(sig)
        for i, s in enumerate(sig):
            P.sigma[i] = s
        P.alpha_B, P.coll_ion = alpha_B, coll_ion
        P.base_level, P.max_level, P.n_ray_min = base_level, max_level, n_ray_min
        P.flux_floor, P.max_dist, P.c_ray, P.n_chunks = flux_floor, max_dist_cm, c_ray, n_chunks
        P.chem_iterations = chem_iterations
        P.opacity_mode, P.he_chi = opacity_mode, he_chi
        P.merge, P.merge_level, P.merge_exempt = int(bool(merge)), merge_level, merge_exempt
        P.temperature, P.hubble, P.cmb_z = int(bool(temperature)), hubble_s, cmb_z
        P.t_reion, P.spectral_index = t_reion, spectral_index
        for i, e in enumerate(heat_ev if heat_ev is not None else []):
            P.heat_ev[i] = e
        self.P = P
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        self.n_bins = len(sig)
        self._nH = np.ascontiguousarray(n_H, dtype=np.float32).reshape(-1)
        self._kap = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float32).reshape(-1)
        self._x0 = None if x_HI0 is None else np.ascontiguousarray(x_HI0, dtype=np.float64).reshape(-1)
        assert self._nH.size == self.ncell
        self.h = lib().orc_create(C.byref(P), self._nH.ctypes.data,
                                  None if self._kap is None else self._kap.ctypes.data,
                                  None if self._x0 is None else self._x0.ctypes.data)
        if not self.h:
            raise ValueError("oracle: invalid parameters")
        self.n_src = 0
        if T0 is not None:
            self.set_temperature(T0)

    def set_temperature(self, T):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(T, dtype=np.float64), self.shape)).reshape(-1)
        lib().orc_set_temperature(self.h, t)

    def temperature(self):
        t = np.empty(self.ncell)
        lib().orc_read_temperature(self.h, t)
        return t.reshape(self.shape)

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_kappa(self, kappa):
        self._kap = np.ascontiguousarray(kappa, dtype=np.float32).reshape(-1)
        assert self._kap.size == self.ncell
        lib().orc_set_kappa(self.h, self._kap.ctypes.data)

    def set_density(self, n_H):
        self._nH = np.ascontiguousarray(n_H, dtype=np.float32).reshape(-1)
        assert self._nH.size == self.ncell
        if lib().orc_set_density(self.h, self._nH.ctypes.data) != 0:
            raise ValueError("oracle: the mean density must be > 0")

    def set_sources(self, pos_cm, ndot_bins):
        pos = np.ascontiguousarray(pos_cm, dtype=np.float64).reshape(-1, 3)
        nd = np.ascontiguousarray(ndot_bins, dtype=np.float64).reshape(pos.shape[0], self.n_bins)
        self.n_src = pos.shape[0]
        if lib().orc_set_sources(self.h, self.n_src, pos.reshape(-1), nd.reshape(-1)) != 0:
            raise MemoryError("oracle: set_sources")

    def step(self, dt_s, uniforms, threads=None, merge_uniforms=None):
        """One step; uniforms: three per source for the sphere rotations;
        merge_uniforms: three per cell for the merging spheres (required
        when merging)."""
        u = np.ascontiguousarray(uniforms, dtype=np.float64).reshape(-1)
        assert u.size == 3 * self.n_src
        um = None
        if self.P.merge:
            assert merge_uniforms is not None, "merging needs the cells' sphere uniforms"
            um = np.ascontiguousarray(merge_uniforms, dtype=np.float64).reshape(-1)
            assert um.size == 3 * self.ncell
        if threads is None:
            # the host's share of cores where a launcher states it, else all
            threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count() or 1
        if lib().orc_step(self.h, dt_s, u if u.size else np.zeros(3), None if um is None else um.ctypes.data,
                          int(threads)) != 0:
            raise MemoryError("oracle: step")

    def fields(self):
        x = np.empty(self.ncell)
        g = np.empty(self.ncell)
        lib().orc_read(self.h, x.ctypes.data, g.ctypes.data)
        return x.reshape(self.shape), g.reshape(self.shape)

    def ledger(self) -> dict:
        L = Ledger()
        lib().orc_ledger_get(self.h, C.byref(L))
        return L.as_dict()

    def flight_radii(self) -> np.ndarray:
        """Distances from their sources (cm) of the packets carried into the
        next step."""
        n = int(lib().orc_flight_radii(self.h, None, 0))
        out = np.empty(max(n, 1))
        lib().orc_flight_radii(self.h, out.ctypes.data, n)
        return out[:n]

    def flight(self) -> dict:
        """The carried packets: r, origin (n, 3), dir (n, 3), level, pixel
        and photons per bin (n, n_bins)."""
        w = 9 + self.n_bins
        n = int(lib().orc_flight_dump(self.h, None, 0))
        a = np.empty((max(n, 1), w))
        lib().orc_flight_dump(self.h, a.ctypes.data, n)
        a = a[:n]
        return {"r": a[:, 0], "origin": a[:, 1:4], "dir": a[:, 4:7], "level": a[:, 7].astype(int),
                "pix": a[:, 8].astype(np.int64), "N": a[:, 9:]}

    def merge_now(self, merge_uniforms):
        """Merge the carried packets as the end of a step does."""
        um = np.ascontiguousarray(merge_uniforms, dtype=np.float64).reshape(-1)
        assert um.size == 3 * self.ncell
        if lib().orc_merge_now(self.h, um) != 0:
            raise MemoryError("oracle: merge")

    def last_crossings(self) -> int:
        return int(lib().orc_last_crossings(self.h))

    def save(self) -> bytes:
        n = int(lib().orc_state_bytes(self.h))
        buf = C.create_string_buffer(n)
        lib().orc_save(self.h, buf)
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        if lib().orc_load(self.h, buf) != 0:
            raise ValueError("oracle: state does not match this problem")

    def transmit(self, origin_cm, direction, N_bins, dt_s=1.0, heat=False):
        """March one ray (no split, floor or cap) through the current field.
        Returns (photons left per bin when it leaves the box, Gamma field,
        crossings), and with heat=True also the photo-heating field (eV per
        cell, heat_ev per photon of each bin that HI absorbs)."""
        g = np.zeros(self.ncell)
        out = np.zeros(MAX_BINS)
        N = np.zeros(MAX_BINS)
        N[: self.n_bins] = N_bins
        h = np.zeros(self.ncell) if heat else None
        nc = lib().orc_debug_transmit(self.h, np.ascontiguousarray(origin_cm, dtype=np.float64),
                                      np.ascontiguousarray(direction, dtype=np.float64), N, dt_s, g, out,
                                      None if h is None else h.ctypes.data)
        if heat:
            return out[: self.n_bins], g.reshape(self.shape), nc, h.reshape(self.shape)
        return out[: self.n_bins], g.reshape(self.shape), nc
