"""Thin ctypes binding of libfrt.so (include/frt.h).

Argument marshalling only: every step of the ray-tracing path runs in the
HIP library.  Arrays may be numpy (host) or torch CUDA tensors (device);
PyTorch is used only for device memory and streams.  If the library has not
been built, loading raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# FRT_LIB names another build of the library (the host-sanitized one, say)
LIB_PATH = os.environ.get("FRT_LIB") or os.path.join(PKG, "libfrt.so")

FRT_OK, FRT_EINVAL, FRT_ENOMEM, FRT_EDEVICE, FRT_EOVERFLOW, FRT_ESTATE = 0, -1, -2, -3, -4, -5
FRT_HOST, FRT_DEVICE = 0, 1
FRT_F32, FRT_F64 = 0, 1
MAX_BINS = 8

# Symbols declared in include/frt.h.
EXPORTS = ("frt_params_default", "frt_ctx_create", "frt_ctx_destroy", "frt_last_error", "frt_solve_create",
           "frt_solve_destroy", "frt_load_grid", "frt_set_opacity", "frt_load_sources", "frt_set_rotations", "frt_step",
           "frt_batch_step", "frt_sync", "frt_read_fields", "frt_read_ledger", "frt_save_state",
           "frt_load_state", "frt_mark", "frt_rewind", "frt_set_timing", "frt_read_timing",
           "frt_rotation_uniforms", "frt_batch_run", "frt_tuning_default", "frt_ctx_set_tuning",
           "frt_ctx_get_tuning", "frt_autotune", "frt_request_bytes", "frt_server_create", "frt_server_submit",
           "frt_server_poll", "frt_server_wait", "frt_server_take", "frt_server_times", "frt_server_get_stats",
           "frt_server_destroy", "frt_debug_cast", "frt_step_static", "frt_merge_uniforms",
           "frt_read_temperature", "frt_microbench", "frt_set_density", "frt_server_read_temperature")
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class FrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"frt error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("size", C.c_size_t), ("n_bins", C.c_int), ("sigma_bins", C.c_double * MAX_BINS),
                ("alpha_B", C.c_double), ("coll_ion", C.c_double), ("base_level", C.c_int),
                ("max_level", C.c_int), ("n_ray_min", C.c_double), ("flux_floor", C.c_double),
                ("max_distance_cm", C.c_double), ("c_ray_cm_s", C.c_double), ("march_precision", C.c_int),
                ("seed", C.c_uint64), ("queue_capacity", C.c_uint64), ("queue_hint", C.c_uint64),
                ("chem_iterations", C.c_int), ("opacity_mode", C.c_int), ("he_chi", C.c_double),
                ("merge", C.c_int), ("merge_level", C.c_int), ("merge_exempt", C.c_double),
                ("temperature", C.c_int), ("heat_ev", C.c_double * MAX_BINS), ("hubble_s", C.c_double),
                ("cmb_z", C.c_double), ("t_reion_k", C.c_double), ("spectral_index", C.c_double)]


class Ledger(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed_HI", C.c_double), ("absorbed_sub", C.c_double),
                ("escaped", C.c_double), ("dropped", C.c_double), ("in_flight", C.c_double),
                ("lost", C.c_double), ("crossings", C.c_uint64), ("ray_visits", C.c_uint64),
                ("splits", C.c_uint64), ("n_escaped", C.c_uint64), ("n_dropped", C.c_uint64),
                ("n_in_flight", C.c_uint64), ("rays_emitted", C.c_uint64), ("step_crossings", C.c_uint64),
                ("steps", C.c_uint64), ("err_flags", C.c_uint32), ("max_items", C.c_uint32),
                ("absorbed_front", C.c_double), ("merge_residual", C.c_double), ("merges", C.c_uint64),
                ("rays_merged", C.c_uint64), ("front_excess", C.c_double), ("heat_in", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("emit_ms", C.c_double), ("march_ms", C.c_double), ("chem_ms", C.c_double),
                ("other_ms", C.c_double), ("march_launches", C.c_uint64), ("chem_launches", C.c_uint64),
                ("steps", C.c_uint64), ("merge_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class MicrobenchResult(C.Structure):
    _fields_ = [("size", C.c_size_t), ("copy_bytes", C.c_double), ("copy_GBps", C.c_double),
                ("atomic_ops", C.c_double), ("atomic_per_s", C.c_double), ("atomic_slots", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "size"}


class Tuning(C.Structure):
    _fields_ = [("size", C.c_size_t), ("item_rays", C.c_int), ("scatter_blocks_per_cu", C.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "size"}


class Request(C.Structure):
    _fields_ = [("size", C.c_size_t), ("params", Params), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("box_cm", C.c_double), ("n_H", C.c_void_p), ("T", C.c_void_p), ("kappa_sub", C.c_void_p),
                ("x_HI0", C.c_void_p), ("n_src", C.c_int), ("pos_cm", C.c_void_p), ("ndot_bins", C.c_void_p),
                ("rotation_steps", C.c_int), ("rotation_uniforms", C.c_void_p), ("n_steps", C.c_int),
                ("dt_s", C.c_double), ("ptr_kind", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("ticks", C.c_uint64), ("solve_steps", C.c_uint64), ("max_in_flight", C.c_uint32),
                ("bytes_in_use", C.c_uint64), ("peak_bytes", C.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# Device memory hooks of a context (include/frt.h, frt_alloc_fn / frt_free_fn).
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator on
    `device`: the library's buffers then count in torch.cuda.memory_allocated()
    and reuse the cache.  Keeps its callbacks alive while any block is out."""

    def __init__(self, device: int = 0):
        import torch

        self.device = device
        self.live = {}

        def alloc(nbytes, user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
            except RuntimeError:
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def free(ptr, user):
            if self.live.pop(ptr, None) is not None:
                torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = ALLOC_FN(alloc)
        self.free_fn = FREE_FN(free)

    def bytes_out(self) -> int:
        return sum(self.live.values())


# allocators whose blocks the library may still hand back (a solve can
# outlive its Context object on the Python side)
_ALLOCATORS = []

_lib = None


def lib():
    """Load libfrt.so (built by paper_2409_04521_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2409_04521_amd.build)")
        try:
            # PyTorch brings a HIP runtime of its own: loaded first, it is the
            # one the library binds to, so tensors, streams and allocator
            # hooks are shared (loaded after the library's, torch finds no GPU)
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.frt_last_error.restype = C.c_char_p
        L.frt_params_default.argtypes = [C.POINTER(Params)]
        L.frt_ctx_create.argtypes = [C.c_int, ALLOC_FN, FREE_FN, vp, C.POINTER(vp)]
        L.frt_ctx_destroy.argtypes = [vp]
        L.frt_solve_create.argtypes = [vp, C.POINTER(Params), vp, C.POINTER(vp)]
        L.frt_solve_destroy.argtypes = [vp]
        L.frt_load_grid.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, vp, vp, vp, vp, C.c_int]
        L.frt_load_sources.argtypes = [vp, C.c_int, vp, vp, C.c_int]
        L.frt_set_opacity.argtypes = [vp, vp, C.c_int]
        L.frt_set_density.argtypes = [vp, vp, C.c_int]
        L.frt_set_rotations.argtypes = [vp, C.c_int, vp]
        L.frt_step.argtypes = [vp, C.c_double]
        L.frt_step_static.argtypes = [vp, C.c_double]
        L.frt_batch_step.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_double)]
        L.frt_sync.argtypes = [vp]
        L.frt_read_fields.argtypes = [vp, vp, vp, C.c_int]
        L.frt_read_ledger.argtypes = [vp, C.POINTER(Ledger)]
        L.frt_read_temperature.argtypes = [vp, vp, C.c_int]
        L.frt_microbench.argtypes = [vp, C.c_size_t, C.c_size_t, C.POINTER(MicrobenchResult)]
        L.frt_save_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.frt_load_state.argtypes = [vp, vp, C.c_size_t]
        L.frt_mark.argtypes = [vp]
        L.frt_rewind.argtypes = [vp]
        L.frt_set_timing.argtypes = [vp, C.c_int]
        L.frt_read_timing.argtypes = [vp, C.POINTER(Timing)]
        L.frt_rotation_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(C.c_double)]
        L.frt_merge_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(C.c_double)]
        L.frt_batch_run.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_double), C.c_int, C.c_int]
        L.frt_tuning_default.argtypes = [C.POINTER(Tuning)]
        L.frt_ctx_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.frt_ctx_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.frt_autotune.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_double), C.POINTER(Tuning)]
        L.frt_request_bytes.argtypes = [C.POINTER(Request), C.POINTER(C.c_size_t)]
        L.frt_server_create.argtypes = [vp, C.c_size_t, C.c_int, C.POINTER(vp)]
        L.frt_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.frt_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int)]
        L.frt_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(C.c_int)]
        L.frt_server_take.argtypes = [vp, C.c_uint64, vp, C.POINTER(Ledger)]
        L.frt_server_times.argtypes = [vp, C.c_uint64, C.POINTER(C.c_double)]
        L.frt_server_read_temperature.argtypes = [vp, C.c_uint64, vp]
        L.frt_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.frt_server_destroy.argtypes = [vp]
        L.frt_debug_cast.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.c_double, vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_uint64)]
        _lib = L
    return _lib


def _check(rc):
    if rc != FRT_OK:
        raise FrtError(rc, lib().frt_last_error().decode())


def _ptr(a):
    """(address, kind, keepalive) for a numpy array or torch tensor; None -> NULL."""
    if a is None:
        return None, FRT_HOST, None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            a = np.ascontiguousarray(a)
        return a.ctypes.data, FRT_HOST, a
    import torch  # device tensors

    if isinstance(a, torch.Tensor):
        t = a.contiguous()
        return t.data_ptr(), (FRT_DEVICE if t.is_cuda else FRT_HOST), t
    raise TypeError(f"unsupported array type {type(a)}")


def params_default() -> Params:
    p = Params()
    _check(lib().frt_params_default(C.byref(p)))
    return p


def rotation_uniforms(seed: int, step: int, src: int):
    out = (C.c_double * 3)()
    _check(lib().frt_rotation_uniforms(seed, step, src, out))
    return np.array(out[:])


def merge_uniforms(seed: int, step: int, cell: int):
    out = (C.c_double * 3)()
    _check(lib().frt_merge_uniforms(seed, step, cell, out))
    return np.array(out[:])


class Context:
    """frt_ctx on HIP device `device`; allocator=None uses hipMalloc, a
    TorchAllocator (or anything with alloc_fn / free_fn ctypes callbacks)
    routes the library's device memory through it."""

    def __init__(self, device: int = 0, allocator=None):
        h = C.c_void_p()
        self.allocator = allocator
        if allocator is None:
            _check(lib().frt_ctx_create(device, ALLOC_FN(), FREE_FN(), None, C.byref(h)))
        else:
            _ALLOCATORS.append(allocator)
            _check(lib().frt_ctx_create(device, allocator.alloc_fn, allocator.free_fn, None, C.byref(h)))
        self.h = h
        self.device = device

    def tuning(self) -> dict:
        t = Tuning()
        t.size = C.sizeof(Tuning)
        _check(lib().frt_ctx_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, item_rays=None, scatter_blocks_per_cu=None):
        t = Tuning()
        t.size = C.sizeof(Tuning)
        _check(lib().frt_ctx_get_tuning(self.h, C.byref(t)))
        if item_rays is not None:
            t.item_rays = item_rays
        if scatter_blocks_per_cu is not None:
            t.scatter_blocks_per_cu = scatter_blocks_per_cu
        _check(lib().frt_ctx_set_tuning(self.h, C.byref(t)))

    def close(self):
        if self.h:
            lib().frt_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solve:
    """One RT problem resident on the device (frt_solve)."""

    def __init__(self, ctx: Context, *, sigma_bins, alpha_B=2.59e-13, coll_ion=0.0, base_level=0,
                 max_level=12, n_ray_min=1.0, flux_floor=0.0, max_distance_cm=0.0, c_ray=2.99792458e10,
                 precision="f32", seed=0, queue_capacity=0, queue_hint=0, chem_iterations=0, opacity_mode=0,
                 he_chi=0.0, merge=False, merge_level=0, merge_exempt=4.0, temperature=False, heat_ev=None,
                 hubble_s=0.0, cmb_z=-1.0, t_reion=2e4, spectral_index=1.5, stream=None):
        p = params_default()
        sig = list(sigma_bins)
        p.n_bins = len(sig)
        for i, s in enumerate(sig):
            p.sigma_bins[i] = s
        p.alpha_B, p.coll_ion = alpha_B, coll_ion
        p.base_level, p.max_level, p.n_ray_min = base_level, max_level, n_ray_min
        p.flux_floor, p.max_distance_cm = flux_floor, max_distance_cm
        p.c_ray_cm_s = c_ray if c_ray is not None else math.inf
        p.march_precision = FRT_F64 if precision == "f64" else FRT_F32
        p.seed, p.queue_capacity, p.queue_hint = seed, queue_capacity, queue_hint
        p.chem_iterations = chem_iterations
        p.opacity_mode, p.he_chi = opacity_mode, he_chi
        p.merge, p.merge_level, p.merge_exempt = int(bool(merge)), merge_level, merge_exempt
        p.temperature, p.hubble_s, p.cmb_z = int(bool(temperature)), hubble_s, cmb_z
        p.t_reion_k, p.spectral_index = t_reion, spectral_index
        for i, e in enumerate(heat_ev if heat_ev is not None else []):
            p.heat_ev[i] = e
        self.ctx = ctx
        self.params = p
        self.n_bins = p.n_bins
        self.shape = None
        h = C.c_void_p()
        _check(lib().frt_solve_create(ctx.h, C.byref(p), stream, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().frt_solve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_grid(self, n_H, box_cm, kappa=None, x_HI0=None, T=None):
        shape = tuple(n_H.shape)
        nz, ny, nx = shape
        pn, kind, k1 = _ptr(n_H)
        pk, _, k2 = _ptr(kappa)
        px, _, k3 = _ptr(x_HI0)
        pt, _, k4 = _ptr(T)
        _check(lib().frt_load_grid(self.h, nx, ny, nz, box_cm, pn, pt, pk, px, kind))
        self.shape = shape

    def set_opacity(self, kappa):
        pk, kind, k = _ptr(kappa)
        _check(lib().frt_set_opacity(self.h, pk, kind))

    def set_density(self, n_H):
        if isinstance(n_H, np.ndarray):
            n_H = np.ascontiguousarray(n_H, dtype=np.float32)
        pn, kind, k = _ptr(n_H)
        _check(lib().frt_set_density(self.h, pn, kind))

    def load_sources(self, pos_cm, ndot_bins):
        pos = np.ascontiguousarray(pos_cm, dtype=np.float64).reshape(-1, 3) if isinstance(pos_cm, np.ndarray) else pos_cm
        nd = np.ascontiguousarray(ndot_bins, dtype=np.float64) if isinstance(ndot_bins, np.ndarray) else ndot_bins
        n = int(pos.shape[0])
        pp, kind, k1 = _ptr(pos)
        pd, _, k2 = _ptr(nd)
        _check(lib().frt_load_sources(self.h, n, pp, pd, kind))

    def set_rotations(self, uniforms):
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        _check(lib().frt_set_rotations(self.h, int(u.shape[0]), u.ctypes.data))

    def step(self, dt_s: float):
        _check(lib().frt_step(self.h, float(dt_s)))

    def step_static(self, dt_s: float):
        """One step that allocates no device memory (frt_step_static)."""
        _check(lib().frt_step_static(self.h, float(dt_s)))

    def sync(self):
        _check(lib().frt_sync(self.h))

    def fields(self):
        n = int(np.prod(self.shape))
        x = np.empty(n)
        g = np.empty(n, dtype=np.float32)
        _check(lib().frt_read_fields(self.h, x.ctypes.data, g.ctypes.data, FRT_HOST))
        return x.reshape(self.shape), g.reshape(self.shape)

    def fields_into(self, x_dev=None, gamma_dev=None):
        """Copy fields into device tensors (no host round trip)."""
        px, kind, k1 = _ptr(x_dev)
        pg, kind2, k2 = _ptr(gamma_dev)
        _check(lib().frt_read_fields(self.h, px, pg, FRT_DEVICE))

    def ledger(self) -> dict:
        L = Ledger()
        _check(lib().frt_read_ledger(self.h, C.byref(L)))
        return L.as_dict()

    def temperature(self):
        """The gas temperature (K) of every cell."""
        t = np.empty(int(np.prod(self.shape)))
        _check(lib().frt_read_temperature(self.h, t.ctypes.data, FRT_HOST))
        return t.reshape(self.shape)

    def debug_cast(self, origin_cm, direction, N_bins, dt_s=1.0):
        """March one packet through the current opacity (frt_debug_cast).
        Returns (absorbed photons, escaped photons, crossings, rate field)."""
        o = (C.c_double * 3)(*[float(v) for v in origin_cm])
        d = (C.c_double * 3)(*[float(v) for v in direction])
        N = (C.c_double * MAX_BINS)(*[float(v) for v in N_bins])
        g = np.zeros(int(np.prod(self.shape)), dtype=np.float32)
        ab, es, nc = C.c_double(), C.c_double(), C.c_uint64()
        _check(lib().frt_debug_cast(self.h, o, d, N, float(dt_s), g.ctypes.data, FRT_HOST, C.byref(ab),
                                    C.byref(es), C.byref(nc)))
        return ab.value, es.value, int(nc.value), g.reshape(self.shape)

    def mark(self):
        _check(lib().frt_mark(self.h))

    def rewind(self):
        _check(lib().frt_rewind(self.h))

    def set_timing(self, on: bool = True):
        _check(lib().frt_set_timing(self.h, 1 if on else 0))

    def timing(self) -> dict:
        t = Timing()
        _check(lib().frt_read_timing(self.h, C.byref(t)))
        return t.as_dict()

    def save(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().frt_save_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().frt_save_state(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().frt_load_state(self.h, buf, len(blob)))


def _group(solves, dts):
    arr = (C.c_void_p * len(solves))(*[s.h for s in solves])
    d = (C.c_double * len(solves))(*[float(x) for x in dts])
    return arr, d


def batch_step(solves, dts):
    arr, d = _group(solves, dts)
    _check(lib().frt_batch_step(arr, len(solves), d))


def batch_run(solves, dts, n_steps: int, graph: bool = True, check_every: int = 1):
    """n_steps steps of every solve, one captured HIP graph replayed per step
    (graph=True; the queue counters are read back after every `check_every`
    replays) or launched step by step."""
    arr, d = _group(solves, dts)
    _check(lib().frt_batch_run(arr, len(solves), d, int(n_steps), int(check_every) if graph else 0))


def microbench(ctx: Context, copy_bytes: int = 2 << 30, atomic_slots: int = 1 << 24) -> dict:
    """Achievable HBM bandwidth (streaming copy) and random-address FP32
    atomic rate of the context's device (frt_microbench)."""
    r = MicrobenchResult()
    r.size = C.sizeof(MicrobenchResult)
    _check(lib().frt_microbench(ctx.h, int(copy_bytes), int(atomic_slots), C.byref(r)))
    return r.as_dict()


def autotune(solves, dts) -> dict:
    """Time the candidate launch shapes on one step of these solves (their
    state is restored), set the fastest on their context and return it."""
    arr, d = _group(solves, dts)
    t = Tuning()
    t.size = C.sizeof(Tuning)
    _check(lib().frt_autotune(arr, len(solves), d, C.byref(t)))
    return t.as_dict()


def _params_for(prob, precision="f32", **kw) -> Params:
    p = params_default()
    sig = list(prob.sigma_bins)
    p.n_bins = len(sig)
    for i, v in enumerate(sig):
        p.sigma_bins[i] = v
    p.alpha_B, p.coll_ion = prob.alpha_B, prob.coll_ion
    p.base_level, p.max_level, p.n_ray_min = prob.base_level, prob.max_level, prob.n_ray_min
    p.flux_floor, p.max_distance_cm = prob.flux_floor, prob.max_dist_cm
    p.c_ray_cm_s = prob.c_ray if prob.c_ray is not None else math.inf
    p.march_precision = FRT_F64 if precision == "f64" else FRT_F32
    p.seed = prob.seed
    p.queue_capacity = kw.get("queue_capacity", 0)
    p.queue_hint = kw.get("queue_hint", 0)
    p.chem_iterations = getattr(prob, "chem_iterations", 0)
    p.opacity_mode = getattr(prob, "opacity_mode", 0)
    p.he_chi = getattr(prob, "he_chi", 0.0)
    p.merge = int(bool(getattr(prob, "merge", False)))
    p.merge_level = getattr(prob, "merge_level", 0)
    p.merge_exempt = getattr(prob, "merge_exempt", 4.0)
    p.temperature = int(bool(getattr(prob, "temperature", False)))
    for i, e in enumerate(getattr(prob, "heat_ev", None) if getattr(prob, "heat_ev", None) is not None else []):
        p.heat_ev[i] = e
    p.hubble_s = getattr(prob, "hubble_s", 0.0)
    p.cmb_z = getattr(prob, "cmb_z", -1.0)
    p.t_reion_k = getattr(prob, "t_reion", 2e4)
    p.spectral_index = getattr(prob, "spectral_index", 1.5)
    return p


def request_from_problem(prob, n_steps: int, precision="f32", use_table=True, **kw):
    """(frt_request, keepalive) for a workloads.Problem: host arrays, the
    problem's parameters and, with use_table, its rotation uniforms."""
    import numpy as np
    r = Request()
    r.size = C.sizeof(Request)
    r.params = _params_for(prob, precision, **kw)
    nz, ny, nx = prob.shape
    r.nx, r.ny, r.nz = nx, ny, nz
    r.box_cm = prob.dx_cm * nx
    keep = []

    def host(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    r.n_H = host(prob.n_H, np.float32)
    r.T = host(prob.T, np.float32)
    r.kappa_sub = host(prob.kappa, np.float32)
    r.x_HI0 = host(prob.x_HI0, np.float64)
    r.n_src = prob.n_src
    r.pos_cm = host(prob.src_pos_cm, np.float64)
    r.ndot_bins = host(prob.ndot_bins, np.float64)
    if use_table and prob.n_src > 0 and n_steps > 0:
        from .workloads import rotation_table
        r.rotation_steps = n_steps
        r.rotation_uniforms = host(rotation_table(prob.seed, 0, n_steps, prob.n_src), np.float64)
    r.n_steps = n_steps
    r.dt_s = prob.dt_s
    r.ptr_kind = FRT_HOST
    return r, keep


def request_bytes(prob, n_steps: int, **kw) -> int:
    r, keep = request_from_problem(prob, n_steps, **kw)
    b = C.c_size_t()
    _check(lib().frt_request_bytes(C.byref(r), C.byref(b)))
    return b.value


class Server:
    """Continuous-batching server (frt_server): admits solves by memory
    budget and slots, steps every admitted solve once per tick."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 64):
        h = C.c_void_p()
        _check(lib().frt_server_create(ctx.h, int(budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self.open = True
        self.ctx = ctx
        self.shapes = {}

    def submit(self, prob, n_steps: int, **kw) -> int:
        r, keep = request_from_problem(prob, n_steps, **kw)
        rid = C.c_uint64()
        _check(lib().frt_server_submit(self.h, C.byref(r), C.byref(rid)))
        self.shapes[rid.value] = prob.shape
        return rid.value

    def poll(self, rid: int) -> int:
        st = C.c_int()
        _check(lib().frt_server_poll(self.h, rid, C.byref(st)))
        return st.value

    def wait(self, rid: int, timeout_s: float = -1.0) -> int:
        st = C.c_int()
        _check(lib().frt_server_wait(self.h, rid, float(timeout_s), C.byref(st)))
        return st.value

    def take(self, rid: int):
        """(x_HI, ledger dict) of a finished request."""
        import numpy as np
        x = np.empty(self.shapes[rid], dtype=np.float64)
        L = Ledger()
        _check(lib().frt_server_take(self.h, rid, x.ctypes.data, C.byref(L)))
        self.shapes.pop(rid, None)
        return x, L.as_dict()

    def temperature(self, rid: int):
        """T (K) of a finished request that evolved its temperature; before take()."""
        import numpy as np
        t = np.empty(self.shapes[rid], dtype=np.float64)
        _check(lib().frt_server_read_temperature(self.h, rid, t.ctypes.data))
        return t

    def times(self, rid: int):
        t = (C.c_double * 3)()
        _check(lib().frt_server_times(self.h, rid, t))
        return tuple(t)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().frt_server_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "open", False):
            lib().frt_server_destroy(self.h)
            self.open = False
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_from_problem(ctx: Context, prob, precision="f32", use_table=True, **kw) -> Solve:
    """Create and load a Solve from a workloads.Problem."""
    s = Solve(ctx, sigma_bins=prob.sigma_bins, alpha_B=prob.alpha_B, coll_ion=prob.coll_ion,
              base_level=prob.base_level, max_level=prob.max_level, n_ray_min=prob.n_ray_min,
              flux_floor=prob.flux_floor, max_distance_cm=prob.max_dist_cm, c_ray=prob.c_ray,
              precision=precision, seed=prob.seed, chem_iterations=getattr(prob, "chem_iterations", 0),
              opacity_mode=getattr(prob, "opacity_mode", 0), he_chi=getattr(prob, "he_chi", 0.0),
              merge=getattr(prob, "merge", False), merge_level=getattr(prob, "merge_level", 0),
              merge_exempt=getattr(prob, "merge_exempt", 4.0), temperature=getattr(prob, "temperature", False),
              heat_ev=getattr(prob, "heat_ev", None), hubble_s=getattr(prob, "hubble_s", 0.0),
              cmb_z=getattr(prob, "cmb_z", -1.0), t_reion=getattr(prob, "t_reion", 2e4),
              spectral_index=getattr(prob, "spectral_index", 1.5), **kw)
    nz, ny, nx = prob.shape
    s.load_grid(prob.n_H, prob.dx_cm * nx, kappa=prob.kappa, x_HI0=prob.x_HI0, T=prob.T)
    s.load_sources(prob.src_pos_cm, prob.ndot_bins)
    if use_table and prob.n_src > 0:
        from .workloads import rotation_table
        s.set_rotations(rotation_table(prob.seed, 0, prob.n_steps, prob.n_src))
    return s
