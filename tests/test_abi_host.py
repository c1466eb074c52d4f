"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/frt.h declares, its host-side rotation generator equals the input
module's, it fails loudly without a GPU, and the Python binding marshals
every call (exercised against a stub of the library)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "frt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(frt_\w+)\s*\(", src, re.M)))


def test_header_declares_what_binding_lists():
    assert _declared() == sorted(frt.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = frt.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_params_default_and_struct_size():
    p = frt.params_default()
    assert p.size == C.sizeof(frt.Params)
    assert p.n_bins == 1 and p.sigma_bins[0] == 6.3e-18 and p.max_level == 12
    assert p.c_ray_cm_s == 2.99792458e10
    assert p.temperature == 0 and p.cmb_z == -1.0 and p.t_reion_k == 2e4 and p.spectral_index == 1.5


@pytest.mark.parametrize("seed,step,src", [(0, 0, 0), (7, 3, 11), (2 ** 40 + 5, 99, 1999)])
def test_library_generator_matches_inputs_module(seed, step, src):
    assert np.array_equal(frt.rotation_uniforms(seed, step, src), W.rotation_uniforms(seed, step, src + 1)[src])


@pytest.mark.parametrize("seed,step,cell", [(0, 0, 0), (21, 2, 13823), (2 ** 40 + 5, 99, 16777215)])
def test_library_merge_generator_matches_inputs_module(seed, step, cell):
    assert np.array_equal(frt.merge_uniforms(seed, step, cell), W.merge_uniforms(seed, step, cell + 1)[cell])


def test_no_device_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(frt.FrtError) as e:
        frt.Context(0)
    assert e.value.code == frt.FRT_EDEVICE


class _Stub:
    """Stands in for libfrt.so: records calls, returns FRT_OK."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        if not name.startswith("frt_"):
            raise AttributeError(name)

        def f(*args):
            self.calls.append(name)
            if name == "frt_last_error":
                return b""
            return 0

        return f


def test_binding_marshals_every_call(monkeypatch):
    stub = _Stub()
    monkeypatch.setattr(frt, "_lib", stub)
    p = W.lognormal_c2(n=8, n_src=3, n_steps=2, box_cmpc_h=1.25)
    ctx = frt.Context(0)
    s = frt.solve_from_problem(ctx, p)
    s.set_opacity(p.kappa)
    s.step(p.dt_s)
    frt.batch_step([s], [p.dt_s])
    frt.batch_run([s], [p.dt_s], 2, graph=True)
    frt.autotune([s], [p.dt_s])
    ctx.set_tuning(item_rays=512)
    ctx.tuning()
    srv = frt.Server(ctx, 1 << 30, 4)
    rid = srv.submit(p, 2)
    srv.poll(rid)
    srv.wait(rid, 1.0)
    srv.take(rid)
    srv.times(rid)
    srv.stats()
    srv.close()
    s.sync()
    s.fields()
    s.ledger()
    s.load(b"x" * 16)
    for name in ("frt_ctx_create", "frt_solve_create", "frt_load_grid", "frt_set_opacity", "frt_load_sources",
                 "frt_set_rotations",
                 "frt_step", "frt_batch_step", "frt_sync", "frt_read_fields", "frt_read_ledger", "frt_load_state",
                 "frt_batch_run", "frt_autotune", "frt_ctx_set_tuning", "frt_ctx_get_tuning",
                 "frt_server_create", "frt_server_submit", "frt_server_poll", "frt_server_wait", "frt_server_take",
                 "frt_server_times", "frt_server_get_stats", "frt_server_destroy"):
        assert name in stub.calls, name


def _request(n=8, n_src=3, steps=2):
    p = W.lognormal_c2(n=n, n_src=n_src, n_steps=steps, box_cmpc_h=1.25 * n / 8)
    return p, frt.request_from_problem(p, steps)


def test_request_bytes_is_host_arithmetic_and_grows_with_the_problem():
    # no device needed: the estimate the server admits by
    p, (r, keep) = _request(8, 3)
    b = C.c_size_t()
    assert frt.lib().frt_request_bytes(C.byref(r), C.byref(b)) == frt.FRT_OK
    small = b.value
    ncell = 8 ** 3
    # resident fields alone are 36 bytes per cell (FP32 march, no T)
    assert small > 36 * ncell
    _, (r2, keep2) = _request(16, 3)
    assert frt.lib().frt_request_bytes(C.byref(r2), C.byref(b)) == frt.FRT_OK
    assert b.value > small
    _, (r3, keep3) = _request(8, 30)
    assert frt.lib().frt_request_bytes(C.byref(r3), C.byref(b)) == frt.FRT_OK
    assert b.value > small


def test_request_validation_errors():
    p, (r, keep) = _request()
    b = C.c_size_t()
    r.size = 3
    assert frt.lib().frt_request_bytes(C.byref(r), C.byref(b)) == frt.FRT_EINVAL
    r.size = C.sizeof(frt.Request)
    r.n_steps = -1
    assert frt.lib().frt_request_bytes(C.byref(r), C.byref(b)) == frt.FRT_EINVAL
    r.n_steps = 2
    r.nx = 0
    assert frt.lib().frt_request_bytes(C.byref(r), C.byref(b)) == frt.FRT_EINVAL
