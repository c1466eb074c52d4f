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


@pytest.mark.parametrize("seed,step,src", [(0, 0, 0), (7, 3, 11), (2 ** 40 + 5, 99, 1999)])
def test_library_generator_matches_inputs_module(seed, step, src):
    assert np.array_equal(frt.rotation_uniforms(seed, step, src), W.rotation_uniforms(seed, step, src + 1)[src])


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
    s.step(p.dt_s)
    frt.batch_step([s], [p.dt_s])
    frt.batch_run([s], [p.dt_s], 2, graph=True)
    frt.autotune([s], [p.dt_s])
    ctx.set_tuning(item_rays=512)
    ctx.tuning()
    s.sync()
    s.fields()
    s.ledger()
    s.load(b"x" * 16)
    for name in ("frt_ctx_create", "frt_solve_create", "frt_load_grid", "frt_load_sources", "frt_set_rotations",
                 "frt_step", "frt_batch_step", "frt_sync", "frt_read_fields", "frt_read_ledger", "frt_load_state",
                 "frt_batch_run", "frt_autotune", "frt_ctx_set_tuning", "frt_ctx_get_tuning"):
        assert name in stub.calls, name
