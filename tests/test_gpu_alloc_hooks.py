"""Device memory routed through a caller's allocator (frt_ctx_create hooks):
PyTorch's caching allocator gives every device buffer of a context and its
solves, the results equal those of a hipMalloc context, and every block
goes back when the solves and the context are destroyed, also when the
server's worker and loader threads make the calls."""
import numpy as np
import pytest

from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_torch_caching_allocator_backs_the_library():
    import torch

    torch.cuda.init()
    base = torch.cuda.memory_allocated(0)
    alloc = frt.TorchAllocator(0)
    ctx = frt.Context(0, allocator=alloc)
    p = W.lognormal_c2(n=32, n_src=6, n_steps=3, box_cmpc_h=20.0 * 32 / 128)
    s = frt.solve_from_problem(ctx, p)
    assert alloc.bytes_out() >= p.ncell * 36          # the resident fields at least
    # torch rounds every block up to a multiple of 512 bytes
    held = lambda: torch.cuda.memory_allocated(0) - base
    assert alloc.bytes_out() <= held() <= alloc.bytes_out() + 512 * len(alloc.live)
    for _ in range(p.n_steps):
        s.step(p.dt_s)
    assert alloc.bytes_out() <= held() <= alloc.bytes_out() + 512 * len(alloc.live)
    ref_ctx = frt.Context(0)
    ref = frt.solve_from_problem(ref_ctx, p)
    for _ in range(p.n_steps):
        ref.step(p.dt_s)
    x, g = s.fields()
    xr, gr = ref.fields()
    assert np.abs(x - xr).max() <= 1e-6
    La, Lb = s.ledger(), ref.ledger()
    for k in ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight"):
        assert La[k] == pytest.approx(Lb[k], rel=1e-9, abs=1e-12 * Lb["emitted"]), k
    s.close()
    ctx.close()
    ref.close()
    ref_ctx.close()
    assert alloc.bytes_out() == 0
    assert torch.cuda.memory_allocated(0) == base


def test_server_threads_allocate_through_the_hooks():
    alloc = frt.TorchAllocator(0)
    ctx = frt.Context(0, allocator=alloc)
    srv = frt.Server(ctx, 8 << 30, 4)
    reqs = W.served_c5(n_requests=3, n_steps=2, sizes=(24, 32), max_src=20)
    ids = [srv.submit(r.problem, 2) for r in reqs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
        srv.take(rid)
    assert alloc.bytes_out() > 0                      # the context's pass queues
    srv.close()
    ctx.close()
    assert alloc.bytes_out() == 0


def test_hooks_must_come_in_pairs():
    h = frt.C.c_void_p()
    rc = frt.lib().frt_ctx_create(0, frt.TorchAllocator(0).alloc_fn, frt.FREE_FN(), None, frt.C.byref(h))
    assert rc == frt.FRT_EINVAL
