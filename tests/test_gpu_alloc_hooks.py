"""Device memory routed through a caller's allocator (frt_ctx_create hooks):
PyTorch's caching allocator gives every device buffer of a context and its
solves, the results equal those of a hipMalloc context, and every block
goes back when the solves and the context are destroyed, also when the
server's worker and loader threads make the calls.  Refused allocations
(a solve's creation, a queue growth inside a step, a served request's load)
fail that call alone: the other solves and requests give the results they
give alone, and nothing stays allocated."""
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


class _FailingAllocator(frt.TorchAllocator):
    """Torch-backed hooks that refuse chosen allocation calls (counted from
    1), to inject an out-of-memory failure at a known point."""

    def __init__(self, fail_at=()):
        super().__init__(0)
        import threading

        self.fail_at = set(fail_at)
        self.calls = 0
        self.refused = 0
        self._mu = threading.Lock()
        inner = self.alloc_fn

        def alloc(nbytes, user):
            with self._mu:
                self.calls += 1
                refuse = self.calls in self.fail_at
                self.refused += refuse
            return None if refuse else inner(nbytes, user)

        self.alloc_fn = frt.ALLOC_FN(alloc)


def _solo(p, steps):
    ctx = frt.Context(0)
    s = frt.solve_from_problem(ctx, p)
    for _ in range(steps):
        s.step(p.dt_s)
    out = s.fields()[0], s.ledger()
    s.close()
    ctx.close()
    return out


def _same_as_solo(s, p, steps, label):
    xr, Lr = _solo(p, steps)
    x, L = s.fields()[0], s.ledger()
    assert np.abs(x - xr).max() <= 1e-5, label
    assert L["steps"] == Lr["steps"] == steps and L["err_flags"] == 0, label
    for k in ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight"):
        assert abs(L[k] - Lr[k]) <= 1e-6 * Lr["emitted"], (label, k)


def test_allocation_failure_fails_only_its_own_solve():
    probs = [W.lognormal_c2(n=24, n_src=4, n_steps=3, box_cmpc_h=20.0 * 24 / 128, seed=s) for s in (61, 62, 63)]
    # allocation calls each creation makes, on a context of its own
    count = _FailingAllocator()
    cctx = frt.Context(0, allocator=count)
    made = []
    for p in probs:
        before = count.calls
        made.append(frt.solve_from_problem(cctx, p))
        print(f"creating {p.name} makes {count.calls - before} allocation calls", flush=True)
    for m in made:
        m.close()
    cctx.close()
    alloc = _FailingAllocator()
    ctx = frt.Context(0, allocator=alloc)
    a = frt.solve_from_problem(ctx, probs[0])
    alloc.fail_at = {alloc.calls + 3}             # inside the second solve's creation
    with pytest.raises(frt.FrtError) as e:
        frt.solve_from_problem(ctx, probs[1])
    assert e.value.code == frt.FRT_ENOMEM and alloc.refused == 1
    c = frt.solve_from_problem(ctx, probs[2])
    for _ in range(3):
        frt.batch_step([a, c], [probs[0].dt_s, probs[2].dt_s])
    _same_as_solo(a, probs[0], 3, "first solve")
    _same_as_solo(c, probs[2], 3, "third solve")
    a.close()
    c.close()
    ctx.close()
    assert alloc.bytes_out() == 0                  # nothing of the failed creation stays out


def test_allocation_failure_inside_a_step_leaves_the_solve_at_its_start():
    # small first queues: the step grows them, and the growth is refused once
    p = W.grf_c3(n=32, n_src=40, throughput=True, n_steps=2, box_cmpc_h=100.0 * 32 / 256)
    p.x_HI0 = np.full(p.shape, 1e-6)
    p.flux_floor = 0.0
    p.n_ray_min = 4.0
    alloc = _FailingAllocator()
    ctx = frt.Context(0, allocator=alloc)
    s = frt.solve_from_problem(ctx, p, queue_hint=4096)
    x0 = s.fields()[0]
    alloc.fail_at = set(range(alloc.calls + 1, alloc.calls + 200))   # every growth of this step
    with pytest.raises(frt.FrtError) as e:
        s.step(p.dt_s)
    assert e.value.code == frt.FRT_ENOMEM and alloc.refused >= 1
    L = s.ledger()
    assert L["steps"] == 0 and L["emitted"] == 0 and L["err_flags"] == 0
    assert np.array_equal(s.fields()[0], x0)
    alloc.fail_at = set()
    for _ in range(2):
        s.step(p.dt_s)
    _same_as_solo(s, p, 2, "after the refused growth")
    s.close()
    ctx.close()
    assert alloc.bytes_out() == 0


def test_server_allocation_failure_fails_one_request():
    reqs = W.served_c5(n_requests=4, n_steps=3, sizes=(24, 32), max_src=20, seed=64)
    alloc = _FailingAllocator()
    ctx = frt.Context(0, allocator=alloc)
    srv = frt.Server(ctx, 8 << 30, 1)              # one slot: the requests load one after another
    first = srv.submit(reqs[0].problem, 3)
    assert srv.wait(first, 120.0) == frt.REQ_DONE
    alloc.fail_at = {alloc.calls + 2}              # the next request's load
    ids = [srv.submit(r.problem, 3) for r in reqs[1:]]
    states = [srv.wait(rid, 120.0) for rid in ids]
    print(f"states {states}, refused {alloc.refused}", flush=True)
    assert states.count(frt.REQ_FAILED) == 1 and states[0] == frt.REQ_FAILED
    with pytest.raises(frt.FrtError) as e:
        srv.take(ids[0])
    assert e.value.code == frt.FRT_ENOMEM
    for r, rid in zip(reqs[1:], ids):
        if rid == ids[0]:
            continue
        x, L = srv.take(rid)
        xr, Lr = _solo(r.problem, 3)
        assert np.abs(x - xr).max() <= 1e-5 and L["steps"] == 3
    srv.take(first)
    srv.close()
    ctx.close()
    assert alloc.bytes_out() == 0
