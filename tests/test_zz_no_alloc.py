"""The allocation-free step (frt_step_static), through the C ABI: its pass
queues live in the library's static device scratch.  It gives frt_step's
results (neutral fraction within 1e-3, every ledger term within 1e-4 of the
emitted photons, the parity bar of the rest of the GPU tests; in practice
rounding-level), on two calls in a row, the second on a smaller problem, and
makes no device allocation: a context whose allocator hooks count every
block sees none during the static steps."""
import ctypes as C

import numpy as np
import pytest

from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight")


class _Counting:
    """Allocator hooks over PyTorch's caching allocator that count calls."""

    def __init__(self):
        import torch

        self.allocs = 0
        self.frees = 0

        def alloc(n, user):
            self.allocs += 1
            return torch.cuda.caching_allocator_alloc(int(n), 0)

        def free(p, user):
            self.frees += 1
            torch.cuda.caching_allocator_delete(p)

        self.alloc_fn = frt.ALLOC_FN(alloc)
        self.free_fn = frt.FREE_FN(free)


def _compare(a, b, label):
    xa, _ = a.fields()
    xb, _ = b.fields()
    La, Lb = a.ledger(), b.ledger()
    dx = float(np.abs(xa - xb).max())
    worst = max(abs(La[k] - Lb[k]) / Lb["emitted"] for k in TERMS)
    print(f"[{label}] max|dx_HI| = {dx:.2e}, ledger terms within {worst:.1e} of emitted, "
          f"crossings {La['crossings']} / {Lb['crossings']}", flush=True)
    assert dx <= 1e-3 and worst <= 1e-4, label
    assert La["steps"] == Lb["steps"] and La["err_flags"] == 0


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_static_step_equals_step_on_two_calls_in_a_row(precision):
    counter = _Counting()
    ctx = frt.Context(0, allocator=counter)
    # nearly ionized gas, so that packets cross the box, split to level 5 and
    # take many passes: finite c with sub-grid opacity (packets carried from
    # step to step), then a smaller box without it at c = inf (the other march)
    big = W.lognormal_c2(n=40, n_src=2, n_steps=4, box_cmpc_h=20.0 * 40 / 128)
    big.x_HI0 = np.full(big.shape, 1e-3)
    small = W.lognormal_c2(n=24, n_src=3, n_steps=3, box_cmpc_h=20.0 * 24 / 128, seed=9)
    small.kappa = None
    small.c_ray = np.inf
    small.x_HI0 = np.full(small.shape, 1e-2)
    for prob, label in ((big, "40^3 2 sources c"), (small, "24^3 3 sources c=inf")):
        ref = frt.solve_from_problem(ctx, prob, precision=precision)
        sta = frt.solve_from_problem(ctx, prob, precision=precision)
        for _ in range(prob.n_steps):
            ref.step(prob.dt_s)
        n0 = (counter.allocs, counter.frees)
        for _ in range(prob.n_steps):
            sta.step_static(prob.dt_s)
        assert (counter.allocs, counter.frees) == n0, "the static step allocated or freed device memory"
        _compare(sta, ref, f"{label} {precision}")
        assert ref.ledger()["splits"] > 0 and ref.ledger()["crossings"] > 100000
        ref.close()
        sta.close()
    ctx.close()


def test_static_step_limits_are_errors_and_leave_the_solve_unchanged():
    ctx = frt.Context(0)
    # more packets per pass than the scratch holds: 60 sources splitting to
    # level 6 in a nearly transparent 32^3 box
    p = W.grf_c3(n=32, n_src=60, throughput=True, n_steps=1, box_cmpc_h=100.0 * 32 / 256)
    p.x_HI0 = np.full(p.shape, 1e-6)
    p.flux_floor = 0.0
    p.n_ray_min = 4.0
    s = frt.solve_from_problem(ctx, p)
    x0, _ = s.fields()
    L0 = s.ledger()
    with pytest.raises(frt.FrtError) as e:
        s.step_static(p.dt_s)
    assert e.value.code == frt.FRT_EOVERFLOW
    x1, _ = s.fields()
    L1 = s.ledger()
    assert np.array_equal(x0, x1) and L1["steps"] == L0["steps"] and L1["emitted"] == L0["emitted"]
    assert L1["err_flags"] == 0
    s.step(p.dt_s)                          # the allocating step still runs it
    # a grid of more bricks than the scratch's key table (FP64: 8^3 bricks)
    q = frt.Solve(ctx, sigma_bins=[6.3e-18], precision="f64")
    q.load_grid(np.full((128, 128, 136), 1e-4, np.float32), 1e21 * 136)
    q.load_sources(np.array([[1e22, 1e22, 1e22]]), np.array([[1e50]]))
    with pytest.raises(frt.FrtError) as e:
        q.step_static(1e13)
    assert e.value.code == frt.FRT_EINVAL
