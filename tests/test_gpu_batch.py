"""Batched runs on the GPU: graph-replayed steps, queue growth inside a
graph run, fixed capacities, and the autotuner.  Every result is checked
against the same solves stepped one launch sequence at a time (atomic order
is the only difference: x_HI within 1e-5, ledger terms within 1e-6 of
emitted) and, for some boxes, against the FP64 oracle at the parity
tolerances (1e-3 in x_HI, 1e-4 of emitted)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight")


def _oracle(prob, steps):
    o = O.Oracle(**prob.oracle_kwargs())
    o.set_sources(prob.src_pos_cm, prob.ndot_bins)
    for s in range(steps):
        o.step(prob.dt_s, prob.uniforms(s))
    return o


def _same(a, b, label):
    xa, xb = a.fields()[0], b.fields()[0]
    assert np.abs(xa - xb).max() <= 1e-5, f"{label}: x_HI differs by {np.abs(xa - xb).max():.2e}"
    La, Lb = a.ledger(), b.ledger()
    for k in TERMS:
        assert abs(La[k] - Lb[k]) <= 1e-6 * max(La["emitted"], 1e-300), (label, k)
    assert La["steps"] == Lb["steps"], label
    assert Lb["err_flags"] == 0 and Lb["lost"] == 0, label


def _versus_oracle(prob, g, steps, label):
    o = _oracle(prob, steps)
    xo, xg = o.fields()[0], g.fields()[0]
    assert np.abs(xo - xg).max() <= 1e-3, f"{label}: x_HI differs from the oracle by {np.abs(xo - xg).max():.2e}"
    Lo, Lg = o.ledger(), g.ledger()
    for k in TERMS:
        assert abs(Lo[k] - Lg[k]) <= 1e-4 * Lo["emitted"], (label, k)


def _dense_ray_problem():
    # 32^3, nearly transparent, N_min = 4: passes hold far more packets than
    # the first automatic queue size
    p = W.grf_c3(n=32, n_src=60, throughput=True, n_steps=2, box_cmpc_h=100.0 * 32 / 256)
    p.x_HI0 = np.full(p.shape, 1e-6)
    p.flux_floor = 0.0
    p.n_ray_min = 4.0
    return p


def test_graph_run_equals_stepwise_and_oracle():
    ctx = frt.Context(0)
    boxes = W.batch_c4(n_boxes=6, n_steps=5, sizes=(16, 24, 32, 40), max_src=10, seed=43)
    dts = [b.dt_s for b in boxes]
    stepwise = [frt.solve_from_problem(ctx, b) for b in boxes]
    graphed = [frt.solve_from_problem(ctx, b) for b in boxes]
    for _ in range(5):
        frt.batch_step(stepwise, dts)
    frt.batch_run(graphed, dts, 5, graph=True)
    for b, a, g in zip(boxes, stepwise, graphed):
        _same(a, g, b.name)
    for b, g in list(zip(boxes, graphed))[:2]:
        _versus_oracle(b, g, 5, f"graph {b.name}")
    # the same run without a graph, continued from where the graph left off
    frt.batch_run(graphed, dts, 1, graph=False)
    frt.batch_step(stepwise, dts)
    for b, a, g in zip(boxes, stepwise, graphed):
        _same(a, g, b.name + " +1")


@pytest.mark.parametrize("check_every", [1, 2])
def test_graph_run_grows_its_queues(check_every):
    p = _dense_ray_problem()
    a = frt.solve_from_problem(frt.Context(0), p)
    for _ in range(2):
        a.step(p.dt_s)
    small = frt.Context(0)            # own workspace, first sized from the hint
    g = frt.solve_from_problem(small, p, queue_hint=4096)
    frt.batch_run([g], [p.dt_s], 2, graph=True, check_every=check_every)
    _same(a, g, f"grown in a graph run, checked every {check_every}")
    _versus_oracle(p, g, 2, "grown in a graph run")


def _carrying_box(seed=51, kappa=False):
    # packets carried at a finite speed pile up over the steps, so the passes
    # grow from step to step
    p = W.lognormal_c2(n=24, n_src=6, n_steps=7, box_cmpc_h=20.0 * 24 / 128, seed=seed)
    p.x_HI0 = np.full(p.shape, 1e-4)
    if not kappa:
        p.kappa = None
    p.c_ray = 2.0 * p.dx_cm / p.dt_s
    return p


@pytest.mark.parametrize("check_every", [3, 7])
def test_windowed_graph_run_equals_a_check_per_step(check_every):
    # several replays between host reads change nothing: FP64, so the only
    # difference allowed is the order of the ledger's atomic additions
    ctx = frt.Context(0)
    boxes = [_carrying_box(51), _carrying_box(52), _carrying_box(53, kappa=True)]
    dts = [b.dt_s for b in boxes]
    each = [frt.solve_from_problem(ctx, b, precision="f64") for b in boxes]
    win = [frt.solve_from_problem(ctx, b, precision="f64") for b in boxes]
    frt.batch_run(each, dts, 7, graph=True, check_every=1)
    frt.batch_run(win, dts, 7, graph=True, check_every=check_every)
    for b, a, w in zip(boxes, each, win):
        assert np.abs(a.fields()[0] - w.fields()[0]).max() <= 1e-12, b.name
        La, Lw = a.ledger(), w.ledger()
        assert La["steps"] == Lw["steps"] == 7
        for k in TERMS:
            assert abs(La[k] - Lw[k]) <= 1e-12 * La["emitted"], (b.name, k)
        assert Lw["err_flags"] == 0 and Lw["crossings"] == La["crossings"]
    _versus_oracle(boxes[0], win[0], 7, f"windowed graph run, checked every {check_every}")


def test_overflow_inside_a_window_stops_at_the_failed_step():
    # a fixed capacity that the first steps fit and a later one does not:
    # the windowed graph run applies the steps before the failed one and
    # leaves the solve exactly where stepping one by one stops
    p = _carrying_box()
    steps = p.n_steps
    found = None
    cap = 512
    while cap < (1 << 26):
        # the smallest capacity (in steps of 1.5x) that the first step fits
        probe = frt.solve_from_problem(frt.Context(0), p, precision="f64", queue_capacity=cap)
        fail_at = None
        for k in range(steps):
            try:
                probe.step(p.dt_s)
            except frt.FrtError as e:
                assert e.code == frt.FRT_EOVERFLOW
                fail_at = k
                break
        if fail_at is None:
            break
        if fail_at >= 1:
            found = (cap, fail_at, probe)
            break
        cap = int(cap * 1.5)
    assert found is not None, "no capacity that a later step overflows"
    cap, fail_at, probe = found
    print(f"capacity {cap}: stepping one by one stops at step {fail_at}", flush=True)
    g = frt.solve_from_problem(frt.Context(0), p, precision="f64", queue_capacity=cap)
    with pytest.raises(frt.FrtError) as e:
        frt.batch_run([g], [p.dt_s], steps, graph=True, check_every=steps)
    assert e.value.code == frt.FRT_EOVERFLOW
    Lg, Lp = g.ledger(), probe.ledger()
    assert Lg["steps"] == Lp["steps"] == fail_at and Lg["err_flags"] == 0
    assert np.abs(g.fields()[0] - probe.fields()[0]).max() <= 1e-12
    for k in TERMS:
        assert abs(Lg[k] - Lp[k]) <= 1e-12 * Lp["emitted"], k
    assert Lg["n_in_flight"] == Lp["n_in_flight"]


def test_graph_run_fixed_capacity_overflow_is_not_applied():
    p = _dense_ray_problem()
    g = frt.solve_from_problem(frt.Context(0), p, queue_capacity=2000)
    x0 = g.fields()[0]
    L0 = g.ledger()
    with pytest.raises(frt.FrtError) as e:
        frt.batch_run([g], [p.dt_s], 2, graph=True)
    assert e.value.code == frt.FRT_EOVERFLOW
    assert np.array_equal(g.fields()[0], x0)
    L1 = g.ledger()
    assert L1["steps"] == L0["steps"] and L1["emitted"] == L0["emitted"] and L1["err_flags"] == 0


def test_autotune_changes_no_result():
    ctx = frt.Context(0)
    boxes = W.batch_c4(n_boxes=3, n_steps=3, sizes=(16, 24, 32), max_src=8, seed=44)
    dts = [b.dt_s for b in boxes]
    ref = [frt.solve_from_problem(ctx, b) for b in boxes]
    tuned = [frt.solve_from_problem(ctx, b) for b in boxes]
    frt.batch_step(ref, dts)
    frt.batch_step(tuned, dts)
    before = [t.fields() for t in tuned]
    best = frt.autotune(tuned, dts)
    assert best == ctx.tuning()
    assert best["item_rays"] in (256, 512, 1024)
    for (x, gam), t in zip(before, tuned):
        x2, gam2 = t.fields()
        assert np.array_equal(x, x2) and np.array_equal(gam, gam2)
    for _ in range(2):
        frt.batch_step(ref, dts)
        frt.batch_step(tuned, dts)
    for b, a, t in zip(boxes, ref, tuned):
        _same(a, t, b.name)
    _versus_oracle(boxes[0], tuned[0], 3, "after autotune")


def test_tuning_is_validated_and_changes_no_result():
    ctx = frt.Context(0)
    with pytest.raises(frt.FrtError) as e:
        ctx.set_tuning(item_rays=100)
    assert e.value.code == frt.FRT_EINVAL
    with pytest.raises(frt.FrtError):
        ctx.set_tuning(scatter_blocks_per_cu=0)
    p = W.lognormal_c2(n=24, n_src=6, n_steps=3, box_cmpc_h=20.0 * 24 / 128)
    a = frt.solve_from_problem(ctx, p)
    for _ in range(3):
        a.step(p.dt_s)
    ctx.set_tuning(item_rays=64, scatter_blocks_per_cu=1)
    b = frt.solve_from_problem(ctx, p)
    for _ in range(3):
        b.step(p.dt_s)
    _same(a, b, "smallest launch shape")
