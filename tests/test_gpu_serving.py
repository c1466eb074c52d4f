"""The continuous-batching server on the GPU: each request's result is the
same alone and in the mix (x_HI within 1e-5, ledger terms within 1e-6 of
emitted: only the order of the atomic deposits differs), one of them matches
the FP64 oracle at the parity tolerances, admission respects the memory
budget and the slots, requests submitted while others run join them, a
request larger than the whole budget fails cleanly, and requests with the
temperature on hand back the T they reach alone."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight")


def _requests(k=4, steps=4, seed=71, sizes=(16, 24, 32)):
    # the served recipe (lognormal density, sub-grid opacity, finite c) at sizes
    # the oracle finishes quickly
    reqs = W.served_c5(n_requests=k, seed=seed, n_steps=steps, sizes=sizes, max_src=24)
    return [r.problem for r in reqs]


def _alone(ctx, prob, steps):
    s = frt.solve_from_problem(ctx, prob)
    for _ in range(steps):
        s.step(prob.dt_s)
    return s.fields()[0], s.ledger()


def _same(xa, La, xb, Lb, label):
    assert np.abs(xa - xb).max() <= 1e-5, f"{label}: x_HI differs by {np.abs(xa - xb).max():.2e}"
    for k in TERMS:
        assert abs(La[k] - Lb[k]) <= 1e-6 * max(La["emitted"], 1e-300), (label, k)
    assert La["steps"] == Lb["steps"], label


def test_each_result_is_the_same_alone_and_in_the_mix():
    steps = 4
    probs = _requests(4, steps)
    ctx = frt.Context(0)
    alone = [_alone(ctx, p, steps) for p in probs]
    srv = frt.Server(frt.Context(0), budget_bytes=64 << 30, max_slots=8)
    ids = [srv.submit(p, steps) for p in probs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
    mixed = [srv.take(rid) for rid in ids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(probs) and st["failed"] == 0
    assert st["max_in_flight"] >= 2, st          # they did share ticks
    for p, (xa, La), (xb, Lb) in zip(probs, alone, mixed):
        _same(xa, La, xb, Lb, p.name)
    # one request against the oracle
    p = probs[0]
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    for k in range(steps):
        o.step(p.dt_s, p.uniforms(k))
    xo = o.fields()[0]
    xb, Lb = mixed[0]
    assert np.abs(xo - xb).max() <= 1e-3
    Lo = o.ledger()
    for k in TERMS:
        assert abs(Lo[k] - Lb[k]) <= 1e-4 * Lo["emitted"], k


def test_admission_respects_budget_and_slots():
    steps = 3
    probs = _requests(5, steps, seed=72, sizes=(24,))
    sizes = sorted(frt.request_bytes(p, steps) for p in probs)
    # room for the largest request but not for any two together
    budget = sizes[-1]
    assert budget < sizes[0] + sizes[1]
    srv = frt.Server(frt.Context(0), budget_bytes=budget, max_slots=8)
    ids = [srv.submit(p, steps) for p in probs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["max_in_flight"] == 1, st
    spans = [srv.times(rid) for rid in ids]
    # arrival order, one at a time: each starts after the previous finished
    for (a0, a1, a2), (b0, b1, b2) in zip(spans, spans[1:]):
        assert b1 >= a2
    for rid in ids:
        srv.take(rid)
    srv.close()
    # two slots, ample memory: never more than two in flight
    srv = frt.Server(frt.Context(0), budget_bytes=64 << 30, max_slots=2)
    ids = [srv.submit(p, steps) for p in probs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
    assert srv.stats()["max_in_flight"] == 2
    srv.close()


def test_late_arrivals_join_running_requests():
    probs = _requests(2, 40, seed=73)
    srv = frt.Server(frt.Context(0), budget_bytes=64 << 30, max_slots=4)
    first = srv.submit(probs[0], 40)
    while srv.poll(first) == frt.REQ_QUEUED:
        time.sleep(0.001)
    second = srv.submit(probs[1], 4)
    assert srv.wait(second, 120.0) == frt.REQ_DONE
    assert srv.wait(first, 120.0) == frt.REQ_DONE
    t1, t2 = srv.times(first), srv.times(second)
    # the short request was admitted while the long one ran and finished first
    assert t2[1] < t1[2] and t2[2] < t1[2], (t1, t2)
    ctx = frt.Context(0)
    for rid, p, n in ((first, probs[0], 40), (second, probs[1], 4)):
        xb, Lb = srv.take(rid)
        xa, La = _alone(ctx, p, n)
        _same(xa, La, xb, Lb, p.name)
    srv.close()


def test_request_larger_than_the_budget_fails_cleanly():
    probs = _requests(2, 2, seed=74)
    need = frt.request_bytes(probs[0], 2)
    srv = frt.Server(frt.Context(0), budget_bytes=need // 2, max_slots=2)
    rid = srv.submit(probs[0], 2)
    assert srv.wait(rid, 60.0) == frt.REQ_FAILED
    with pytest.raises(frt.FrtError) as e:
        srv.take(rid)
    assert e.value.code == frt.FRT_ENOMEM
    srv.close()


def test_temperature_requests_return_their_temperature():
    steps = 3
    probs = _requests(3, steps, seed=77)
    for p in probs[:2]:
        p.temperature = True
        p.heat_ev = W.blackbody_heat(p.n_bins, T_bb=5e4)
        p.T = np.full(p.shape, 2e3, np.float32)
    ctx = frt.Context(0)
    alone = []
    for p in probs[:2]:
        s = frt.solve_from_problem(ctx, p)
        for _ in range(steps):
            s.step(p.dt_s)
        alone.append(s.temperature())
    srv = frt.Server(frt.Context(0), budget_bytes=64 << 30, max_slots=8)
    ids = [srv.submit(p, steps) for p in probs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
    for Ta, rid in zip(alone, ids[:2]):
        Tb = srv.temperature(rid)
        print(f"served T vs alone: max rel {np.max(np.abs(Tb / Ta - 1)):.2e}, T {Ta.min():.0f}-{Ta.max():.0f} K",
              flush=True)
        assert np.max(np.abs(Tb / Ta - 1)) <= 1e-3 and Ta.max() > 2.5e3
    with pytest.raises(frt.FrtError) as e:
        srv.temperature(ids[2])
    assert e.value.code == frt.FRT_ESTATE
    for rid in ids:
        srv.take(rid)
    srv.close()
