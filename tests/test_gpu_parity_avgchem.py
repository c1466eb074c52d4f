"""GPU (HIP, gfx950) versus the FP64 oracle with the time-averaged chemistry
of §4.1 (chem_iterations = K: K marches per step, each from the step's
packets, n_HI from <x> of the march before).  Same tolerances as the
backward-Euler parity: neutral fraction within 1e-3 absolute (FP32 march),
ledger terms within 1e-4 of the emitted photons, ledger closure 1e-9; the
FP64 march within 1e-9."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight")


@pytest.fixture(scope="module")
def ctx():
    return frt.Context(0)


def _oracle(prob, steps):
    o = O.Oracle(**prob.oracle_kwargs())
    o.set_sources(prob.src_pos_cm, prob.ndot_bins)
    for s in range(steps):
        o.step(prob.dt_s, prob.uniforms(s))
    return o


def _gpu(ctx, prob, steps, **kw):
    g = frt.solve_from_problem(ctx, prob, **kw)
    for _ in range(steps):
        g.step(prob.dt_s)
    return g


def _compare(o, g, x_tol, led_tol, label):
    xo, _ = o.fields()
    xg, _ = g.fields()
    dx = np.abs(xo - xg)
    Lo, Lg = o.ledger(), g.ledger()
    E = Lo["emitted"]
    worst = {k: abs(Lo[k] - Lg[k]) / E for k in TERMS}
    print(f"[{label}] max|dx_HI| = {dx.max():.3e}  ledger rel = " +
          ", ".join(f"{k}:{v:.1e}" for k, v in worst.items()) +
          f"  crossings oracle={Lo['crossings']} gpu={Lg['crossings']}", flush=True)
    assert dx.max() <= x_tol, f"{label}: neutral fraction differs by {dx.max():.3e}"
    for k, v in worst.items():
        assert v <= led_tol, f"{label}: ledger term {k} differs by {v:.3e} of emitted"
    closure = abs(Lg["emitted"] - sum(Lg[k] for k in TERMS[1:]) - Lg["lost"]) / Lg["emitted"]
    assert closure <= 1e-9, f"{label}: GPU ledger does not close ({closure:.2e})"
    assert Lg["err_flags"] == 0 and Lg["lost"] == 0


@pytest.mark.parametrize("precision,K,x_tol,led_tol", [("f32", 3, 1e-3, 1e-4), ("f64", 3, 1e-9, 1e-9),
                                                       ("f32", 1, 1e-3, 1e-4)])
def test_lognormal_subgrid_finite_c(ctx, precision, K, x_tol, led_tol):
    # carried packets, 4 bins, kappa_sub, flux floor, ragged 27^3
    p = W.lognormal_c2(n=27, n_src=7, n_steps=5, box_cmpc_h=20.0 * 27 / 128)
    p.chem_iterations = K
    _compare(_oracle(p, 5), _gpu(ctx, p, 5, precision=precision), x_tol, led_tol, f"27^3 K={K} {precision}")


def _thick_box(K):
    rng = np.random.Generator(np.random.PCG64(11))
    n = 12
    nH = (2e-4 * np.exp(0.5 * rng.standard_normal((n, n, n)) - 0.125)).astype(np.float32)
    dx = W.cmpc_h_to_cm(20.0) / 1280
    return W.Problem(name="thick", shape=(n, n, n), dx_cm=dx, n_H=nH, x_HI0=np.ones((n, n, n)), kappa=None,
                     src_pos_cm=np.array([[3.5, 4.5, 6.5], [8.5, 7.5, 2.5]]) * dx,
                     ndot_bins=np.array([[3e51, 1e51], [1e51, 5e50]]), sigma_bins=np.array([6.3e-18, 2e-18]),
                     dt_s=3.15e13, n_steps=1, c_ray=np.inf, alpha_B=0.0, seed=1, chem_iterations=K)


def test_converged_iteration_conserves_photons(ctx):
    # alpha = C = 0: atoms ionized equal photons absorbed by the last march
    # once the iteration has converged (the oracle reaches 1e-10 at K = 80)
    p = _thick_box(48)
    g = _gpu(ctx, p, 1)
    _compare(_oracle(p, 1), g, 1e-3, 1e-4, "thick box K=48")
    x, _ = g.fields()
    ionized = float(np.sum(p.n_H.astype(np.float64) * p.dx_cm ** 3 * (1.0 - x)))
    absorbed = g.ledger()["absorbed_HI"]
    assert abs(ionized - absorbed) <= 1e-4 * absorbed


def test_queue_growth_reruns_every_march(ctx):
    # the first march overflows the automatic pass buffers: the step restarts
    # with larger ones, and the later marches start from the same packets
    p = W.grf_c3(n=32, n_src=60, throughput=True, n_steps=2, box_cmpc_h=100.0 * 32 / 256)
    p.x_HI0 = np.full(p.shape, 1e-6)
    p.flux_floor = 0.0
    p.n_ray_min = 4.0
    p.chem_iterations = 2
    g = _gpu(ctx, p, 2)
    assert g.ledger()["max_items"] > 4 * 60 * 12 + 65536
    _compare(_oracle(p, 2), g, 1e-3, 1e-4, "queue growth K=2")


def test_batched_and_graph_replay_equal_alone(ctx):
    boxes = W.batch_c4(n_boxes=4, n_steps=3, sizes=(16, 24), max_src=10, seed=43)
    for i, b in enumerate(boxes):
        b.chem_iterations = (0, 2, 2, 3)[i]      # three launch groups
    alone = [_gpu(ctx, b, 3) for b in boxes]
    stepped = [frt.solve_from_problem(ctx, b) for b in boxes]
    for _ in range(3):
        frt.batch_step(stepped, [b.dt_s for b in boxes])
    replayed = [frt.solve_from_problem(ctx, b) for b in boxes]
    frt.batch_run(replayed, [b.dt_s for b in boxes], 3, graph=True)
    for b, a, s, r in zip(boxes, alone, stepped, replayed):
        for other in (s, r):
            assert np.abs(a.fields()[0] - other.fields()[0]).max() <= 1e-5, b.name
            La, Lo = a.ledger(), other.ledger()
            for k in TERMS:
                assert abs(La[k] - Lo[k]) <= 1e-6 * La["emitted"], (b.name, k)
    _compare(_oracle(boxes[3], 3), replayed[3], 1e-3, 1e-4, "graph replay K=3")


def test_iteration_count_is_checked(ctx):
    p = W.stromgren_c1(n=8, n_steps=1)
    for bad in (-1, 65):
        p.chem_iterations = bad
        with pytest.raises(frt.FrtError) as e:
            frt.solve_from_problem(ctx, p)
        assert e.value.code == frt.FRT_EINVAL


def test_served_mix_of_chemistries_equals_alone(ctx):
    # the server steps its admitted requests together; requests with
    # different chemistry settings go to different launch groups
    probs = [r.problem for r in W.served_c5(n_requests=3, seed=73, n_steps=3, sizes=(16, 24), max_src=24)]
    for p, K in zip(probs, (0, 2, 3)):
        p.chem_iterations = K
    alone = []
    for p in probs:
        g = _gpu(ctx, p, 3)
        alone.append((g.fields()[0], g.ledger()))
    srv = frt.Server(frt.Context(0), budget_bytes=64 << 30, max_slots=8)
    ids = [srv.submit(p, 3) for p in probs]
    for rid in ids:
        assert srv.wait(rid, 120.0) == frt.REQ_DONE
    mixed = [srv.take(rid) for rid in ids]
    srv.close()
    for p, (xa, La), (xb, Lb) in zip(probs, alone, mixed):
        assert np.abs(xa - xb).max() <= 1e-5, p.name
        for k in TERMS:
            assert abs(La[k] - Lb[k]) <= 1e-6 * La["emitted"], (p.name, k)


def test_no_sources_is_pure_recombination_at_the_largest_k(ctx):
    # Gamma = 0 everywhere: every march deposits nothing and x relaxes by
    # recombination alone, the same on both sides; K at its maximum
    p = W.stromgren_c1(n=8, n_steps=3)
    p.src_pos_cm = p.src_pos_cm[:0]
    p.ndot_bins = p.ndot_bins[:0]
    p.x_HI0 = np.full(p.shape, 0.2)
    p.chem_iterations = 64
    g = _gpu(ctx, p, 3, precision="f64")
    o = O.Oracle(**p.oracle_kwargs())
    for s in range(3):
        o.step(p.dt_s, np.zeros(0))
    xg, xo = g.fields()[0], o.fields()[0]
    assert np.abs(xg - xo).max() <= 1e-12
    assert np.all(xg > 0.2)                       # recombination raised x_HI


@pytest.mark.parametrize("precision,x_tol,led_tol", [("f64", 1e-9, 1e-9), ("f32", 1e-3, 1e-4)])
def test_c1_as_configured_with_the_time_averaged_update(ctx, precision, x_tol, led_tol):
    # C1 as configured (corner vertex source, 2 Myr x 50 steps) with the
    # chemistry that meets its Stromgren gate on the oracle (K = 20): the HIP
    # path against the oracle over the whole run
    p = W.stromgren_c1()
    p.chem_iterations = 20
    _compare(_oracle(p, p.n_steps), _gpu(ctx, p, p.n_steps, precision=precision), x_tol, led_tol,
             f"C1 K=20 {precision}")
