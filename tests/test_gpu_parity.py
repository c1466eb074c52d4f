"""GPU (HIP, gfx950) versus the FP64 oracle on the same seeded inputs.

Tolerances (from the FP32 march with FP64 chemistry): neutral fraction within
1e-3 absolute in every cell, every photon-ledger term within 1e-4 of the
emitted photons.  The FP64 march is held to 1e-9.  Every call goes through
the C ABI (libfrt.so) via the ctypes binding."""
import math

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


def _gpu(ctx, prob, steps, precision="f32", use_table=True, **kw):
    g = frt.solve_from_problem(ctx, prob, precision=precision, use_table=use_table, **kw)
    for _ in range(steps):
        g.step(prob.dt_s)
    return g


def _compare(o, g, x_tol, led_tol, label=""):
    xo, go = o.fields()
    xg, gg = g.fields()
    dx = np.abs(xo - xg)
    Lo, Lg = o.ledger(), g.ledger()
    E = Lo["emitted"]
    worst = {k: abs(Lo[k] - Lg[k]) / E for k in TERMS} if E > 0 else {}
    print(f"[{label}] max|dx_HI| = {dx.max():.3e}  ledger rel = " +
          ", ".join(f"{k}:{v:.1e}" for k, v in worst.items()) +
          f"  crossings oracle={Lo['crossings']} gpu={Lg['crossings']}", flush=True)
    assert dx.max() <= x_tol, f"{label}: neutral fraction differs by {dx.max():.3e} at {np.unravel_index(dx.argmax(), dx.shape)}"
    for k, v in worst.items():
        assert v <= led_tol, f"{label}: ledger term {k} differs by {v:.3e} of emitted"
    closure = abs(Lg["emitted"] - sum(Lg[k] for k in TERMS[1:]) - Lg["lost"]) / max(Lg["emitted"], 1e-300)
    assert closure <= 1e-9, f"{label}: GPU ledger does not close ({closure:.2e})"
    assert Lg["err_flags"] == 0 and Lg["lost"] == 0
    return xo, xg, go, gg


@pytest.mark.parametrize("precision,x_tol,led_tol", [("f64", 1e-9, 1e-9), ("f32", 1e-3, 1e-4)])
def test_stromgren_corner_source(ctx, precision, x_tol, led_tol):
    p = W.stromgren_c1(n=32, n_steps=12)
    o = _oracle(p, 12)
    g = _gpu(ctx, p, 12, precision=precision)
    xo, xg, go, gg = _compare(o, g, x_tol, led_tol, f"C1 32^3 {precision}")
    # deposition itself, cell by cell, on the last step (the ABI hands the
    # rate out as float32, hence 1e-6 for the FP64 march)
    scale = go.max()
    err = float(np.abs(go - gg).max())
    assert err <= (1e-6 if precision == "f64" else 2e-3) * scale, f"gamma differs by {err:.3e} (scale {scale:.3e})"


def test_stromgren_full_50_steps_f64(ctx):
    p = W.stromgren_c1(n=32, n_steps=50)
    _compare(_oracle(p, 50), _gpu(ctx, p, 50, precision="f64"), 1e-9, 1e-9, "C1 50 steps f64")


@pytest.mark.parametrize("n,n_src,steps", [(24, 6, 8), (37, 11, 6)])
def test_lognormal_subgrid_finite_c(ctx, n, n_src, steps):
    # finite speed of light (packets carried between steps), 4 bins, kappa_sub,
    # flux floor; 37^3 is a ragged size
    p = W.lognormal_c2(n=n, n_src=n_src, n_steps=steps, box_cmpc_h=20.0 * n / 128)
    _compare(_oracle(p, steps), _gpu(ctx, p, steps), 1e-3, 1e-4, f"C2-like {n}^3")


def test_grf_throughput_form(ctx):
    # highly ionized start, packets finish inside the step, distance cap
    p = W.grf_c3(n=48, n_src=24, throughput=True, n_steps=2, box_cmpc_h=100.0 * 48 / 256)
    _compare(_oracle(p, 2), _gpu(ctx, p, 2), 1e-3, 1e-4, "C3b-like 48^3")


def test_grf_neutral_finite_c(ctx):
    p = W.grf_c3(n=40, n_src=16, throughput=False, n_steps=5, box_cmpc_h=100.0 * 40 / 256)
    _compare(_oracle(p, 5), _gpu(ctx, p, 5), 1e-3, 1e-4, "C3a-like 40^3")


def test_non_cubic_grid_levels_and_nmin(ctx):
    rng = np.random.Generator(np.random.PCG64(77))
    shape = (13, 29, 21)
    dx = W.cmpc_h_to_cm(0.15625)
    nH = W.lognormal_white(rng, shape, 2e-4, 0.8).astype(np.float32)
    pos = np.array([[3.5, 20.5, 6.5], [17.5, 2.5, 11.5], [0.5, 0.5, 0.5]]) * dx
    w, sig = W.blackbody_bins(2)
    ndot = np.array([3e51, 1e50, 4e52])[:, None] * w[None, :]
    p = W.Problem(name="odd", shape=shape, dx_cm=dx, n_H=nH, x_HI0=np.full(shape, 0.3), kappa=None,
                  src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig, dt_s=0.5 * W.MYR, n_steps=4,
                  c_ray=W.C_LIGHT, flux_floor=1e-3, base_level=1, max_level=5, n_ray_min=2.0, seed=9)
    _compare(_oracle(p, 4), _gpu(ctx, p, 4), 1e-3, 1e-4, "non-cubic L0=1 Nmin=2")


def test_no_sources_is_pure_recombination(ctx):
    p = W.stromgren_c1(n=8, n_steps=3)
    p.src_pos_cm = np.zeros((0, 3))
    p.ndot_bins = np.zeros((0, 1))
    p.x_HI0 = np.full(p.shape, 0.25)
    o = _oracle(p, 3)
    g = _gpu(ctx, p, 3)
    assert np.abs(o.fields()[0] - g.fields()[0]).max() <= 1e-12
    assert g.ledger()["emitted"] == 0


def test_single_cell_box_and_boundary_source(ctx):
    shape = (1, 1, 1)
    dx = 1e21
    p = W.Problem(name="one", shape=shape, dx_cm=dx, n_H=np.full(shape, 1e-3, np.float32), x_HI0=np.ones(shape),
                  kappa=None, src_pos_cm=np.array([[dx, 0.5 * dx, 0.25 * dx]]), ndot_bins=np.array([[1e49]]),
                  sigma_bins=np.array([W.SIGMA_HI_0]), dt_s=1e13, n_steps=2, c_ray=math.inf, seed=4)
    _compare(_oracle(p, 2), _gpu(ctx, p, 2, precision="f64"), 1e-9, 1e-9, "1-cell box")


def test_no_split_when_max_level_is_base(ctx):
    p = W.lognormal_c2(n=20, n_src=4, n_steps=3, box_cmpc_h=20.0 * 20 / 128)
    p.max_level = 0
    _compare(_oracle(p, 3), _gpu(ctx, p, 3), 1e-3, 1e-4, "max_level = 0")


def test_internal_generator_equals_table(ctx):
    p = W.lognormal_c2(n=20, n_src=5, n_steps=3, box_cmpc_h=20.0 * 20 / 128)
    a = _gpu(ctx, p, 3, use_table=True)
    b = _gpu(ctx, p, 3, use_table=False)
    xa, _ = a.fields()
    xb, _ = b.fields()
    assert np.abs(xa - xb).max() <= 1e-6
    assert a.ledger()["crossings"] == b.ledger()["crossings"]


def test_checkpoint_resume(ctx):
    p = W.lognormal_c2(n=20, n_src=5, n_steps=6, box_cmpc_h=20.0 * 20 / 128)
    a = _gpu(ctx, p, 6)
    b = _gpu(ctx, p, 3)
    blob = b.save()
    c = frt.solve_from_problem(ctx, p)
    c.load(blob)
    for _ in range(3):
        c.step(p.dt_s)
    assert np.abs(a.fields()[0] - c.fields()[0]).max() <= 1e-5
    La, Lc = a.ledger(), c.ledger()
    for k in TERMS:
        assert abs(La[k] - Lc[k]) <= 1e-6 * La["emitted"]
    assert La["crossings"] == Lc["crossings"]


def test_mark_and_rewind_repeat_a_step(ctx):
    p = W.lognormal_c2(n=24, n_src=6, n_steps=3, box_cmpc_h=20.0 * 24 / 128)
    a = _gpu(ctx, p, 1)
    b = frt.solve_from_problem(ctx, p)
    b.mark()
    for _ in range(3):
        b.rewind()
        b.step(p.dt_s)
    xa, ga = a.fields()
    xb, gb = b.fields()
    assert np.abs(xa - xb).max() <= 1e-6
    assert np.abs(ga - gb).max() <= 1e-5 * ga.max()
    La, Lb = a.ledger(), b.ledger()
    assert Lb["crossings"] == 3 * La["crossings"]
    assert Lb["step_crossings"] == La["step_crossings"]


def test_batched_equals_alone(ctx):
    boxes = W.batch_c4(n_boxes=5, n_steps=4, sizes=(16, 24, 32), max_src=12, seed=41)
    alone = [_gpu(ctx, b, 4) for b in boxes]
    batched = [frt.solve_from_problem(ctx, b) for b in boxes]
    for _ in range(4):
        frt.batch_step(batched, [b.dt_s for b in boxes])
    for b, a, s in zip(boxes, alone, batched):
        assert np.abs(a.fields()[0] - s.fields()[0]).max() <= 1e-5, b.name
        La, Ls = a.ledger(), s.ledger()
        for k in TERMS:
            assert abs(La[k] - Ls[k]) <= 1e-6 * max(La["emitted"], 1e-300), (b.name, k)
    # and the batch against the oracle for two of the boxes
    for b, s in list(zip(boxes, batched))[:2]:
        _compare(_oracle(b, 4), s, 1e-3, 1e-4, f"batched {b.name}")


def _dense_ray_problem():
    # 32^3 box, nearly transparent, N_min = 4 (split radius 0.49 * 2^l cells),
    # 60 sources: level-5 packets number up to 12 * 4^5 per source, far more
    # per pass than the automatic initial pass buffers (about 7e4 records)
    p = W.grf_c3(n=32, n_src=60, throughput=True, n_steps=2, box_cmpc_h=100.0 * 32 / 256)
    p.x_HI0 = np.full(p.shape, 1e-6)
    p.flux_floor = 0.0
    p.n_ray_min = 4.0
    return p


def test_queue_growth_reruns_the_step(ctx):
    p = _dense_ray_problem()
    g = _gpu(ctx, p, 2)
    assert g.ledger()["max_items"] > 4 * 60 * 12 + 65536
    _compare(_oracle(p, 2), g, 1e-3, 1e-4, "queue growth")


def test_fixed_capacity_overflow_is_reported_and_not_applied(ctx):
    # a step that overflows a fixed queue is reported by the step call and
    # leaves the solve exactly at the start of that step (fields, ledger,
    # step index, no error bits left behind), so that stepping can go on
    p = _dense_ray_problem()
    g = frt.solve_from_problem(ctx, p, queue_capacity=2000)
    x0, _ = g.fields()
    L0 = g.ledger()
    for attempt in range(2):
        with pytest.raises(frt.FrtError) as e:
            g.step(p.dt_s)
        assert e.value.code == frt.FRT_EOVERFLOW
        g.sync()                                   # nothing deferred
        x1, _ = g.fields()
        L1 = g.ledger()
        assert np.array_equal(x0, x1), attempt
        assert L1["steps"] == L0["steps"] and L1["emitted"] == L0["emitted"] and L1["err_flags"] == 0
    # a fixed capacity that holds the step gives the oracle's result
    big = frt.solve_from_problem(ctx, p, queue_capacity=16_000_000)
    for _ in range(2):
        big.step(p.dt_s)
    _compare(_oracle(p, 2), big, 1e-3, 1e-4, "fixed capacity")


def _lognormal_24(seed, ionized, c_cells=5.0, n_ray_min=None):
    p = W.lognormal_c2(n=24, n_src=5, n_steps=2, box_cmpc_h=20.0 * 24 / 128, seed=seed)
    if ionized:
        p.x_HI0 = np.full(p.shape, 1e-3)
    p.kappa = None
    p.c_ray = c_cells * p.dx_cm / p.dt_s
    if n_ray_min is not None:
        p.n_ray_min = n_ray_min
    return p


@pytest.mark.parametrize("K", [0, 3])
def test_a_batch_run_again_after_an_overflow_leaves_each_solve_as_alone(K):
    # a batch whose second solve overflows its carried-packet queue is run
    # again from the start of the step with that queue enlarged; the first
    # solve's chemistry of the failed run (x and opacity are updated in
    # place) must not be kept, so each solve ends as if stepped alone
    a = _lognormal_24(31, ionized=False)
    b = _lognormal_24(37, ionized=True, c_cells=12.0, n_ray_min=4.0)
    for p in (a, b):
        p.chem_iterations = K
    c1 = frt.Context(0)
    ga = frt.solve_from_problem(c1, a, precision="f64")
    gb = frt.solve_from_problem(c1, b, precision="f64")
    frt.batch_step([ga, gb], [a.dt_s, b.dt_s])
    # more packets carried than the carried queue first held (the cast
    # packets, 1024 more and the cells): the step was run again
    cast = b.n_src * 12 * 4 ** b.base_level
    first_cap = cast + 1024 + min(b.ncell, 8 * cast + 65536)
    assert gb.ledger()["n_in_flight"] > first_cap
    frt.batch_step([ga, gb], [a.dt_s, b.dt_s])
    c2 = frt.Context(0)
    for p, g in ((a, ga), (b, gb)):
        r = _gpu(c2, p, 2, precision="f64")
        dx = float(np.abs(r.fields()[0] - g.fields()[0]).max())
        Lr, Lg = r.ledger(), g.ledger()
        print(f"[{p.name} K={K}] batched vs alone max|dx_HI| = {dx:.1e}, crossings {Lg['crossings']} / {Lr['crossings']}",
              flush=True)
        assert dx <= 1e-12
        assert Lg["crossings"] == Lr["crossings"]
        for k in ("emitted", "absorbed_HI", "escaped", "dropped", "in_flight"):
            assert Lg[k] == pytest.approx(Lr[k], rel=1e-12, abs=1e-12 * Lr["emitted"]), k
        r.close()
    for g in (ga, gb):
        g.close()
    c1.close()
    c2.close()


def test_fixed_capacity_overflow_in_a_batch_applies_no_solve(ctx):
    # one solve's carried queue is too small: the batch step fails and no
    # solve of the batch changes, also those whose own queues held
    a = _lognormal_24(31, ionized=False)
    b = _lognormal_24(37, ionized=True, c_cells=12.0, n_ray_min=4.0)
    ga = frt.solve_from_problem(ctx, a, precision="f64", queue_capacity=8_000_000)
    gb = frt.solve_from_problem(ctx, b, precision="f64", queue_capacity=1000)
    xa0, xb0 = ga.fields()[0], gb.fields()[0]
    with pytest.raises(frt.FrtError) as e:
        frt.batch_step([ga, gb], [a.dt_s, b.dt_s])
    assert e.value.code == frt.FRT_EOVERFLOW
    for g, x0 in ((ga, xa0), (gb, xb0)):
        L = g.ledger()
        assert np.array_equal(g.fields()[0], x0)
        assert L["steps"] == 0 and L["emitted"] == 0 and L["err_flags"] == 0
    # the solve that fits then steps as it does alone
    ga.step(a.dt_s)
    r = _gpu(ctx, a, 1, precision="f64", queue_capacity=8_000_000)
    assert float(np.abs(r.fields()[0] - ga.fields()[0]).max()) <= 1e-12


def test_invalid_inputs_are_rejected(ctx):
    p = W.stromgren_c1(n=8)
    s = frt.Solve(ctx, sigma_bins=[W.SIGMA_HI_0])
    bad = p.n_H.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(frt.FrtError) as e:
        s.load_grid(bad, p.dx_cm * 8)
    assert e.value.code == frt.FRT_EINVAL
    s.load_grid(p.n_H, p.dx_cm * 8)
    with pytest.raises(frt.FrtError) as e:
        s.load_sources(np.array([[-1.0, 0, 0]]), np.array([[1e49]]))
    assert e.value.code == frt.FRT_EINVAL
    with pytest.raises(frt.FrtError) as e:
        s.step(1e13)
    assert e.value.code == frt.FRT_ESTATE


def test_many_splits_per_step_at_finite_c(ctx):
    # N_min = 16: split radius 0.24 * 2^l cells, so a packet cast this step
    # splits six times within its 13-cell travel; the pass count bounded by
    # the split radii one step's travel can cross must still finish the step
    rng = np.random.Generator(np.random.PCG64(123))
    n = 24
    dx = W.cmpc_h_to_cm(0.15625)
    nH = W.lognormal_white(rng, (n, n, n), 2e-4, 0.7).astype(np.float32)
    pos = (rng.integers(2, n - 2, size=(3, 3)) + 0.5) * dx
    w, sig = W.blackbody_bins(2)
    ndot = np.array([3e52, 1e52, 5e51])[:, None] * w[None, :]
    p = W.Problem(name="many splits", shape=(n, n, n), dx_cm=dx, n_H=nH, x_HI0=np.full((n, n, n), 1e-3), kappa=None,
                  src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig, dt_s=W.MYR, n_steps=3, c_ray=W.C_LIGHT,
                  flux_floor=1e-3, max_level=9, n_ray_min=16.0, seed=124)
    g = _gpu(ctx, p, 3)
    assert g.ledger()["splits"] > 0
    _compare(_oracle(p, 3), g, 1e-3, 1e-4, "N_min 16 finite c")


def _carried_radii(g, n_src, ncell, fp64):
    """Distances from their sources (cells) of the packets a solve carries,
    read from its checkpoint: 8 u64 header (the carried count last), the
    ledger (176 bytes), x_HI, the rotation quaternions of the steps so far,
    then the packet records (64 bytes in FP32 with r at byte 20, 112 in FP64
    with r at byte 24)."""
    blob = g.save()
    hdr = np.frombuffer(blob[:64], dtype=np.uint64)
    step, nc = int(hdr[2]), int(hdr[7])
    off = 64 + 176 + 8 * ncell + 32 * step * n_src
    size, at, dt = (112, 24, np.float64) if fp64 else (64, 20, np.float32)
    recs = np.frombuffer(blob[off: off + nc * size], dtype=np.uint8).reshape(nc, size)
    return recs[:, at: at + np.dtype(dt).itemsize].copy().view(dt).reshape(-1).astype(np.float64)


@pytest.mark.parametrize("precision,rtol", [("f64", 1e-12), ("f32", 2e-6)])
def test_carried_packets_travel_exactly_c_dt_per_step(ctx, precision, rtol):
    # §3.1 packets move c dt per step: in a transparent box the packets cast
    # at step j sit at (k - j + 1) c dt from their source after step k, each
    # shell with the HEALPix count of the level reached at its radius
    n, dx, dt, step_cells = 64, 1e21, 1e13, 3.7
    shape = (n, n, n)
    p = W.Problem(name="transparent", shape=shape, dx_cm=dx, n_H=np.full(shape, 1e-3, np.float32),
                  x_HI0=np.zeros(shape), kappa=None, src_pos_cm=np.array([[32.5 * dx] * 3]),
                  ndot_bins=np.array([[1e50]]), sigma_bins=np.array([6.3e-18]), dt_s=dt, n_steps=4,
                  c_ray=step_cells * dx / dt, alpha_B=0.0, max_level=12, seed=3)
    g = frt.solve_from_problem(ctx, p, precision=precision)
    for k in range(1, 5):
        g.step(dt)
        r = _carried_radii(g, 1, n ** 3, precision == "f64")
        assert r.size == g.ledger()["n_in_flight"]
        shells = np.rint(r / step_cells)
        assert np.allclose(r, shells * step_cells, rtol=rtol, atol=0), (k, np.abs(r / (shells * step_cells) - 1).max())
        for m in range(1, k + 1):
            levels = sum(1 for l in range(13) if O.split_radius(1.0, l, 1.0) <= m * step_cells)
            assert int((shells == m).sum()) == 12 * 4 ** levels, (k, m)


@pytest.mark.parametrize("precision,rtol", [("f64", 1e-10), ("f32", 2e-3)])
def test_flux_floor_drops_where_the_photons_fall_below_it(ctx, precision, rtol):
    # Uniform neutral gas, n_H sigma_0 dx = 1, two bins (cross-section ratio
    # 1 and 1/3, photons 0.6 / 0.4), floor 1e-3 (reading R9): the summed
    # photons of a packet fall below the floor at r* = 17.97 cells, after
    # its last split (level 5): all 12 4^5 packets are dropped, each with
    # S(r_drop) = 0.6 e^-r + 0.4 e^-(r/3) of its cast photons at the first
    # face it crosses beyond r*, and everything else is absorbed.
    from scipy.optimize import brentq
    n, dx, sig0 = 64, 1e21, 6.3e-18
    shape = (n, n, n)
    nH = np.full(shape, 1.0 / (sig0 * dx), np.float32)
    w = np.array([0.6, 0.4])
    src = np.array([32.5, 32.5, 32.5])
    p = W.Problem(name="floor", shape=shape, dx_cm=dx, n_H=nH, x_HI0=np.ones(shape), kappa=None,
                  src_pos_cm=src[None, :] * dx, ndot_bins=(1e50 * w)[None, :], sigma_bins=np.array([sig0, sig0 / 3]),
                  dt_s=1e13, n_steps=1, c_ray=np.inf, flux_floor=1e-3, alpha_B=0.0, max_level=12, seed=11)
    g = _gpu(ctx, p, 1, precision=precision)
    L = g.ledger()
    tau_cell = float(nH[0, 0, 0]) * sig0 * dx
    S = lambda r: w[0] * np.exp(-tau_cell * r) + w[1] * np.exp(-tau_cell * r / 3)
    r_star = brentq(lambda r: S(r) - 1e-3, 10, 30)
    R = O.rotation(p.uniforms(0)[0])
    d = np.stack([R @ O.healpix_center(5, q) for q in range(12 * 4 ** 5)])
    # the first face beyond r* along each packet's line from the source
    r_drop = np.full(d.shape[0], np.inf)
    for a in range(3):
        da = d[:, a]
        pos = src[a] + r_star * da
        k = np.where(da > 0, np.floor(pos) + 1, np.ceil(pos) - 1)
        r_drop = np.minimum(r_drop, np.where(da != 0, (k - src[a]) / np.where(da != 0, da, 1), np.inf))
    emitted = 1e50 * p.dt_s
    expect = (emitted / (12 * 4 ** 5) * S(r_drop)).sum()
    print(f"[floor {precision}] dropped {L['dropped']:.6e} expected {expect:.6e}", flush=True)
    assert L["n_dropped"] == 12 * 4 ** 5 and L["n_escaped"] == 0
    assert L["dropped"] == pytest.approx(expect, rel=rtol)
    assert L["absorbed_HI"] + L["dropped"] == pytest.approx(L["emitted"], rel=1e-9)
