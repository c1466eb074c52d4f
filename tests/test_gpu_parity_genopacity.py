"""GPU (HIP, gfx950) versus the FP64 oracle in the Generalized Opacity Mode
(§4.2): ionized-phase absorption coefficient, rate over the ionized part of
each cell, moving-screen fronts that stop packets and advance the ionized
fraction.  Bars as elsewhere: x_HI (here 1 - x_ion) within 1e-3 absolute
with the FP32 march and 1e-9 with the FP64 march, every ledger term (the
front term included) within 1e-4 of emitted, closure 1e-9."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "absorbed_front", "front_excess", "escaped", "dropped", "in_flight")
DX = W.cmpc_h_to_cm(0.15625)


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
    assert dx.max() <= x_tol, f"{label}: x_HI differs by {dx.max():.3e}"
    for k, v in worst.items():
        assert v <= led_tol, f"{label}: ledger term {k} differs by {v:.3e} of emitted"
    closure = abs(Lg["emitted"] - sum(Lg[k] for k in TERMS[1:]) - Lg["lost"]) / Lg["emitted"]
    assert closure <= 1e-9, f"{label}: GPU ledger does not close ({closure:.2e})"
    assert Lg["err_flags"] == 0 and Lg["lost"] == 0


def _fronts_box(n, seed, n_src=5, bins=4, c_ray=W.C_LIGHT, steps=4):
    # lognormal gas, mostly ionized with scattered partly ionized and neutral
    # cells, ionized-gas mean free path ~5 cells
    rng = np.random.Generator(np.random.PCG64(seed))
    nH = W.lognormal_white(rng, (n, n, n), 2e-4, 1.0).astype(np.float32)
    kap = (W.lognormal_white(rng, (n, n, n), 1.0, 0.5) / (5 * DX)).astype(np.float32)
    u = rng.uniform(size=(n, n, n))
    xi0 = np.where(u < 0.9, 1.0, np.where(u < 0.95, 0.0, rng.uniform(size=(n, n, n))))
    w, sig = W.blackbody_bins(bins)
    pos = (rng.integers(0, n, size=(n_src, 3)) + 0.5) * DX
    ndot = (10 ** rng.uniform(51, 53, size=n_src))[:, None] * w[None, :]
    return W.Problem(name=f"gen_{n}^3", shape=(n, n, n), dx_cm=DX, n_H=nH, x_HI0=1.0 - xi0, kappa=kap,
                     src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig, dt_s=W.MYR, n_steps=steps, c_ray=c_ray,
                     flux_floor=1e-3, seed=seed, opacity_mode=1, he_chi=0.08)


@pytest.mark.parametrize("precision,x_tol,led_tol", [("f32", 1e-3, 1e-4), ("f64", 1e-9, 1e-9)])
@pytest.mark.parametrize("n,c_ray", [(24, W.C_LIGHT), (27, np.inf)])
def test_fronts_in_clumpy_gas(ctx, precision, x_tol, led_tol, n, c_ray):
    p = _fronts_box(n, 51 + n, c_ray=c_ray)
    _compare(_oracle(p, 4), _gpu(ctx, p, 4, precision=precision), x_tol, led_tol,
             f"generalized {n}^3 c={'inf' if np.isinf(c_ray) else 'c'} {precision}")


def test_front_sphere_in_neutral_gas(ctx):
    n, nh, Nd = 24, 2e-5, 3e51
    p = W.Problem(name="front sphere", shape=(n, n, n), dx_cm=DX, n_H=np.full((n, n, n), nh, np.float32),
                  x_HI0=np.ones((n, n, n)), kappa=np.zeros((n, n, n), np.float32),
                  src_pos_cm=np.array([[11.5, 11.5, 11.5]]) * DX, ndot_bins=np.array([[Nd]]),
                  sigma_bins=np.array([6.3e-18]), dt_s=0.1 * W.MYR, n_steps=40, c_ray=np.inf, seed=1,
                  opacity_mode=1, he_chi=0.08)
    g = _gpu(ctx, p, 40)
    _compare(_oracle(p, 40), g, 1e-3, 1e-4, "front sphere")
    x, _ = g.fields()
    R_num = (3 * float(np.sum(1 - x)) / (4 * np.pi)) ** (1 / 3)
    R_an = (3 * Nd * 40 * p.dt_s / (4 * np.pi * 1.08 * nh)) ** (1 / 3) / DX
    assert R_num == pytest.approx(R_an, rel=0.03)


def test_ionized_gas_matches_standard_mode_rates(ctx):
    # kappa = n_HI sigma_0 with x_ion = 1: the rate field of Standard Mode
    n = 20
    rng = np.random.Generator(np.random.PCG64(61))
    nH = W.lognormal_white(rng, (n, n, n), 2e-4, 1.0).astype(np.float32)
    xh = rng.uniform(1e-3, 1e-2, size=(n, n, n))
    w, sig = W.blackbody_bins(3)
    kap = (nH.astype(np.float64) * xh * sig[0]).astype(np.float32)
    xh_std = kap.astype(np.float64) / (nH.astype(np.float64) * sig[0])
    pos = (rng.integers(0, n, size=(3, 3)) + 0.5) * DX
    ndot = np.array([1e52, 3e51, 2e52])[:, None] * w[None, :]
    base = dict(shape=(n, n, n), dx_cm=DX, n_H=nH, src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig, dt_s=W.MYR,
                n_steps=1, c_ray=np.inf, seed=62)
    std = _gpu(ctx, W.Problem(name="std", x_HI0=xh_std, kappa=None, **base), 1)
    gen = _gpu(ctx, W.Problem(name="gen", x_HI0=np.zeros((n, n, n)), kappa=kap, opacity_mode=1, **base), 1)
    gs, gg = std.fields()[1].astype(np.float64), gen.fields()[1].astype(np.float64)
    assert np.abs(gs - gg).max() <= 2e-3 * gs.max()
    Ls, Lg = std.ledger(), gen.ledger()
    for k in ("emitted", "absorbed_HI", "escaped", "dropped"):
        assert abs(Ls[k] - Lg[k]) <= 1e-4 * Ls["emitted"], k
    assert Lg["absorbed_front"] == 0.0


def test_batched_with_subgrid_standard_equals_alone(ctx):
    # a generalized and a standard solve with sub-grid opacity share the
    # 16^3 launch group
    a = _fronts_box(20, 71, n_src=3, bins=2)
    b = W.lognormal_c2(n=20, n_src=4, n_steps=3, box_cmpc_h=20.0 * 20 / 128, n_bins=2)
    alone = [_gpu(ctx, p, 3) for p in (a, b)]
    both = [frt.solve_from_problem(ctx, p) for p in (a, b)]
    for _ in range(3):
        frt.batch_step(both, [a.dt_s, b.dt_s])
    for p, s1, s2 in zip((a, b), alone, both):
        assert np.abs(s1.fields()[0] - s2.fields()[0]).max() <= 1e-5, p.name
        L1, L2 = s1.ledger(), s2.ledger()
        for k in TERMS:
            assert abs(L1[k] - L2[k]) <= 1e-6 * L1["emitted"], (p.name, k)


def test_checkpoint_resume_in_generalized_mode(ctx):
    p = _fronts_box(20, 81, n_src=3, bins=2, steps=4)
    ref = _gpu(ctx, p, 4)
    g = _gpu(ctx, p, 2)
    blob = g.save()
    h = frt.solve_from_problem(ctx, p)
    h.load(blob)
    for _ in range(2):
        h.step(p.dt_s)
    # equal up to the order of the atomic deposits and front counts
    assert np.abs(ref.fields()[0] - h.fields()[0]).max() <= 1e-5
    La, Lh = ref.ledger(), h.ledger()
    for k in TERMS:
        assert abs(La[k] - Lh[k]) <= 1e-6 * La["emitted"], k
    assert La["crossings"] == Lh["crossings"]


def test_generalized_parameters_are_checked(ctx):
    p = _fronts_box(8, 91, n_src=1, bins=1)
    for bad in (dict(chem_iterations=-1), dict(he_chi=-1.0), dict(opacity_mode=2)):
        q = W.Problem(**{**p.__dict__, **bad})
        with pytest.raises(frt.FrtError) as e:
            frt.solve_from_problem(ctx, q)
        assert e.value.code == frt.FRT_EINVAL


def test_nearly_ionized_cells_still_stop_packets(ctx):
    # cells ionized to within 1e-9 of 1 keep their fronts in the FP32 march
    # as in the FP64 state: a shell of them around the source stops every
    # packet
    n = 16
    xi = np.ones((n, n, n))
    zz, yy, xx = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    rr = np.sqrt((xx - 8.0) ** 2 + (yy - 8.0) ** 2 + (zz - 8.0) ** 2)
    xi[(rr > 4.0) & (rr < 6.0)] = 1.0 - 1e-9
    p = W.Problem(name="thin fronts", shape=(n, n, n), dx_cm=DX, n_H=np.full((n, n, n), 2e-4, np.float32),
                  x_HI0=1.0 - xi, kappa=np.full((n, n, n), 0.01 / DX, np.float32),
                  src_pos_cm=np.array([[8.0, 8.0, 8.0]]) * DX, ndot_bins=np.array([[1e52]]),
                  sigma_bins=np.array([6.3e-18]), dt_s=W.MYR, n_steps=1, c_ray=np.inf, seed=5,
                  opacity_mode=1, he_chi=0.08)
    g = _gpu(ctx, p, 1)
    _compare(_oracle(p, 1), g, 1e-3, 1e-4, "nearly ionized shell")
    L = g.ledger()
    # the shell has almost no atoms left: its front photons are nearly all excess
    assert L["escaped"] == 0.0 and L["absorbed_front"] + L["front_excess"] > 0.9 * L["emitted"]
    assert L["front_excess"] > 0.99 * (L["absorbed_front"] + L["front_excess"])


def test_graph_replay_equals_stepwise(ctx):
    # the front counts are cleared by the chemistry kernel, not by a memset,
    # so the step can be captured and replayed
    boxes = [_fronts_box(16, 101, n_src=2, bins=2, steps=3), _fronts_box(20, 102, n_src=3, bins=2, steps=3)]
    alone = [_gpu(ctx, b, 3) for b in boxes]
    replayed = [frt.solve_from_problem(ctx, b) for b in boxes]
    frt.batch_run(replayed, [b.dt_s for b in boxes], 3, graph=True)
    for b, a, r in zip(boxes, alone, replayed):
        assert np.abs(a.fields()[0] - r.fields()[0]).max() <= 1e-5, b.name
        La, Lr = a.ledger(), r.ledger()
        for k in TERMS:
            assert abs(La[k] - Lr[k]) <= 1e-6 * La["emitted"], (b.name, k)


def test_opacity_updated_between_steps(ctx):
    # the caller's opacity model changes kappa between steps (§4.2, Eq.
    # lambda_nu_general): the library and the oracle take the same new field
    p = _fronts_box(20, 111, n_src=3, bins=2, steps=4)
    rng = np.random.Generator(np.random.PCG64(112))
    new_kap = [(p.kappa * rng.uniform(0.3, 3.0, size=p.shape)).astype(np.float32) for _ in range(3)]
    g = frt.solve_from_problem(ctx, p)
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    for s in range(4):
        if s > 0:
            g.set_opacity(new_kap[s - 1])
            o.set_kappa(new_kap[s - 1])
        g.step(p.dt_s)
        o.step(p.dt_s, p.uniforms(s))
    _compare(o, g, 1e-3, 1e-4, "kappa updated between steps")
    # and the update matters: the same steps without it end elsewhere
    h = _gpu(ctx, p, 4)
    assert np.abs(h.fields()[0] - g.fields()[0]).max() > 1e-3


def test_opacity_update_needs_a_kappa_term(ctx):
    p = W.stromgren_c1(n=8, n_steps=1)      # Standard Mode without sub-grid opacity
    g = frt.solve_from_problem(ctx, p)
    with pytest.raises(frt.FrtError) as e:
        g.set_opacity(np.ones(p.shape, np.float32))
    assert e.value.code == frt.FRT_EINVAL


def test_no_sources_and_empty_cells(ctx):
    # without photons the screen stays put, except in cells without
    # hydrogen, which count as ionized from the first step (the same reading
    # on both sides)
    n = 12
    rng = np.random.Generator(np.random.PCG64(131))
    nH = W.lognormal_white(rng, (n, n, n), 2e-4, 1.0).astype(np.float32)
    nH[rng.uniform(size=nH.shape) < 0.05] = 0.0
    xi0 = rng.uniform(size=(n, n, n))
    p = W.Problem(name="dark", shape=(n, n, n), dx_cm=DX, n_H=nH, x_HI0=1.0 - xi0,
                  kappa=np.full((n, n, n), 0.1 / DX, np.float32), src_pos_cm=np.zeros((0, 3)),
                  ndot_bins=np.zeros((0, 1)), sigma_bins=np.array([6.3e-18]), dt_s=W.MYR, n_steps=2,
                  c_ray=W.C_LIGHT, seed=7, opacity_mode=1)
    g = _gpu(ctx, p, 2)
    o = O.Oracle(**p.oracle_kwargs())
    for s in range(2):
        o.step(p.dt_s, np.zeros(0))
    xg, xo = g.fields()[0], o.fields()[0]
    assert np.array_equal(xg, xo)
    assert np.abs(xg[nH > 0] - (1.0 - xi0)[nH > 0]).max() <= 1e-15
    assert np.all(xg[nH == 0] == 0.0)


KPC = 3.0857e21


def _test1(n, steps, dt_myr=1.0, K=2):
    """The paper's Test 1 (§5.1) for the equilibrium opacity: n_H = 1e-3,
    Ndot = 5e48 at 13.6 eV, alpha_B at 1e4 K, 13.2 kpc box, source at the
    centre, no input kappa, Generalized Opacity Mode with K marches a step."""
    dx = 13.2 * KPC / n
    return W.Problem(name=f"test1 {n}^3", shape=(n, n, n), dx_cm=dx, n_H=np.full((n, n, n), 1e-3, np.float32),
                     x_HI0=np.ones((n, n, n)), kappa=np.zeros((n, n, n), np.float32),
                     src_pos_cm=np.array([[n / 2, n / 2, n / 2]]) * dx, ndot_bins=np.array([[5e48]]),
                     sigma_bins=np.array([6.3e-18]), dt_s=dt_myr * W.MYR, n_steps=steps, c_ray=np.inf,
                     n_ray_min=4.0, seed=7, opacity_mode=1, chem_iterations=K)


@pytest.mark.parametrize("precision,x_tol,led_tol", [("f32", 1e-3, 1e-4), ("f64", 1e-9, 1e-9)])
def test_equilibrium_opacity_matches_the_oracle(ctx, precision, x_tol, led_tol):
    # the opacity of the ionized gas iterated with Gamma (photo-ionization
    # equilibrium, §5.1): the front of Test 1 on 16^3, and the clumpy box with
    # its input kappa added, both at K = 2 and 3 marches a step
    p = _test1(16, 12, dt_myr=4.0)
    _compare(_oracle(p, 12), _gpu(ctx, p, 12, precision=precision), x_tol, led_tol, f"equilibrium test1 {precision}")
    q = _fronts_box(20, 77, c_ray=W.C_LIGHT)
    q.chem_iterations = 3
    _compare(_oracle(q, 4), _gpu(ctx, q, 4, precision=precision), x_tol, led_tol, f"equilibrium clumpy {precision}")


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_equilibrium_stromgren_front(ctx, precision):
    # Test 1 to 3 t_rec on the GPU: the front within 0.5% of the analytic
    # r(t) = r_S (1 - e^-t/t_rec)^(1/3) after 2 t_rec (Eqs. r_of_t, rS, trec)
    n = 24
    alpha, nh, Nd = 2.59e-13, float(np.float32(1e-3)), 5e48
    t_rec = 1.0 / (alpha * nh)
    r_S = (3 * Nd / (4 * np.pi * alpha * nh * nh)) ** (1 / 3)
    steps = int(round(3.0 * t_rec / W.MYR))
    p = _test1(n, steps)
    g = frt.solve_from_problem(ctx, p, precision=precision)
    worst = 0.0
    for s in range(steps):
        g.step(p.dt_s)
        t = (s + 1) * p.dt_s
        if t > 2 * t_rec and s % 10 == 0:
            x, _ = g.fields()
            r = (3 * float(np.sum(1 - x)) * p.dx_cm ** 3 / (4 * np.pi)) ** (1 / 3)
            worst = max(worst, abs(r / (r_S * (1 - np.exp(-t / t_rec)) ** (1 / 3)) - 1))
    print(f"[test1 {precision}] worst |r/r(t) - 1| after 2 t_rec: {worst:.3%}", flush=True)
    assert worst <= 0.005
    L = g.ledger()
    closure = abs(L["emitted"] - sum(L[k] for k in TERMS[1:]) - L["lost"]) / L["emitted"]
    assert closure <= 1e-9


def test_equilibrium_checkpoint_and_bookmark_keep_the_rate(ctx):
    # the previous step's rate starts each step's iteration, so it is part of
    # the state: a resumed or rewound run repeats the continuous one
    p = _test1(16, 8, dt_myr=4.0, K=2)
    a = _gpu(ctx, p, 8, precision="f64")
    b = _gpu(ctx, p, 5, precision="f64")
    blob = b.save()
    c = frt.solve_from_problem(ctx, p, precision="f64")
    c.load(blob)
    for _ in range(3):
        c.step(p.dt_s)
    assert np.abs(a.fields()[0] - c.fields()[0]).max() <= 1e-12
    La, Lc = a.ledger(), c.ledger()
    for k in TERMS:
        assert La[k] == pytest.approx(Lc[k], rel=1e-12, abs=1e-12 * La["emitted"]), k
    # bookmark at step 5, three steps, rewind, the same three steps again
    b.mark()
    for _ in range(3):
        b.step(p.dt_s)
    x1 = b.fields()[0]
    b.rewind()
    for _ in range(3):
        b.step(p.dt_s)
    assert np.abs(b.fields()[0] - x1).max() <= 1e-12
    assert np.abs(b.fields()[0] - a.fields()[0]).max() <= 1e-12
