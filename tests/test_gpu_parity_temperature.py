"""Temperature evolution (§4.1, Eq. temp_evolution_standard) on the GPU
against the FP64 oracle on the same seeded inputs: a uniform box with a
central blackbody source starting at 100 K (the paper's Test 2 set-up,
small) and a clumpy box with sub-grid absorbers (which take their share of
the photons and heat nothing) at a finite packet speed, with backward-Euler
and time-averaged chemistry.  Bars: FP64 march, x_HI within 1e-9, T within
1e-8 relative, the photo-heating ledger within 1e-9; FP32 march, x_HI within
1e-3, T within 1e-3 relative (T follows the FP32 rates of absorption through
the cooling curve), the heating within 1e-4; the photon ledger closes as
without the temperature.  Checkpoints and bookmarks keep T; a batch of
solves with and without it equals each alone; the paper's Test 2 trend."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

KPC = 3.0857e21
TERMS = ("emitted", "absorbed_HI", "absorbed_sub", "escaped", "dropped", "in_flight")


@pytest.fixture(scope="module")
def ctx():
    return frt.Context(0)


def _uniform(n=20, steps=6, K=0, dt_myr=10.0):
    dx = 13.2 * KPC / n
    w, sig = W.blackbody_bins(3, T_bb=1e5)
    return W.Problem(name=f"test2_{n}^3", shape=(n, n, n), dx_cm=dx, n_H=np.full((n, n, n), 1e-3, np.float32),
                     x_HI0=np.ones((n, n, n)), kappa=None, src_pos_cm=np.array([[n / 2, n / 2, n / 2]]) * dx,
                     ndot_bins=np.array([5e48 * w]), sigma_bins=sig, dt_s=dt_myr * W.MYR, n_steps=steps,
                     c_ray=np.inf, n_ray_min=4.0, chem_iterations=K, seed=17,
                     T=np.full((n, n, n), 100.0, np.float32), temperature=True, heat_ev=W.blackbody_heat(3, T_bb=1e5))


def _clumpy(n=24, steps=5, K=0, seed=19):
    p = W.lognormal_c2(n=n, n_src=5, n_steps=steps, box_cmpc_h=20.0 * n / 128, seed=seed)
    p.x_HI0 = np.full(p.shape, 0.5)
    p.c_ray = 3.0 * p.dx_cm / p.dt_s
    p.chem_iterations = K
    p.temperature = True
    p.heat_ev = W.blackbody_heat(p.n_bins, T_bb=5e4)
    p.T = np.full(p.shape, 2e3, np.float32)
    return p


def _oracle(p, steps):
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    for s in range(steps):
        o.step(p.dt_s, p.uniforms(s))
    return o


def _gpu(ctx, p, steps, **kw):
    g = frt.solve_from_problem(ctx, p, **kw)
    for _ in range(steps):
        g.step(p.dt_s)
    return g


def _compare(o, g, x_tol, t_rtol, h_rtol, label):
    xo, xg = o.fields()[0], g.fields()[0]
    To, Tg = o.temperature(), g.temperature()
    Lo, Lg = o.ledger(), g.ledger()
    dx = float(np.abs(xo - xg).max())
    dT = float(np.max(np.abs(Tg / To - 1)))
    dh = abs(Lg["heat_in"] / Lo["heat_in"] - 1)
    print(f"[{label}] max|dx_HI| {dx:.2e}  max|dT/T| {dT:.2e}  heat_in {dh:.2e}  T range {To.min():.0f}-{To.max():.0f} K",
          flush=True)
    assert dx <= x_tol, label
    assert dT <= t_rtol, label
    assert dh <= h_rtol, label
    E = Lo["emitted"]
    for k in TERMS:
        assert abs(Lo[k] - Lg[k]) <= max(x_tol, 1e-9) * E, (label, k)
    closure = abs(Lg["emitted"] - sum(Lg[k] for k in TERMS[1:]) - Lg["lost"]) / Lg["emitted"]
    assert closure <= 1e-9 and Lg["err_flags"] == 0, label


@pytest.mark.parametrize("K", [0, 2])
@pytest.mark.parametrize("precision,x_tol,t_rtol,h_rtol", [("f64", 1e-9, 1e-8, 1e-9), ("f32", 1e-3, 1e-3, 1e-4)])
def test_uniform_box_from_100K_matches_the_oracle(ctx, K, precision, x_tol, t_rtol, h_rtol):
    p = _uniform(K=K)
    _compare(_oracle(p, p.n_steps), _gpu(ctx, p, p.n_steps, precision=precision), x_tol, t_rtol, h_rtol,
             f"uniform K={K} {precision}")


@pytest.mark.parametrize("K", [0, 2])
@pytest.mark.parametrize("precision,x_tol,t_rtol,h_rtol", [("f64", 1e-9, 1e-8, 1e-9), ("f32", 1e-3, 1e-3, 1e-4)])
def test_clumpy_box_with_subgrid_absorbers_matches_the_oracle(ctx, K, precision, x_tol, t_rtol, h_rtol):
    p = _clumpy(K=K)
    _compare(_oracle(p, p.n_steps), _gpu(ctx, p, p.n_steps, precision=precision), x_tol, t_rtol, h_rtol,
             f"clumpy K={K} {precision}")


def test_checkpoint_and_bookmark_keep_the_temperature(ctx):
    p = _clumpy(steps=4)
    ref = _gpu(ctx, p, 4, precision="f64")
    a = _gpu(ctx, p, 2, precision="f64")
    blob = a.save()
    b = frt.solve_from_problem(ctx, p, precision="f64")
    b.load(blob)
    for _ in range(2):
        b.step(p.dt_s)
    # FP64 deposits differ only in the order of their atomic additions; T,
    # through the cooling curve, moves a little more than x_HI
    assert np.abs(ref.temperature() / b.temperature() - 1).max() <= 1e-10
    assert np.abs(ref.fields()[0] - b.fields()[0]).max() <= 1e-12
    assert ref.ledger()["heat_in"] == pytest.approx(b.ledger()["heat_in"], rel=1e-12)
    a.mark()
    for _ in range(2):
        a.step(p.dt_s)
    T1 = a.temperature()
    a.rewind()
    for _ in range(2):
        a.step(p.dt_s)
    assert np.abs(a.temperature() / T1 - 1).max() <= 1e-10


def test_batch_with_and_without_temperature_equals_each_alone(ctx):
    pt = _clumpy(steps=3, seed=23)
    pn = _clumpy(steps=3, seed=29)
    pn.temperature = False
    pn.T = None                     # no temperature loaded either: none to read
    at, an = _gpu(ctx, pt, 3, precision="f64"), _gpu(ctx, pn, 3, precision="f64")
    bt = frt.solve_from_problem(ctx, pt, precision="f64")
    bn = frt.solve_from_problem(ctx, pn, precision="f64")
    frt.batch_run([bt, bn], [pt.dt_s, pn.dt_s], 3, graph=True, check_every=3)
    assert np.abs(at.temperature() / bt.temperature() - 1).max() <= 1e-10
    for a, b in ((at, bt), (an, bn)):
        assert np.abs(a.fields()[0] - b.fields()[0]).max() <= 1e-12
    with pytest.raises(frt.FrtError) as e:
        bn.temperature()
    assert e.value.code == frt.FRT_ESTATE


def test_temperature_parameters_are_checked(ctx):
    for kw in ({"temperature": True, "heat_ev": [-1.0]}, {"temperature": True, "hubble_s": -1e-18},
               {"temperature": True, "cmb_z": float("nan")}, {"temperature": True, "opacity_mode": 1, "t_reion": 0.0},
               {"temperature": True, "opacity_mode": 1, "t_reion": float("inf")},
               {"temperature": True, "opacity_mode": 1, "spectral_index": -0.5},
               {"temperature": True, "opacity_mode": 1, "spectral_index": float("nan")}):
        with pytest.raises(frt.FrtError) as e:
            frt.Solve(ctx, sigma_bins=[6.3e-18], **kw)
        assert e.value.code == frt.FRT_EINVAL, kw


def test_papers_test2_front_ends_beyond_the_isothermal_radius(ctx):
    # the oracle's Test 2 pin, run on the GPU (FP32 march, K = 3, 24^3,
    # 10 Myr steps to 500 Myr), and its radius against the oracle's
    p = _uniform(n=24, steps=50, K=3)
    g = _gpu(ctx, p, 50)
    o = _oracle(p, 50)
    n32, alpha, Nd = float(np.float32(1e-3)), 2.59e-13, 5e48
    t_rec, t = 1 / (alpha * n32), 50 * p.dt_s
    r_S = (3 * Nd / (4 * np.pi * alpha * n32 ** 2)) ** (1 / 3)
    ratio = {}
    for k, s in (("gpu", g), ("oracle", o)):
        x = s.fields()[0]
        r = (3 * float(np.sum(1 - x)) * p.dx_cm ** 3 / (4 * np.pi)) ** (1 / 3)
        ratio[k] = r / (r_S * (1 - np.exp(-t / t_rec)) ** (1 / 3))
    print(f"r / r_isothermal: GPU {ratio['gpu']:.4f}, oracle {ratio['oracle']:.4f}", flush=True)
    assert 1.04 <= ratio["gpu"] <= 1.25
    assert abs(ratio["gpu"] - ratio["oracle"]) <= 1e-3
