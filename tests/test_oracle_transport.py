"""Pins of the oracle's transport (§3.1 packets, §3.2 splitting, §4.1-4.2
deposition) and chemistry (Eq. ion_balance_eqn, backward Euler).  Expected
values come from an independent slab-intersection geometry, closed forms,
ODE solvers, counting arguments and the paper's equations, never from the
oracle itself."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W

SIG = [6.3e-18, 2.1e-18, 0.7e-18]


def _slab_paths(shape, dx, o, d):
    """Per-cell entry distance and path length of the ray o + t d (t >= 0)
    through every cell of the box, by the slab method on each cell's box."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lo = np.stack([i * dx, j * dx, k * dx], axis=-1).astype(float)
    hi = lo + dx
    par = (d == 0)
    dd = np.where(par, 1.0, d)
    t1 = (lo - o) / dd
    t2 = (hi - o) / dd
    # an axis the ray runs parallel to admits only the slab [lo, hi) holding o
    inside = (lo <= o) & (o < hi)
    tmin = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(t1, t2))
    tmax = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(t1, t2))
    t_in = np.maximum(tmin.max(axis=-1), 0.0)
    t_out = tmax.min(axis=-1)
    length = np.clip(t_out - t_in, 0.0, None)
    return t_in, length


def _problem(shape, dx, nH, x, kappa, sig):
    return O.Oracle(shape=shape, dx_cm=dx, sigma_bins=sig, alpha_B=W.ALPHA_B_1E4, n_H=nH,
                    kappa=kappa, x_HI0=x, max_level=0, c_ray=np.inf)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("with_kappa", [False, True])
def test_single_ray_deposits_match_slab_geometry(seed, with_kappa):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    shape = (9, 10, 11)
    dx = 2.0e21
    nH = (1e-3 * np.exp(rng.standard_normal(shape))).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape)
    kappa = (rng.uniform(0, 3, shape) / (10 * dx)).astype(np.float32) if with_kappa else None
    o = np.array([rng.uniform(0.5, 10.5), rng.uniform(0.5, 9.5), rng.uniform(0.5, 8.5)]) * dx
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    N = np.array([3e50, 2e50, 1e50])
    dt = 1e13
    orc = _problem(shape, dx, nH, x, kappa, SIG)
    N_exit, gamma, ncross = orc.transmit(o, d, N, dt)

    t_in, ds = _slab_paths(shape, dx, o, d)
    hit = ds > 0
    order = np.argsort(t_in[hit], kind="stable")
    cells = np.argwhere(hit)[order]
    nhi = (nH.astype(float) * x)
    kap = np.zeros(shape) if kappa is None else kappa.astype(float)
    V = dx ** 3
    expect = np.zeros(shape)
    Nin = N.astype(float).copy()
    for c in map(tuple, cells):
        for b, s in enumerate(SIG):
            lam = 1.0 / (nhi[c] * s + kap[c])
            # Eq. gamma_avg_subgrid with lambda = 1/(n_HI sigma + kappa)
            expect[c] += Nin[b] * (1 - math.exp(-ds[c] / lam)) * s * lam / (V * dt)
            Nin[b] *= math.exp(-ds[c] / lam)
    assert ncross == len(cells)
    assert np.allclose(gamma, expect, rtol=1e-10, atol=0)
    # exact exp(-tau) transmission along the whole path
    for b, s in enumerate(SIG):
        tau = ((nhi * s + kap) * ds).sum()
        assert N_exit[b] == pytest.approx(N[b] * math.exp(-tau), rel=1e-12)


def test_deposit_equals_absorbed_over_neutral_atoms():
    # Eq. gamma_initial_standard (kappa = 0): Gamma_i n_HI V dt equals the
    # photons the cell absorbed, N_in (1 - exp(-n_HI sigma ds)).
    shape = (6, 6, 6)
    dx = 1e21
    nH = np.full(shape, 2e-3, dtype=np.float32)
    x = np.full(shape, 0.3)
    orc = _problem(shape, dx, nH, x, None, [6.3e-18])
    o = np.array([0.2, 0.3, 0.1]) * dx
    d = np.array([0.6, 0.48, 0.64])
    N = np.array([1e52])
    N_exit, gamma, _ = orc.transmit(o, d, N, 1.0)
    t_in, ds = _slab_paths(shape, dx, o, d)
    absorbed_total = N[0] - N_exit[0]
    nhi = float(np.float32(2e-3)) * 0.3
    got = (gamma * nhi * dx ** 3 * 1.0).sum()
    assert got == pytest.approx(absorbed_total, rel=1e-12)


def test_optically_thin_limit_and_path_sum():
    # Eq. gamma_initial_subgrid: with no absorber Gamma_i = N sigma ds/(V dt);
    # the per-cell lengths add up to the distance to the box boundary.
    shape = (8, 8, 8)
    dx = 1e21
    orc = _problem(shape, dx, np.full(shape, 1e-3, dtype=np.float32), np.zeros(shape), None, [6.3e-18])
    o = np.array([4.3, 4.1, 3.7]) * dx
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    N = np.array([1e50])
    N_exit, gamma, _ = orc.transmit(o, d, N, 2.0)
    assert N_exit[0] == N[0]
    t_in, ds = _slab_paths(shape, dx, o, d)
    assert np.allclose(gamma, N[0] * 6.3e-18 * ds / (dx ** 3 * 2.0), rtol=1e-12, atol=0)
    exit_t = min(((8 * dx if c > 0 else 0.0) - oc) / c for oc, c in zip(o, d))
    assert ds.sum() == pytest.approx(exit_t, rel=1e-12)


def test_face_and_corner_ties_do_not_lose_length():
    # rays through cell edges and corners: lengths still add up, no cell twice
    shape = (5, 5, 5)
    dx = 1.0e21
    orc = _problem(shape, dx, np.full(shape, 1e-3, dtype=np.float32), np.zeros(shape), None, [6.3e-18])
    for o, d in [((0.0, 0.0, 0.0), (1, 1, 1)), ((2.5, 2.5, 2.5), (1, 1, 0)), ((1.0, 2.0, 0.5), (1, -1, 1)),
                 ((5.0, 5.0, 5.0), (-1, -1, -1)), ((2.0, 2.5, 2.5), (-1, 0, 0))]:
        o = np.array(o, dtype=float) * dx
        d = np.array(d, dtype=float)
        d /= np.linalg.norm(d)
        _, gamma, _ = orc.transmit(o, d, np.array([1e50]), 1.0)
        t_in, ds = _slab_paths(shape, dx, o, d)
        length = gamma * dx ** 3 / (1e50 * 6.3e-18)
        assert length.sum() == pytest.approx(ds.sum(), rel=1e-12)


def _transparent(n, c_ray=np.inf, cap_cells=0.0, src=None):
    shape = (n, n, n)
    dx = 1e21
    o = O.Oracle(shape=shape, dx_cm=dx, sigma_bins=[6.3e-18], alpha_B=0.0, n_H=np.full(shape, 1e-3, np.float32),
                 x_HI0=np.zeros(shape), max_level=20, c_ray=c_ray, max_dist_cm=cap_cells * dx)
    o.set_sources(np.array([src if src is not None else [n / 2 * dx] * 3]), np.array([[1e50]]))
    return o, dx


def test_split_counts_full_sphere():
    # A source at the centre of a 64^3 transparent box: r_split(l) =
    # 0.977 * 2^l cells, so levels 0..5 split inside the inscribed sphere
    # (r_split(5) = 31.3 < 32) and every level-6 ray escapes (Eq. Nray).
    o, _ = _transparent(64)
    o.step(1e13, W.rotation_uniforms(1, 0, 1))
    L = o.ledger()
    assert L["splits"] == sum(12 * 4 ** l for l in range(6))
    assert L["n_escaped"] == 12 * 4 ** 6
    assert L["escaped"] == pytest.approx(L["emitted"], rel=1e-14)
    # photons are shared equally among children: each escaping ray carries
    # exactly emitted / (12 * 4^6)
    assert L["emitted"] == pytest.approx(1e50 * 1e13, rel=1e-15)


def test_distance_cap_drops_every_last_level_ray():
    o, _ = _transparent(128, cap_cells=40.0)
    o.step(1e13, W.rotation_uniforms(2, 0, 1))
    L = o.ledger()
    assert L["n_dropped"] == 12 * 4 ** 6 and L["n_escaped"] == 0
    assert L["dropped"] == pytest.approx(L["emitted"], rel=1e-14)


def test_vertex_source_casts_only_into_the_box():
    o, dx = _transparent(16, src=[0.0, 0.0, 0.0])
    u = W.rotation_uniforms(9, 0, 1)
    o.step(1e13, u)
    R = O.rotation(u[0])
    dirs = np.stack([R @ O.healpix_center(0, p) for p in range(12)])
    inward = int(np.all(dirs > 0, axis=1).sum())
    L = o.ledger()
    assert L["crossings"] > 0 or inward == 0
    # every ray that points out of the octant leaves at casting
    assert L["n_escaped"] >= 12 - inward


def test_finite_speed_packets_carry_photons():
    # packets move c_ray * dt per step; what is in flight at step end is
    # carried and the ledger closes including it.
    o, dx = _transparent(64, c_ray=10 * 1e21 / 1e13)   # 10 cells per step
    for s in range(4):
        o.step(1e13, W.rotation_uniforms(3, s, 1))
        L = o.ledger()
        tot = L["absorbed_HI"] + L["absorbed_sub"] + L["escaped"] + L["dropped"] + L["in_flight"]
        assert tot == pytest.approx(L["emitted"], rel=1e-12)
        if s < 2:
            assert L["n_in_flight"] > 0 and L["n_escaped"] == 0


# ---------------------------------------------------------------- chemistry
def _residual(x, xn, g, nH, a, c, dt):
    return (xn - x) - dt * (-g * xn - c * nH * (1 - xn) * xn + a * nH * (1 - xn) ** 2)


def test_backward_euler_satisfies_its_implicit_equation():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(2000):
        x = rng.uniform(0, 1) ** 4
        g = 10 ** rng.uniform(-18, -9)
        nH = 10 ** rng.uniform(-5, -1)
        a = 2.59e-13 * rng.uniform(0.5, 2)
        c = rng.choice([0.0, 1e-15])
        dt = 10 ** rng.uniform(10, 16)
        xn = O.chemistry(x, g, nH, a, c, dt)
        assert 0.0 <= xn <= 1.0
        scale = 1 + dt * (g + 2 * a * nH + c * nH)
        assert abs(_residual(x, xn, g, nH, a, c, dt)) <= 1e-13 * scale


def test_backward_euler_closed_form_limits():
    # alpha = C = 0: x' = x / (1 + Gamma dt)
    for x, g, dt in [(1.0, 1e-12, 1e13), (1e-3, 3e-13, 5e14), (0.5, 1e-15, 1e12)]:
        assert O.chemistry(x, g, 1e-3, 0.0, 0.0, dt) == pytest.approx(x / (1 + g * dt), rel=1e-14)
    # dt -> inf: photo-ionization equilibrium Gamma n_HI = alpha n_e n_HII
    # (Eq. equilibrium_condition) with n_e = n_HII = n_H (1 - x)
    for g, nH in [(1e-12, 2e-4), (1e-14, 1e-2), (3e-13, 1e-3)]:
        x = O.chemistry(1.0, g, nH, 2.59e-13, 0.0, 1e30)
        assert g * x == pytest.approx(2.59e-13 * nH * (1 - x) ** 2, rel=1e-9)


def test_backward_euler_converges_to_the_ode():
    # Eq. ion_balance_eqn for pure H: dx/dt = -G x - C nH (1-x) x + a nH (1-x)^2
    g, nH, a, c = 2e-14, 1e-3, 2.59e-13, 1e-16
    T = 5e14
    ref = solve_ivp(lambda t, x: -g * x - c * nH * (1 - x) * x + a * nH * (1 - x) ** 2, (0, T), [1.0],
                    rtol=1e-12, atol=1e-14).y[0, -1]
    errs = []
    for n in (100, 200, 400):
        x = 1.0
        for _ in range(n):
            x = O.chemistry(x, g, nH, a, c, T / n)
        errs.append(abs(x - ref))
    assert errs[-1] < 1e-3 * ref
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3   # first order


def test_pure_recombination_matches_analytic():
    # Gamma = 0: d(1-x)/dt = -a nH (1-x)^2 -> (1-x)(t) = 1/(1/(1-x0) + a nH t)
    a, nH, x0, T = 2.59e-13, 1e-3, 1e-4, 3e15
    x = x0
    n = 4000
    for _ in range(n):
        x = O.chemistry(x, 0.0, nH, a, 0.0, T / n)
    exact = 1 - 1 / (1 / (1 - x0) + a * nH * T)
    assert x == pytest.approx(exact, rel=2e-3)


# ---------------------------------------------------------- flux floor, travel
def _first_face_after(src_cells, d, r_lo, r_hi):
    """For each direction d[k], the smallest distance r in (r_lo, r_hi) at
    which the line src + r d crosses a cell face (integer coordinate), by
    the slab geometry of each axis; inf if none."""
    best = np.full(d.shape[0], np.inf)
    for a in range(3):
        da = d[:, a]
        ok = da != 0
        s = src_cells[a]
        # crossings s + r d = k for integers k; the first one beyond r_lo
        pos_lo = s + r_lo * da
        k = np.where(da > 0, np.floor(pos_lo) + 1, np.ceil(pos_lo) - 1)
        r = np.where(ok, (k - s) / np.where(ok, da, 1.0), np.inf)
        # the next crossing along this axis after r_lo (a crossing exactly at
        # r_lo belongs to the segment that ended there)
        r = np.where(r <= r_lo, r + np.abs(1.0 / np.where(ok, da, 1.0)), r)
        best = np.minimum(best, np.where(r < r_hi, r, np.inf))
    return best


def test_flux_floor_drops_at_the_first_segment_end_below_the_floor():
    # Uniform neutral gas with n_H sigma_0 dx = 1 and two bins (sigma ratio
    # 1 and 1/3, photons 0.6 / 0.4): a packet's photons relative to its cast
    # photons are S(r) = 0.6 e^-r + 0.4 e^-(r/3) at r cells from its source
    # (the optical depth depends only on the path length in uniform gas, also
    # across splits, which re-centre children at the same radius).  With the
    # floor f = 1e-3 (reading R9: the summed photons against f times the cast
    # photons divided by 4 per split) S crosses f at r* = 17.97 cells, after
    # the last split radius below it (r_split(4) = 15.6, r_split(5) = 31.3):
    # every level-5 packet is dropped at the first face it crosses beyond r*,
    # with S(r_drop) of its photons.  A per-bin floor test would drop at
    # 20.7 cells, a floor without the 4^-dl division right after the split.
    n, dx = 64, 1e21
    sig0 = 6.3e-18
    nH = 1.0 / (sig0 * dx)
    w = np.array([0.6, 0.4])
    ndot = 1e50 * w
    shape = (n, n, n)
    src = np.array([32.5, 32.5, 32.5])
    o = O.Oracle(shape=shape, dx_cm=dx, sigma_bins=[sig0, sig0 / 3], alpha_B=0.0,
                 n_H=np.full(shape, nH, np.float32), x_HI0=np.ones(shape), max_level=12,
                 flux_floor=1e-3, c_ray=np.inf)
    o.set_sources(src[None, :] * dx, ndot[None, :])
    u = W.rotation_uniforms(11, 0, 1)
    dt = 1e13
    o.step(dt, u)
    L = o.ledger()

    nH32 = float(np.float32(nH))
    tau_cell = nH32 * sig0 * dx                       # as the oracle sees the float32 density
    S = lambda r: w[0] * np.exp(-tau_cell * r) + w[1] * np.exp(-tau_cell * r / 3)
    from scipy.optimize import brentq
    r_star = brentq(lambda r: S(r) - 1e-3, 10, 30)
    r_split = [O.split_radius(1.0, l, 1.0) for l in range(7)]
    assert r_split[4] < r_star < r_split[5]
    R = O.rotation(u[0])
    dirs = np.stack([R @ O.healpix_center(5, p) for p in range(12 * 4 ** 5)])
    r_drop = _first_face_after(src, dirs, r_star, r_split[5])
    assert np.all(np.isfinite(r_drop))
    # no face crossing is so close to r* that rounding could move the drop
    just_before = _first_face_after(src, dirs, r_split[4], r_star)
    assert np.min(np.abs(r_drop - r_star)) > 1e-6 and np.min(np.abs(just_before[np.isfinite(just_before)] - r_star)) > 1e-6

    emitted = ndot.sum() * dt
    per_ray = emitted / (12 * 4 ** 5)
    expect_dropped = (per_ray * S(r_drop)).sum()
    assert L["n_dropped"] == 12 * 4 ** 5 and L["n_escaped"] == 0
    assert L["splits"] == sum(12 * 4 ** l for l in range(5))
    assert L["dropped"] == pytest.approx(expect_dropped, rel=1e-10)
    assert L["absorbed_HI"] == pytest.approx(emitted - expect_dropped, rel=1e-12)


def test_carried_packets_travel_exactly_c_dt_per_step():
    # §3.1: a packet moves c dt per step whatever it crosses.  In a
    # transparent box the packets cast at step j sit at (k - j + 1) c dt from
    # their source after step k (children are re-centred at their parent's
    # radius), and each such shell holds the HEALPix count of the level
    # reached at that radius (Eqs. Nray, r_split).
    n, dx, dt = 64, 1e21, 1e13
    step_cells = 3.7
    o, _ = _transparent(n, c_ray=step_cells * dx / dt)
    for k in range(1, 5):
        o.step(dt, W.rotation_uniforms(3, k - 1, 1))
        r = o.flight_radii() / dx
        L = o.ledger()
        assert r.size == L["n_in_flight"]
        shells = np.rint(r / step_cells)
        assert np.allclose(r, shells * step_cells, rtol=1e-13, atol=0)
        for m in range(1, k + 1):
            levels = sum(1 for l in range(20) if O.split_radius(1.0, l, 1.0) <= m * step_cells)
            assert int((shells == m).sum()) == 12 * 4 ** levels, (k, m)
        assert int(shells.min()) == 1 and int(shells.max()) == k
        assert L["in_flight"] == pytest.approx(L["emitted"], rel=1e-13)
