"""One packet through a fixed field on the GPU (frt_debug_cast, which runs
the production march kernels) against exact transmission and per-cell
deposits from an independent slab-intersection geometry (§4.1 Eq. tau_cell:
exp(-(n_HI sigma_nu + kappa) ds) per segment; Eq. gamma_avg_subgrid per
cell, Eq. gamma_initial_standard without kappa), and against the oracle's
own single-ray march.  FP64 march: photon totals to 1e-12 and the rate
(returned in FP32) to its rounding; FP32 march to 2e-5."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import frt
from paper_2409_04521_amd import workloads as W

pytestmark = pytest.mark.gpu

SIG = [6.3e-18, 2.1e-18, 0.7e-18]


@pytest.fixture(scope="module")
def ctx():
    return frt.Context(0)


def _slab_paths(shape, dx, o, d):
    """Per-cell entry distance and path length of o + t d (t >= 0), by the
    slab method on every cell's box."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lo = np.stack([i * dx, j * dx, k * dx], axis=-1).astype(float)
    hi = lo + dx
    par = d == 0
    dd = np.where(par, 1.0, d)
    t1, t2 = (lo - o) / dd, (hi - o) / dd
    inside = (lo <= o) & (o < hi)
    tmin = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(t1, t2))
    tmax = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(t1, t2))
    t_in = np.maximum(tmin.max(axis=-1), 0.0)
    return t_in, np.clip(tmax.min(axis=-1) - t_in, 0.0, None)


def _expected(shape, dx, nhi, kap, o, d, N, sig, dt):
    t_in, ds = _slab_paths(shape, dx, o, d)
    hit = ds > 0
    cells = np.argwhere(hit)[np.argsort(t_in[hit], kind="stable")]
    V = dx ** 3
    gam = np.zeros(shape)
    Nin = np.array(N, dtype=float)
    for c in map(tuple, cells):
        for b, s in enumerate(sig):
            k = nhi[c] * s + kap[c]
            if k > 0:
                gam[c] += Nin[b] * (1 - math.exp(-ds[c] * k)) * s / k / (V * dt)
            else:
                gam[c] += Nin[b] * s * ds[c] / (V * dt)
            Nin[b] *= math.exp(-ds[c] * k)
    return gam, Nin, len(cells)


# the rate field is returned in FP32 (rounding 6e-8), the photon totals in FP64
@pytest.mark.parametrize("precision,rtol,grtol", [("f64", 1e-12, 1.2e-7), ("f32", 2e-5, 2e-5)])
@pytest.mark.parametrize("with_kappa", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_one_packet_matches_slab_geometry(ctx, precision, rtol, grtol, with_kappa, seed):
    rng = np.random.Generator(np.random.PCG64(300 + seed))
    shape = (21, 37, 45)          # several bricks of every shape, ragged edges
    dx = 2.0e21
    nH = (1e-4 * np.exp(rng.standard_normal(shape))).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape)
    kappa = (rng.uniform(0, 3, shape) / (10 * dx)).astype(np.float32) if with_kappa else None
    o = np.array([rng.uniform(0.5, 44.5), rng.uniform(0.5, 36.5), rng.uniform(0.5, 20.5)]) * dx
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    N = np.array([3e50, 2e50, 1e50])
    dt = 1e13
    g = frt.Solve(ctx, sigma_bins=SIG, precision=precision, max_level=12)
    g.load_grid(nH, dx * shape[2], kappa=kappa, x_HI0=x)
    ab, es, nc, gam = g.debug_cast(o, d, N, dt)
    nhi = nH.astype(float) * x
    kap = np.zeros(shape) if kappa is None else kappa.astype(float)
    expect, N_exit, ncell = _expected(shape, dx, nhi, kap, o, d, N, SIG, dt)
    assert nc == ncell
    scale = expect.max()
    err = np.abs(gam.astype(float) - expect).max() / scale
    print(f"[{precision} kappa={with_kappa}] max |dGamma| / max Gamma = {err:.2e}, "
          f"escaped rel {abs(es / N_exit.sum() - 1):.2e}", flush=True)
    assert err <= grtol
    assert es == pytest.approx(N_exit.sum(), rel=rtol)
    # photons are conserved exactly: the FP32 packet holds its photon rates
    # rounded to float (relative to the brightest bin)
    held = N.sum() if precision == "f64" else (np.float32(N / N.max()).astype(float) * N.max()).sum()
    assert ab + es == pytest.approx(held, rel=1e-12)
    # the oracle's single-ray march through the same field
    orc = O.Oracle(shape=shape, dx_cm=dx, sigma_bins=SIG, alpha_B=W.ALPHA_B_1E4, n_H=nH, kappa=kappa,
                   x_HI0=x, max_level=0, c_ray=np.inf)
    No, go, nco = orc.transmit(o, d, N, dt)
    assert nco == nc
    assert np.abs(gam.astype(float) - go).max() / go.max() <= grtol


@pytest.mark.parametrize("precision,rtol", [("f64", 1e-12), ("f32", 1e-5)])
def test_uniform_medium_transmits_exp_minus_n_sigma_l(ctx, precision, rtol):
    # uniform gas: the photons leaving the box are N exp(-n sigma l) with l
    # the distance from the origin to the box boundary along the ray
    n, dx = 40, 1e21
    shape = (n, n, n)
    nH = np.full(shape, 1e-4, np.float32)
    g = frt.Solve(ctx, sigma_bins=[6.3e-18], precision=precision)
    g.load_grid(nH, dx * n)
    o = np.array([13.3, 7.9, 21.2]) * dx
    d = np.array([0.41, 0.73, -0.55])
    d /= np.linalg.norm(d)
    ab, es, nc, _ = g.debug_cast(o, d, [1e52], 1e13)
    l = min(((n * dx if c > 0 else 0.0) - oc) / c for oc, c in zip(o, d))
    tau = float(np.float32(1e-4)) * 6.3e-18 * l
    assert es == pytest.approx(1e52 * math.exp(-tau), rel=rtol)
    assert ab == pytest.approx(1e52 * -math.expm1(-tau), rel=rtol)


def test_debug_cast_leaves_the_solve_unchanged(ctx):
    p = W.lognormal_c2(n=24, n_src=4, n_steps=2, box_cmpc_h=20.0 * 24 / 128)
    g = frt.solve_from_problem(ctx, p)
    g.step(p.dt_s)
    x0, g0 = g.fields()
    L0 = g.ledger()
    g.debug_cast([p.dx_cm * 3.3, p.dx_cm * 5.1, p.dx_cm * 7.7], [1, 2, 3], [1e50] * 4, p.dt_s)
    x1, g1 = g.fields()
    assert np.array_equal(x0, x1) and np.array_equal(g0, g1) and g.ledger() == L0
    g.step(p.dt_s)
    ref = frt.solve_from_problem(ctx, p)
    ref.step(p.dt_s)
    ref.step(p.dt_s)
    # the next step is the one it would have been (up to the order of the
    # rate field's atomic additions)
    assert np.abs(ref.fields()[0] - g.fields()[0]).max() <= 1e-6
    with pytest.raises(frt.FrtError) as e:
        g.debug_cast([-1.0, 0, 0], [1, 0, 0], [1e50] * 4, p.dt_s)
    assert e.value.code == frt.FRT_EINVAL
