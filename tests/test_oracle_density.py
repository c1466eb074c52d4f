"""Pins of the oracle's density update between steps (orc_set_density: the
density a simulation hands to the next step, with the compression term of
Eq. temp_evolution_standard), each against something other than its own
formula:

* along a path of density fields, T follows an ODE solver's integration of
  dT/dt = (2 T / 3 Delta) dDelta/dt with Delta = n_H / <n_H> (the term as
  the paper writes it), whatever the path;
* a change of the mean density alone (the expansion that the Hubble term
  covers) leaves T as it was;
* a step after the update equals the same step of a grid loaded with the new
  density from the start (Standard Mode and the Generalized Opacity Mode).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W

KPC = 3.0857e21


def _lognormal(rng, n, mean, sigma):
    return W.lognormal_white(rng, (n, n, n), mean, sigma).astype(np.float32)


def test_compression_term_follows_an_ode_solver_along_a_path():
    n, k = 5, 6
    rng = np.random.Generator(np.random.PCG64(3))
    path = [_lognormal(rng, n, 10 ** rng.uniform(-4, -2), 1.0) for _ in range(k)]
    T0 = 10 ** rng.uniform(2, 4.5, size=(n, n, n))
    o = O.Oracle((n, n, n), 1e21, [6.3e-18], 2.59e-13, path[0], temperature=True, heat_ev=[1.0], T0=T0)
    for p in path[1:]:
        o.set_density(p)
    nd = [p.astype(np.float64).reshape(-1) for p in path]

    def rhs(t, T):
        j = min(int(t), k - 2)
        a, b = nd[j], nd[j + 1]
        f = t - j
        nn = a + f * (b - a)
        m, dm = nn.mean(), (b - a).mean()
        D = nn / m
        dD = ((b - a) * m - nn * dm) / m ** 2
        return 2.0 * T / (3.0 * D) * dD

    sol = solve_ivp(rhs, (0.0, k - 1.0), T0.reshape(-1), method="DOP853", rtol=1e-11, atol=1e-9,
                    t_eval=[k - 1.0], max_step=0.05)
    np.testing.assert_allclose(o.temperature().reshape(-1), sol.y[:, -1], rtol=1e-8)


def test_a_change_of_the_mean_alone_keeps_t():
    n = 6
    rng = np.random.Generator(np.random.PCG64(5))
    nH = _lognormal(rng, n, 1e-3, 1.0)
    T0 = 10 ** rng.uniform(2, 4.5, size=(n, n, n))
    o = O.Oracle((n, n, n), 1e21, [6.3e-18], 2.59e-13, nH, temperature=True, heat_ev=[1.0], T0=T0)
    o.set_density(nH * np.float32(8.0))
    np.testing.assert_allclose(o.temperature(), T0, rtol=1e-15, atol=0)
    with pytest.raises(ValueError):
        o.set_density(np.zeros_like(nH))


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("temperature", [False, True])
def test_step_after_the_update_equals_a_grid_loaded_with_it(mode, temperature):
    n = 12
    rng = np.random.Generator(np.random.PCG64(7 + mode))
    n1, n2 = _lognormal(rng, n, 1e-3, 1.0), _lognormal(rng, n, 2e-3, 1.0)
    x0 = rng.uniform(0.0, 1.0, size=(n, n, n))
    kap = (W.lognormal_white(rng, (n, n, n), 1.0, 0.5) / (5 * 13.2 * KPC / n)).astype(np.float32) if mode else None
    T0 = 10 ** rng.uniform(2, 4.5, size=(n, n, n))
    dx = 13.2 * KPC / n
    kw = dict(kappa=kap, x_HI0=x0, c_ray=np.inf, opacity_mode=mode, temperature=temperature, heat_ev=[2.0],
              hubble_s=1e-17, t_reion=2e4)
    a = O.Oracle((n, n, n), dx, [6.3e-18], 2.59e-13, n1, T0=T0, **kw)
    a.set_density(n2)
    Ta = a.temperature()
    if temperature:
        assert not np.allclose(Ta, T0)
    b = O.Oracle((n, n, n), dx, [6.3e-18], 2.59e-13, n2, T0=Ta, **kw)
    src = np.array([[n / 2, n / 2, n / 2]]) * dx
    for o in (a, b):
        o.set_sources(src, np.array([[3e51]]))
        for s in range(2):
            o.step(W.MYR, W.rotation_uniforms(11, s, 1))
    assert np.array_equal(a.fields()[0], b.fields()[0])
    assert np.array_equal(a.temperature(), b.temperature())
    assert a.ledger()["absorbed_HI"] == b.ledger()["absorbed_HI"]
