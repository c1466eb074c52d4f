"""Pins of the oracle's time-averaged chemistry (§4.1, Eqs. xi_of_t, xeq, ti,
avg_xi, gamma_updated_standard), each against something other than the
formula itself:

* at fixed n_e the update is the exact solution of the linear rate equation
  (Eq. ion_balance_eqn divided by n_H), and <x> its time average: both are
  compared with a stiff ODE solver that integrates x and its integral;
* iterating n_e = n_H (1 - <x>) over a long step reaches photo-ionization
  equilibrium Gamma x = alpha n_H (1 - x)^2;
* the whole iterated step with alpha = C = 0 ionizes exactly as many atoms
  as its last march absorbed photons (the property of the scheme that §4.1
  cites), once the iteration has converged; a single backward-Euler or
  un-iterated step is far from it on the same grid.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W


def _ode(x0, g, ne, a, c, dt):
    def f(t, y):
        x = y[0]
        return [a * ne * (1.0 - x) - (g + c * ne) * x, x]
    sol = solve_ivp(f, (0.0, dt), [x0, 0.0], method="Radau", rtol=1e-11, atol=[1e-14, 1e-14 * dt])
    return sol.y[1, -1] / dt, sol.y[0, -1]


def test_avg_update_is_the_fixed_ne_ode_solution():
    rng = np.random.Generator(np.random.PCG64(21))
    for _ in range(60):
        x0 = rng.uniform(0, 1) ** 2
        g = 10 ** rng.uniform(-16, -11)
        nH = 10 ** rng.uniform(-4, -2)
        ne = nH * rng.uniform(0, 1)
        a = 2.59e-13 * rng.uniform(0.5, 2)
        c = rng.choice([0.0, 1e-15])
        dt = 10 ** rng.uniform(11, 15)
        xa, xe = O.chemistry_avg(x0, g, ne, a, c, dt)
        ra, re = _ode(x0, g, ne, a, c, dt)
        assert 0.0 <= xe <= 1.0 and 0.0 <= xa <= 1.0
        assert xe == pytest.approx(re, rel=1e-7, abs=1e-11)
        assert xa == pytest.approx(ra, rel=1e-7, abs=1e-11)


def test_avg_update_without_rates_keeps_x():
    assert O.chemistry_avg(0.3, 0.0, 0.0, 2.59e-13, 0.0, 1e14) == (0.3, 0.3)
    # a vanishing step: <x> and x(dt) both tend to x0
    xa, xe = O.chemistry_avg(0.7, 1e-12, 1e-3, 2.59e-13, 0.0, 1e-3)
    assert xa == pytest.approx(0.7, rel=1e-12) and xe == pytest.approx(0.7, rel=1e-12)


def test_iterated_electron_density_reaches_equilibrium():
    # long step: <x> -> x_eq(n_e); n_e = n_H (1 - <x>) then converges to the
    # photo-ionization equilibrium Gamma x = alpha n_H (1 - x)^2
    for g, nH in [(1e-12, 2e-4), (1e-14, 1e-2), (3e-13, 1e-3)]:
        a, x, dt = 2.59e-13, 1.0, 1e22
        for _ in range(400):
            xa, _ = O.chemistry_avg(1.0, g, nH * (1.0 - x), a, 0.0, dt)
            x = xa
        assert g * x == pytest.approx(a * nH * (1 - x) ** 2, rel=1e-6)


def _iterated_step(K, alpha=0.0, n=12):
    rng = np.random.Generator(np.random.PCG64(11))
    nH = (2e-4 * np.exp(0.5 * rng.standard_normal((n, n, n)) - 0.125)).astype(np.float32)
    dx = W.cmpc_h_to_cm(20.0) / 1280
    pos = np.array([[3.5, 4.5, 6.5], [8.5, 7.5, 2.5]]) * dx
    nd = np.array([[3e51, 1e51], [1e51, 5e50]])
    sig = np.array([6.3e-18, 2e-18])
    o = O.Oracle((n, n, n), dx, sig, alpha, nH, c_ray=np.inf, chem_iterations=K)
    o.set_sources(pos, nd)
    o.step(3.15e13, W.rotation_uniforms(1, 0, 2))
    x, _ = o.fields()
    L = o.ledger()
    ionized = float(np.sum(nH.astype(np.float64).reshape(-1) * dx ** 3 * (1.0 - x.reshape(-1))))
    return ionized, L


def test_converged_iteration_conserves_photons():
    err = {}
    for K in (1, 20, 40, 80):
        ion, L = _iterated_step(K)
        err[K] = abs(ion - L["absorbed_HI"]) / L["absorbed_HI"]
        closure = L["emitted"] - L["absorbed_HI"] - L["absorbed_sub"] - L["escaped"] - L["dropped"] - L["in_flight"]
        assert abs(closure) <= 1e-12 * L["emitted"]
    ion_be, L_be = _iterated_step(0)
    assert 0.0 < ion_be < 1.2e65                      # a thick, partly ionized box
    assert abs(ion_be - L_be["absorbed_HI"]) / L_be["absorbed_HI"] > 0.1
    assert err[1] > 0.1
    assert err[1] > err[20] > err[40] > err[80]      # geometric convergence
    assert err[80] < 1e-10


def test_recombination_lowers_the_ionized_count():
    ion0, _ = _iterated_step(8, alpha=0.0)
    ion1, L1 = _iterated_step(8, alpha=2.59e-13)
    assert ion1 < ion0
    assert ion1 <= L1["absorbed_HI"] * (1 + 1e-9)
