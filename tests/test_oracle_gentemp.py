"""Pins of the oracle's temperature in the Generalized Opacity Mode (§4.2,
after Eq. dxidt: gas that the moving screen ionizes enters at T_reion and
then follows Eq. temp_evolution_standard, with the photo-heating of Eq.
analytical_heating_HI and n_HI from photo-ionization equilibrium), each
against something other than its own formulas:

* the heating per recombination over E_HI q(alpha) is the mean energy above
  1 Ryd of the photons HI absorbs from a power law nu^-alpha cut off at 4 Ryd
  (sigma ~ nu^-2.75), by numerical quadrature of that definition;
* the case-A recombination coefficient (Hui & Gnedin 1997 fit) lies within
  3% of an independent fit (Verner & Ferland 1996) from 1e2 to 1e6 K and of
  the textbook 4.18e-13 cm^3/s at 1e4 K, and above case B;
* at a density where the radiative terms take far longer than the run, every
  cell the front reached holds the volume-weighted mean of T_reion (the gas
  ionized in each step) and the older ionized gas cooled by e^(-2 H t), and
  neutral cells keep their temperature;
* highly ionized gas settles at one temperature from above and from below,
  whatever its n_H and Gamma at a fixed neutral fraction (heating and cooling
  both scale as n_e^2), higher for a harder spectrum;
* without photons the ionized gas only cools adiabatically: T0 e^(-2 H t).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W

EV = 1.602176634e-12
RYD_EV = 13.605693122994


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.5, 3.0])
def test_heating_per_recombination_is_the_mean_excess_energy(alpha):
    beta = 2.75
    # photons per unit frequency ~ nu^(-alpha-1); absorbed ~ that times sigma
    num = quad(lambda x: x ** (-alpha - 1 - beta) * (x - 1.0), 1.0, 4.0, epsabs=0, epsrel=1e-13)[0]
    den = quad(lambda x: x ** (-alpha - 1 - beta), 1.0, 4.0, epsabs=0, epsrel=1e-13)[0]
    assert O.reion_heat_per_recombination(alpha) / (RYD_EV * EV) == pytest.approx(num / den, rel=1e-10)


def test_case_a_recombination_fit():
    for T in np.logspace(2, 6, 17):
        s0, s1 = math.sqrt(T / 3.148), math.sqrt(T / 7.036e5)
        vf = 7.982e-11 / (s0 * (1 + s0) ** (1 - 0.748) * (1 + s1) ** (1 + 0.748))
        r = O.rates(T)
        assert r["alpha_A"] == pytest.approx(vf, rel=0.03), T
        assert r["alpha_A"] > r["alpha_B"], T
    assert O.rates(1e4)["alpha_A"] == pytest.approx(4.18e-13, rel=0.03)


def test_front_cells_mix_t_reion_with_the_older_ionized_gas():
    # n_H = 1e-12: heating and cooling per particle take ~1e24 s; the front
    # (photon counting: R ~ 2 cells after the first step) crosses cells over
    # several steps
    n, nh, H, T0, Tre = 12, 1e-12, 2e-15, 300.0, 2.3e4
    dx = 2.1e21
    nH = np.full((n, n, n), nh, dtype=np.float32)
    o = O.Oracle((n, n, n), dx, [6.3e-18], 2.59e-13, nH, kappa=np.zeros((n, n, n), np.float32),
                 x_HI0=np.ones((n, n, n)), c_ray=np.inf, opacity_mode=1, temperature=True, hubble_s=H,
                 t_reion=Tre, spectral_index=1.5, T0=T0)
    o.set_sources(np.array([[6.0, 6.0, 6.0]]) * dx, np.array([[1e40]]))
    dt = W.MYR
    xi_prev, T_prev = np.zeros((n, n, n)), np.full((n, n, n), T0)
    partial = 0
    for s in range(4):
        o.step(dt, W.rotation_uniforms(5, s, 1))
        xi = 1.0 - o.fields()[0]
        T = o.temperature()
        cool = math.exp(-2 * H * dt)
        grown = xi > xi_prev
        want = np.where(grown, (xi_prev * T_prev * cool + (xi - xi_prev) * Tre) / np.where(grown, xi, 1.0),
                        np.where(xi_prev > 0, T_prev * cool, T_prev))
        np.testing.assert_allclose(T, want, rtol=1e-9, atol=0)
        assert np.all(T[xi == 0] == T0)                                   # neutral cells untouched
        partial += int(np.count_nonzero(grown & (xi_prev > 0)))
        xi_prev, T_prev = xi, T
    assert partial > 0 and np.count_nonzero(xi == 0) > 0 and np.count_nonzero(xi == 1) > 0


@pytest.mark.parametrize("alpha", [0.5, 1.5, 3.0])
def test_equilibrium_temperature_of_highly_ionized_gas(alpha):
    y = 1e-7                                  # n_HI / n_H at 2e4 K
    ab = O.rates(2e4)["alpha_B"]
    Ts = []
    for nh in (1e-3, 1e-1):
        G = ab * nh / y
        for T0 in (1e3, 1e5):
            T = T0
            for _ in range(5):                # 5 x 1e17 s (1e-3 / n_H): many cooling times
                T = O.ionized_temperature(T, nh, G, 1e17 * 1e-3 / nh, spectral_index=alpha)
            Ts.append(T)
    assert max(Ts) / min(Ts) - 1 <= 1e-5, Ts
    assert 1e4 < Ts[0] < 1e5
    if alpha > 0.5:
        G = ab * 1e-3 / y
        T = 1e4
        for _ in range(5):
            T = O.ionized_temperature(T, 1e-3, G, 1e17, spectral_index=alpha - 1.0)
        assert T > Ts[0]                      # a harder spectrum heats more


def test_without_photons_ionized_gas_cools_adiabatically():
    H, dt = 3e-17, 5 * W.MYR
    for T0 in (50.0, 2e4, 3e5):
        assert O.ionized_temperature(T0, 1e-3, 0.0, dt, hubble_s=H) == pytest.approx(T0 * math.exp(-2 * H * dt),
                                                                                      rel=1e-12)
