"""Whole-step pins of the oracle: photon conservation, the analytic
Stromgren I-front (§5.1 Eqs. r_of_t, rS, trec) approached as the step
shrinks, the paper's printed worked numbers, checkpoint/resume and
independence of the thread count."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_examples():
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_examples.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v, _ = line.split()
            out[k] = float(v)
    return out


def _run(p, steps=None, threads=None):
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    for s in range(p.n_steps if steps is None else steps):
        o.step(p.dt_s, p.uniforms(s), threads=threads)
    return o


def _closure(L):
    out = L["absorbed_HI"] + L["absorbed_sub"] + L["escaped"] + L["dropped"] + L["in_flight"]
    return abs(L["emitted"] - out) / L["emitted"]


@pytest.mark.parametrize("make", [
    lambda: W.stromgren_c1(n=16, n_steps=6),
    lambda: W.lognormal_c2(n=24, n_src=6, n_steps=6),
    lambda: W.grf_c3(n=32, n_src=12, throughput=True, n_steps=2, box_cmpc_h=12.5),
    lambda: W.grf_c3(n=32, n_src=12, throughput=False, n_steps=4, box_cmpc_h=12.5),
])
def test_photon_ledger_closes(make):
    p = make()
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    for s in range(p.n_steps):
        o.step(p.dt_s, p.uniforms(s))
        assert _closure(o.ledger()) <= 1e-10
    L = o.ledger()
    assert L["crossings"] > 0 and L["emitted"] > 0


def test_paper_stromgren_radius_example():
    # §5.1 footnote: r_S = 5.4 pkpc for n_H = 1e-3, Ndot = 5e48, alpha_B(1e4 K)
    ex = _paper_examples()
    rS = (3 * ex["stromgren_ndot"] / (4 * math.pi * ex["stromgren_alphaB"] * ex["stromgren_nH"] ** 2)) ** (1 / 3)
    assert rS / W.KPC == pytest.approx(ex["stromgren_rS_kpc"], abs=0.05)


def test_paper_time_step_example():
    # §7.2: dt = dx/c = 0.6 Myr for 1 cMpc/h cells at z = 7 with h = 0.68
    ex = _paper_examples()
    dx = ex["step_cell_cmpc_h"] * W.MPC / (W.H_LITTLE * (1 + ex["step_z"]))
    assert dx / W.C_LIGHT / W.MYR == pytest.approx(ex["step_dt_myr"], abs=0.01)


def _stromgren_ratio(dt_myr, n=32, t_stop=100.0):
    """I-front radius from the ionized volume (sharp-front estimate, §5.2)
    over the analytic r(t) for the C1 physics with the source at the box
    centre (the paper's Test 1 geometry)."""
    p = W.stromgren_c1(n=n)
    L = p.meta["L_cm"]
    p.src_pos_cm = np.array([[L / 2] * 3])
    dt = dt_myr * W.MYR
    steps = int(round(t_stop / dt_myr))
    nH = float(np.float32(2e-3))
    a, Nd = p.alpha_B, 1e49
    rS = (3 * Nd / (4 * math.pi * a * nH ** 2)) ** (1 / 3)
    trec = 1 / (a * nH)
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    out = {}
    for s in range(steps):
        o.step(dt, p.uniforms(s))
        t = (s + 1) * dt
        if t >= 0.5 * trec:
            x, _ = o.fields()
            r = (3 * (1 - x).sum() * p.dx_cm ** 3 / (4 * math.pi)) ** (1 / 3)
            out[t / trec] = r / (rS * (1 - math.exp(-t / trec)) ** (1 / 3))
    return out


@pytest.mark.slow
def test_stromgren_front_converges_to_analytic():
    # Eqs. r_of_t/rS/trec: with a short step the front follows the analytic
    # solution within 3% from t_rec/2 on; the error is first order in dt
    # (backward Euler), so halving dt roughly halves it.
    fine = _stromgren_ratio(0.1)
    assert max(abs(v - 1) for v in fine.values()) < 0.03
    e4 = _stromgren_ratio(0.4)
    e2 = _stromgren_ratio(0.2)
    k = min(e4)   # first sample at t >= t_rec/2
    err4 = abs(e4[k] - 1)
    err2 = abs(e2[min(e2)] - 1)
    assert 1.5 < err4 / err2 < 2.6


def test_checkpoint_resume_is_bitwise():
    p = W.lognormal_c2(n=20, n_src=5, n_steps=6)
    a = _run(p)
    b = _run(p, steps=3)
    blob = b.save()
    c = O.Oracle(**p.oracle_kwargs())
    c.set_sources(p.src_pos_cm, p.ndot_bins)
    c.load(blob)
    for s in range(3, 6):
        c.step(p.dt_s, p.uniforms(s))
    xa, ga = a.fields()
    xc, gc = c.fields()
    assert np.array_equal(xa, xc) and np.array_equal(ga, gc)
    assert a.ledger() == c.ledger()


def test_result_independent_of_thread_count():
    p = W.lognormal_c2(n=20, n_src=9, n_steps=3)
    a = _run(p, threads=1)
    b = _run(p, threads=5)
    assert np.array_equal(a.fields()[0], b.fields()[0])
    assert a.ledger() == b.ledger()


def _c1_front(chem_iterations, n_steps=50):
    """C1 as configured (source on the corner vertex, 2 Myr steps to 100
    Myr): per step t >= t_rec/2 the raw ratio r(t)/r_analytic(t) (Eqs. r_of_t,
    rS, trec; octant volume times 8) and the ratio of the ionized volume to
    the injection-corrected analytic volume, which integrates
    dV/dt = Ndot_in / n_H - alpha n_H V exactly over each step with the
    photons that entered the box in that step (emitted minus escaped): the
    12 level-0 packets of a vertex source put k/12 of the photons into the
    octant, not 1/8, so only this form isolates the chemistry."""
    p = W.stromgren_c1()
    p.chem_iterations = chem_iterations
    nH = float(np.float32(2e-3))
    a, Nd = p.alpha_B, 1e49
    rS = (3 * Nd / (4 * math.pi * a * nH ** 2)) ** (1 / 3)
    trec = 1 / (a * nH)
    o = O.Oracle(**p.oracle_kwargs())
    o.set_sources(p.src_pos_cm, p.ndot_bins)
    V = 0.0
    raw, cor = [], []
    for s in range(n_steps):
        L0 = o.ledger()
        o.step(p.dt_s, p.uniforms(s))
        L1 = o.ledger()
        injected = (L1["emitted"] - L0["emitted"]) - (L1["escaped"] - L0["escaped"])
        Veq = injected / p.dt_s / (a * nH * nH)
        V = Veq + (V - Veq) * math.exp(-a * nH * p.dt_s)
        t = (s + 1) * p.dt_s
        if t >= 0.5 * trec:
            x, _ = o.fields()
            Vion = (1 - x).sum() * p.dx_cm ** 3
            r = (3 * 8 * Vion / (4 * math.pi)) ** (1 / 3)
            raw.append(r / (rS * (1 - math.exp(-t / trec)) ** (1 / 3)) - 1)
            cor.append((Vion / V) ** (1 / 3) - 1)
    return np.array(raw), np.array(cor)


def test_c1_time_averaged_chemistry_meets_the_stromgren_gate():
    # The paper's own update (§4.1, Eqs. xi_of_t-gamma_updated_standard,
    # iterated; exact without recombinations) at C1's 2 Myr step: the front
    # follows the injection-corrected analytic solution within 3% from
    # t_rec/2 on (measured 1.5%).  The raw ratio is set by the vertex
    # sampling of the level-0 packets (measured 17%), reported, not gated.
    raw, cor = _c1_front(20)
    print(f"C1 K=20: worst raw {np.abs(raw).max():.3f}, worst corrected {np.abs(cor).max():.4f}")
    assert np.abs(cor).max() <= 0.03
    assert np.abs(raw).max() <= 0.25


def test_c1_backward_euler_is_not_photon_conserving_at_2_myr():
    # Backward Euler with the start-of-step opacity (the default chemistry):
    # a cell absorbs Gamma x n_H V dt photons in a step but, without
    # recombinations, ionizes x Gamma dt / (1 + Gamma dt) n_H V atoms, a
    # fraction 1 / (1 + Gamma dt) of what it absorbed; cells at the front of
    # C1 have Gamma dt >> 1 at 2 Myr, so the ionized volume falls far behind
    # the photons that entered (measured 37% in radius).  The time-averaged
    # update above is the one that meets the C1 gate.
    raw, cor = _c1_front(0)
    print(f"C1 backward Euler: worst raw {np.abs(raw).max():.3f}, worst corrected {np.abs(cor).max():.3f}")
    assert np.abs(cor).max() > 0.25 and np.all(cor < 0)
