"""Seeded synthetic inputs for the ray-tracing step.

This module builds inputs only: density, sub-grid opacity and neutral-fraction
fields, source positions and photon rates, frequency bins, and the uniforms
that fix each step's random sphere rotation.  It holds none of the transport
or chemistry arithmetic, so the HIP library and the FP64 oracle can both be
fed from it without sharing any of the method's code.

The paper's validation runs use external simulation outputs; the recipes here
stand in for them with the same shapes and statistics (uniform Stromgren box,
white lognormal fields, a k^-2.5 Gaussian random field with sources on its
peaks, many uneven boxes, a Poisson stream of solves).

Units are cgs.  Comoving lengths in cMpc/h become proper lengths at a fixed
redshift z = 9 with h = 0.68 (the paper's cosmology, §1), so a static box
with the quoted mean density n_H = 2e-4 cm^-3 is self-consistent.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ------------------------------------------------------------------ units
C_LIGHT = 2.99792458e10          # cm/s
KPC = 3.0857e21                  # cm
MPC = 3.0857e24                  # cm
MYR = 3.15576e13                 # s
EV = 1.602176634e-12             # erg
K_B = 1.380649e-16               # erg/K
H_LITTLE = 0.68
Z_FIX = 9.0
SIGMA_HI_0 = 6.3e-18             # cm^2 at 13.6 eV
ALPHA_B_1E4 = 2.59e-13           # cm^3/s, case B at 1e4 K
E_HI = 13.6                      # eV
SIGMA_SLOPE = 2.75               # sigma ~ nu^-2.75 (§4.2, heating estimate)


def cmpc_h_to_cm(length_cmpc_h: float) -> float:
    """Comoving cMpc/h -> proper cm at the fixed redshift."""
    return length_cmpc_h * MPC / (H_LITTLE * (1.0 + Z_FIX))


# --------------------------------------------------- rotation uniforms
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014), vectorized on
    uint64 arrays with wrap-around arithmetic."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def rotation_uniforms(seed: int, step: int, n_src: int) -> np.ndarray:
    """Three uniforms in [0,1) per source for one step: counter-based, so any
    (seed, step, source, k) can be regenerated independently.
    u = (splitmix64(splitmix64(seed) ^ (step<<32 | src<<2 | k)) >> 11) * 2^-53."""
    src = np.arange(n_src, dtype=np.uint64)[:, None]
    k = np.arange(3, dtype=np.uint64)[None, :]
    ctr = (np.uint64(step) << np.uint64(32)) | (src << np.uint64(2)) | k
    key = splitmix64(np.uint64(seed))
    bits = splitmix64(ctr ^ key)
    return (bits >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


MERGE_STREAM = 0x6D65726765          # ASCII "merge": the cells' merging-sphere stream


def merge_uniforms(seed: int, step: int, ncell: int) -> np.ndarray:
    """Three uniforms in [0,1) per cell for the randomly rotated merging
    sphere of each cell at the end of `step`: shape (ncell, 3).
    u = (splitmix64(key ^ (step<<34 | cell<<2 | k)) >> 11) * 2^-53 with
    key = splitmix64(splitmix64(seed) ^ 0x6D65726765)."""
    cell = np.arange(ncell, dtype=np.uint64)[:, None]
    k = np.arange(3, dtype=np.uint64)[None, :]
    ctr = (np.uint64(step) << np.uint64(34)) | (cell << np.uint64(2)) | k
    key = splitmix64(splitmix64(np.uint64(seed)) ^ np.uint64(MERGE_STREAM))
    return (splitmix64(ctr ^ key) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rotation_table(seed: int, step0: int, n_steps: int, n_src: int) -> np.ndarray:
    """Uniforms for n_steps consecutive steps: shape (n_steps, n_src, 3)."""
    return np.stack([rotation_uniforms(seed, step0 + s, n_src) for s in range(n_steps)])


# ------------------------------------------------------------ spectrum
def blackbody_bins(n_bins: int, T_bb: float = 5e4, e_lo: float = E_HI, e_hi: float = 4 * E_HI):
    """Log-spaced bins e_lo * (e_hi/e_lo)^(k/n) with photon-number weights of
    a blackbody, and the photon-weighted mean cross-section per bin for
    sigma(E) = sigma_0 (E/13.6 eV)^-2.75.  Returns (weights, sigma_bins)."""
    from scipy.integrate import quad

    if n_bins == 1 and T_bb is None:
        return np.array([1.0]), np.array([SIGMA_HI_0])
    kT = K_B * T_bb / EV
    edges = e_lo * (e_hi / e_lo) ** (np.arange(n_bins + 1) / n_bins)
    number = lambda e: e * e / math.expm1(e / kT)
    sig = lambda e: SIGMA_HI_0 * (e / E_HI) ** (-SIGMA_SLOPE)
    w = np.empty(n_bins)
    s = np.empty(n_bins)
    for i in range(n_bins):
        a, b = edges[i], edges[i + 1]
        n_i = quad(number, a, b, epsabs=0, epsrel=1e-12)[0]
        w[i] = n_i
        s[i] = quad(lambda e: number(e) * sig(e), a, b, epsabs=0, epsrel=1e-12)[0] / n_i
    return w / w.sum(), s


def blackbody_heat(n_bins: int, T_bb: float = 5e4, e_lo: float = E_HI, e_hi: float = 4 * E_HI) -> np.ndarray:
    """Mean energy above 13.6 eV (eV) of the photons HI absorbs in each bin
    of blackbody_bins (absorption-weighted: n(E) sigma(E) over the bin)."""
    from scipy.integrate import quad

    kT = K_B * T_bb / EV
    edges = e_lo * (e_hi / e_lo) ** (np.arange(n_bins + 1) / n_bins)
    absorbed = lambda e: e * e / math.expm1(e / kT) * (e / E_HI) ** (-SIGMA_SLOPE)
    out = np.empty(n_bins)
    for i in range(n_bins):
        a, b = edges[i], edges[i + 1]
        out[i] = (quad(lambda e: absorbed(e) * (e - E_HI), a, b, epsabs=0, epsrel=1e-12)[0]
                  / quad(absorbed, a, b, epsabs=0, epsrel=1e-12)[0])
    return out


# -------------------------------------------------------------- fields
def lognormal_white(rng, shape, mean: float, ln_sigma: float) -> np.ndarray:
    """Mean-preserving white lognormal field: mean * exp(s g - s^2/2)."""
    g = rng.standard_normal(shape)
    return mean * np.exp(ln_sigma * g - 0.5 * ln_sigma ** 2)


def gaussian_field_powerlaw(rng, n: int, slope: float = -2.5) -> np.ndarray:
    """Periodic Gaussian random field on n^3 with P(k) ~ k^slope, P(0)=0,
    normalised to zero mean and unit variance."""
    kx = np.fft.fftfreq(n)
    kz = np.fft.rfftfreq(n)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)          # sqrt(P) = k^(slope/2)
    noise = np.fft.rfftn(rng.standard_normal((n, n, n)))
    g = np.fft.irfftn(noise * amp, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def top_peaks(field: np.ndarray, count: int) -> np.ndarray:
    """Indices (z, y, x) of the `count` highest strict local maxima over the 26
    neighbours (periodic), highest first."""
    from scipy.ndimage import maximum_filter

    footprint = np.ones((3, 3, 3), dtype=bool)
    footprint[1, 1, 1] = False
    neigh = maximum_filter(field, footprint=footprint, mode="wrap")
    peaks = np.argwhere(field > neigh)
    vals = field[tuple(peaks.T)]
    order = np.argsort(-vals, kind="stable")[:count]
    return peaks[order]


def loguniform(rng, lo: float, hi: float, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


# ------------------------------------------------------------- problem
@dataclass
class Problem:
    """One RT solve: everything both the library and the oracle need."""
    name: str
    shape: tuple                      # (nz, ny, nx)
    dx_cm: float
    n_H: np.ndarray                   # float32, (nz, ny, nx)
    x_HI0: np.ndarray                 # float64
    kappa: np.ndarray | None          # float32 1/cm, or None
    src_pos_cm: np.ndarray            # (n_src, 3) float64, (x, y, z)
    ndot_bins: np.ndarray             # (n_src, n_bins) float64 photons/s
    sigma_bins: np.ndarray            # (n_bins,) cm^2
    dt_s: float
    n_steps: int
    c_ray: float = C_LIGHT
    flux_floor: float = 0.0
    max_dist_cm: float = 0.0
    base_level: int = 0
    max_level: int = 12
    n_ray_min: float = 1.0
    alpha_B: float = ALPHA_B_1E4
    coll_ion: float = 0.0
    seed: int = 0
    chem_iterations: int = 0          # 0: backward Euler; K: time-averaged, K marches per step
    opacity_mode: int = 0             # 0: Standard Mode; 1: Generalized Opacity Mode (kappa of the
                                      # ionized phase, x_HI0 = 1 - ionized volume fraction)
    he_chi: float = 0.0
    merge: bool = False               # ray merging at the end of each step (§3.3)
    merge_level: int = 0              # l_merge
    merge_exempt: float = 0.0         # N_ex (exempt packets per cell)
    T: np.ndarray | None = None       # float32 K: the starting temperature when it evolves
    temperature: bool = False         # T evolves (§4.1, Eq. temp_evolution_standard)
    heat_ev: np.ndarray | None = None # (n_bins,) eV above 13.6 eV per photon HI absorbs
    hubble_s: float = 0.0             # H(z) of the adiabatic term, 1/s
    cmb_z: float = -1.0               # CMB redshift of Compton cooling (< 0: none)
    t_reion: float = 2e4              # Generalized Opacity Mode: K of gas the front ionizes
    spectral_index: float = 1.5       # Generalized Opacity Mode: power-law index of its heating
    meta: dict = field(default_factory=dict)

    @property
    def n_src(self) -> int:
        return int(self.src_pos_cm.shape[0])

    @property
    def n_bins(self) -> int:
        return int(self.sigma_bins.shape[0])

    @property
    def ncell(self) -> int:
        return int(np.prod(self.shape))

    def uniforms(self, step: int) -> np.ndarray:
        return rotation_uniforms(self.seed, step, self.n_src)

    def oracle_kwargs(self) -> dict:
        return dict(shape=self.shape, dx_cm=self.dx_cm, sigma_bins=self.sigma_bins,
                    alpha_B=self.alpha_B, n_H=self.n_H, kappa=self.kappa, x_HI0=self.x_HI0,
                    coll_ion=self.coll_ion, base_level=self.base_level, max_level=self.max_level,
                    n_ray_min=self.n_ray_min, flux_floor=self.flux_floor,
                    max_dist_cm=self.max_dist_cm, c_ray=self.c_ray,
                    chem_iterations=self.chem_iterations, opacity_mode=self.opacity_mode,
                    he_chi=self.he_chi, merge=self.merge, merge_level=self.merge_level,
                    merge_exempt=self.merge_exempt, temperature=self.temperature, heat_ev=self.heat_ev,
                    hubble_s=self.hubble_s, cmb_z=self.cmb_z, t_reion=self.t_reion,
                    spectral_index=self.spectral_index,
                    T0=None if self.T is None else np.asarray(self.T, dtype=np.float64))

    def merge_uniforms(self, step: int):
        """The cells' merging-sphere uniforms of `step`, or None without merging."""
        return merge_uniforms(self.seed, step, self.ncell) if self.merge else None

    def footprint_bytes(self) -> int:
        return int(self.ncell * 64)


def _cell_centres(rng, shape, n_src, dx):
    nz, ny, nx = shape
    flat = rng.choice(nz * ny * nx, size=n_src, replace=False)
    z, y, x = np.unravel_index(flat, shape)
    return np.stack([(x + 0.5) * dx, (y + 0.5) * dx, (z + 0.5) * dx], axis=1).astype(np.float64)


# -------------------------------------------------------------- recipes
def stromgren_c1(n: int = 32, n_steps: int = 50, seed: int = 1) -> Problem:
    """Plain method, FP64: one 13.6 eV source of 1e49 photons/s at the corner
    vertex of a uniform pure-H box of 10 kpc, n_H = 2e-3, T = 1e4 K, case B,
    initially neutral; 50 steps of 2 Myr (100 Myr)."""
    L = 10.0 * KPC
    dx = L / n
    shape = (n, n, n)
    return Problem(
        name=f"c1_stromgren_{n}^3", shape=shape, dx_cm=dx,
        n_H=np.full(shape, 2e-3, dtype=np.float32), x_HI0=np.ones(shape),
        kappa=None, src_pos_cm=np.zeros((1, 3)), ndot_bins=np.array([[1e49]]),
        sigma_bins=np.array([SIGMA_HI_0]), dt_s=2.0 * MYR, n_steps=n_steps,
        c_ray=C_LIGHT, flux_floor=0.0, max_dist_cm=0.0, max_level=12, seed=seed,
        meta={"L_cm": L})


def lognormal_c2(n: int = 128, n_src: int = 64, n_steps: int = 100, seed: int = 2,
                 n_bins: int = 4, box_cmpc_h: float = 20.0, mfp_cmpc_h: float = 10.0) -> Problem:
    """Single solve: white lognormal density (ln-sigma 1, mean 2e-4 cm^-3),
    sources at random distinct cell centres with Ndot log-uniform in
    [1e50, 1e53], 4 blackbody (5e4 K) bins over 13.6-54.4 eV, sub-grid mean
    free path lognormal (ln-sigma 0.5) around 10 cMpc/h, 1 Myr steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n)
    dx = cmpc_h_to_cm(box_cmpc_h) / n
    nH = lognormal_white(rng, shape, 2e-4, 1.0).astype(np.float32)
    lam = cmpc_h_to_cm(mfp_cmpc_h) * np.exp(0.5 * rng.standard_normal(shape))
    kappa = (1.0 / lam).astype(np.float32)
    pos = _cell_centres(rng, shape, n_src, dx)
    w, sig = blackbody_bins(n_bins)
    ndot = loguniform(rng, 1e50, 1e53, n_src)[:, None] * w[None, :]
    return Problem(
        name=f"c2_lognormal_{n}^3_{n_src}src", shape=shape, dx_cm=dx, n_H=nH,
        x_HI0=np.ones(shape), kappa=kappa, src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig,
        dt_s=1.0 * MYR, n_steps=n_steps, c_ray=C_LIGHT, flux_floor=1e-3, max_level=12, seed=seed)


def grf_c3(n: int = 256, n_src: int = 2000, throughput: bool = True, n_steps: int | None = None,
           seed: int = 3, box_cmpc_h: float = 100.0, n_bins: int = 4) -> Problem:
    """Single large solve: density exp of a k^-2.5 Gaussian random field
    (ln-sigma 1.5, mean 2e-4), sources on the highest 26-neighbour peaks with
    Ndot proportional to the local density (mean 3.16e51), flux floor 1e-3,
    distance cap 50 cMpc/h, level cap 12.  The throughput form starts highly
    ionized (x_HI = 1e-4) with rays finishing inside each step; the parity
    form starts neutral with packets moving at c."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n, n)
    dx = cmpc_h_to_cm(box_cmpc_h) / n
    g = gaussian_field_powerlaw(rng, n)
    nH = (2e-4 * np.exp(1.5 * g - 1.125)).astype(np.float32)
    peaks = top_peaks(g, n_src)
    z, y, x = peaks.T
    pos = np.stack([(x + 0.5) * dx, (y + 0.5) * dx, (z + 0.5) * dx], axis=1).astype(np.float64)
    dens = nH[z, y, x].astype(np.float64)
    total = 6.3e54 * (n_src / 2000.0)
    w, sig = blackbody_bins(n_bins)
    ndot = (total * dens / dens.sum())[:, None] * w[None, :]
    if throughput:
        x0 = np.full(shape, 1e-4)
        c_ray, steps = np.inf, (3 if n_steps is None else n_steps)
    else:
        x0 = np.ones(shape)
        c_ray, steps = C_LIGHT, (20 if n_steps is None else n_steps)
    return Problem(
        name=f"c3{'b' if throughput else 'a'}_grf_{n}^3_{n_src}src", shape=shape, dx_cm=dx,
        n_H=nH, x_HI0=x0, kappa=None, src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig,
        dt_s=1.0 * MYR, n_steps=steps, c_ray=c_ray, flux_floor=1e-3,
        max_dist_cm=cmpc_h_to_cm(50.0 * box_cmpc_h / 100.0), max_level=12, seed=seed)


C4_DX_CMPC_H = 0.15625


def batch_c4(n_boxes: int = 64, seed: int = 4, n_steps: int = 50, sizes=(32, 48, 64, 96, 128),
             max_src: int = 256, n_bins: int = 3) -> list[Problem]:
    """Many independent uneven boxes: edge from `sizes`, cell 0.15625 cMpc/h,
    white lognormal density with ln-sigma in [0.5, 1.5], 1..256 sources with
    Ndot log-uniform in [1e49, 1e52], 3 blackbody bins, 1 Myr steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = cmpc_h_to_cm(C4_DX_CMPC_H)
    w, sig = blackbody_bins(n_bins)
    out = []
    for b in range(n_boxes):
        n = int(rng.choice(sizes))
        shape = (n, n, n)
        s_ln = rng.uniform(0.5, 1.5)
        nH = lognormal_white(rng, shape, 2e-4, s_ln).astype(np.float32)
        ns = int(rng.integers(1, max_src + 1))
        pos = _cell_centres(rng, shape, ns, dx)
        ndot = loguniform(rng, 1e49, 1e52, ns)[:, None] * w[None, :]
        out.append(Problem(
            name=f"c4_box{b}_{n}^3_{ns}src", shape=shape, dx_cm=dx, n_H=nH, x_HI0=np.ones(shape),
            kappa=None, src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig, dt_s=1.0 * MYR,
            n_steps=n_steps, c_ray=C_LIGHT, flux_floor=1e-3, max_level=12, seed=seed * 1000 + b))
    return out


@dataclass
class Request:
    arrival_s: float
    problem: Problem


def served_c5(n_requests: int = 128, rate_per_s: float = 4.0, seed: int = 5, n_steps: int = 50,
              sizes=(64, 96, 128, 192, 256), max_src: int = 2000, n_bins: int = 4) -> list[Request]:
    """A Poisson stream of solves: edge from `sizes` (cell 0.15625 cMpc/h),
    16..2000 sources (log-uniform integer), the lognormal density/spectrum
    recipe, source efficiency x0.5-x2, sub-grid mean free path median
    log-uniform in 3-30 cMpc/h, 1 Myr steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = cmpc_h_to_cm(C4_DX_CMPC_H)
    w, sig = blackbody_bins(n_bins)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(rng.choice(sizes))
        shape = (n, n, n)
        nH = lognormal_white(rng, shape, 2e-4, 1.0).astype(np.float32)
        mfp = cmpc_h_to_cm(loguniform(rng, 3.0, 30.0))
        kappa = (1.0 / (mfp * np.exp(0.5 * rng.standard_normal(shape)))).astype(np.float32)
        ns = int(np.floor(loguniform(rng, 16, max_src + 1)))
        ns = max(16, min(max_src, ns, n ** 3))
        pos = _cell_centres(rng, shape, ns, dx)
        eff = loguniform(rng, 0.5, 2.0)
        ndot = (loguniform(rng, 1e50, 1e53, ns) * eff)[:, None] * w[None, :]
        p = Problem(name=f"c5_req{r}_{n}^3_{ns}src", shape=shape, dx_cm=dx, n_H=nH,
                    x_HI0=np.ones(shape), kappa=kappa, src_pos_cm=pos, ndot_bins=ndot, sigma_bins=sig,
                    dt_s=1.0 * MYR, n_steps=n_steps, c_ray=C_LIGHT, flux_floor=1e-3, max_level=12,
                    seed=seed * 100000 + r)
        reqs.append(Request(arrival_s=t, problem=p))
    return reqs
