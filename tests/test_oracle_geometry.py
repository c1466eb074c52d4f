"""Pins of the oracle's geometry: HEALPix directions (§3.1 Eq. Nray, §3.2
Eq. lhpx), the random sphere rotation (§3.1) and its uniforms, and the split
radius (§3.2 Eq. r_split).  Every expected value comes from a closed form,
a published value or an independent construction, never from the oracle."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04521_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_pixel_count_and_unit_norm(level):
    # Eq. Nray: 12 * 4^l directions, all unit vectors, all distinct
    v = O.healpix_centers(level)
    assert v.shape == (12 * 4 ** level, 3)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-14)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2) + np.eye(len(v))
    assert d.min() > 1e-3


def test_golden_centres():
    for lvl, pix, z, phi_pi in _golden_rows("healpix_nested_centres.txt"):
        v = O.healpix_center(int(lvl), int(pix))
        phi = math.atan2(v[1], v[0]) % (2 * math.pi)
        assert v[2] == pytest.approx(float(z), abs=1e-14)
        assert phi / math.pi == pytest.approx(float(phi_pi), abs=1e-14)


@pytest.mark.parametrize("level", [1, 2, 3])
def test_iso_latitude_rings(level):
    # Gorski et al. 2005: 4 Nside - 1 rings; polar ring i has 4i pixels at
    # z = 1 - i^2/(3 Nside^2); equatorial rings have 4 Nside pixels at
    # z = 4/3 - 2i/(3 Nside); pixels in a ring are equally spaced in phi.
    ns = 2 ** level
    v = O.healpix_centers(level)
    zs = np.round(v[:, 2], 12)
    rings = {}
    for i in range(1, 4 * ns):
        if i < ns:
            z, cnt = 1 - i * i / (3 * ns * ns), 4 * i
        elif i <= 3 * ns:
            z, cnt = 4 / 3 - 2 * i / (3 * ns), 4 * ns
        else:
            j = 4 * ns - i
            z, cnt = -(1 - j * j / (3 * ns * ns)), 4 * j
        rings[round(z, 12)] = cnt
    vals, counts = np.unique(zs, return_counts=True)
    assert len(vals) == 4 * ns - 1
    for z, c in zip(vals, counts):
        assert rings[round(z, 12)] == c
        sel = v[np.isclose(v[:, 2], z, atol=1e-12)]
        phi = np.sort(np.arctan2(sel[:, 1], sel[:, 0]) % (2 * np.pi))
        gaps = np.diff(np.concatenate([phi, [phi[0] + 2 * np.pi]]))
        assert np.allclose(gaps, 2 * np.pi / c, atol=1e-12)


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_round_trip_and_children_nest(level):
    # Eq. lhpx: the children 4p+i of (l, p) sub-sample the parent pixel.
    for p in range(12 * 4 ** level):
        assert O.healpix_pixel(level, O.healpix_center(level, p)) == p
        for i in range(4):
            c = O.healpix_center(level + 1, 4 * p + i)
            assert O.healpix_pixel(level, c) == p


def test_equal_area_monte_carlo():
    # HEALPix pixels have equal area: uniform points fall evenly (chi-square).
    rng = np.random.Generator(np.random.PCG64(11))
    n = 60000
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    level = 1
    counts = np.bincount([O.healpix_pixel(level, x) for x in v], minlength=48)
    assert counts.min() > 0
    exp = n / 48
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 90  # 47 d.o.f.; p ~ 1e-4 cut


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_directions_sum_to_zero(level):
    assert np.abs(O.healpix_centers(level).sum(axis=0)).max() < 1e-12


# ---------------------------------------------------------------- rotation
def _quat_sandwich(u, v):
    """Rotate v by q v q* with explicit Hamilton products (independent of the
    oracle's matrix form)."""
    s1, s2 = math.sqrt(1 - u[0]), math.sqrt(u[0])
    q = np.array([s2 * math.cos(2 * math.pi * u[2]), s1 * math.sin(2 * math.pi * u[1]),
                  s1 * math.cos(2 * math.pi * u[1]), s2 * math.sin(2 * math.pi * u[2])])

    def ham(a, b):
        return np.array([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                         a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                         a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                         a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]])

    qc = q * np.array([1, -1, -1, -1])
    return ham(ham(q, np.concatenate([[0.0], v])), qc)[1:]


def test_rotation_is_proper_and_matches_quaternion():
    u = W.rotation_table(7, 0, 20, 10).reshape(-1, 3)
    rng = np.random.Generator(np.random.PCG64(1))
    for ui in u:
        R = O.rotation(ui)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
        v = rng.standard_normal(3)
        assert np.allclose(R @ v, _quat_sandwich(ui, v), atol=1e-13)


def test_rotation_is_haar_uniform():
    # Haar measure on SO(3): rotation angle density (1 - cos t)/pi, so
    # E[cos t] = -1/2 and E[trace R] = 0; images of a fixed axis are uniform.
    u = W.rotation_table(3, 0, 1, 20000)[0]
    Rs = np.stack([O.rotation(x) for x in u])
    tr = np.trace(Rs, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.05
    cos_t = (tr - 1) / 2
    assert abs(cos_t.mean() + 0.5) < 0.03
    z = Rs[:, :, 2]
    assert np.abs(z.mean(axis=0)).max() < 0.03
    assert np.allclose((z ** 2).mean(axis=0), 1 / 3, atol=0.02)


def test_splitmix64_published_value():
    for ctr, val in _golden_rows("splitmix64.txt"):
        assert int(W.splitmix64(np.uint64(int(ctr)))) == int(val, 16)


def test_rotation_uniforms_range_and_counter():
    a = W.rotation_uniforms(5, 3, 100)
    assert a.shape == (100, 3) and a.min() >= 0 and a.max() < 1
    b = W.rotation_table(5, 0, 5, 100)[3]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, W.rotation_uniforms(6, 3, 100))


# ------------------------------------------------------------ split radius
@pytest.mark.parametrize("level", [0, 1, 4, 9])
@pytest.mark.parametrize("nmin", [1.0, 2.0, 4.0])
def test_split_radius_is_footprint_equal_face(level, nmin):
    # Eq. r_split: a level-l ray covers 4 pi/(12 4^l) sr; its footprint
    # Omega r^2 equals the cell face / N_min exactly at r_split.
    dx = 3.7e21
    r = O.split_radius(dx, level, nmin)
    omega = 4 * math.pi / (12 * 4 ** level)
    assert omega * r * r == pytest.approx(dx * dx / nmin, rel=1e-14)
