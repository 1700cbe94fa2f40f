"""Pins of the oracle's spherical-harmonic analysis of a RING map (the
angular power spectrum of Sec. III, Fig. 4):
a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(n_p)), C_l = sum_m |a_lm|^2/(2l+1).
Fixed against an independent library (scipy's spherical harmonics), the
addition theorem, 40-digit values of the associated Legendre functions at
high l and m (where sin^m theta leaves the double range), the exact
quarter-turn and north-south symmetries of the HEALPix grid, constant and
band-limited maps, and the definition of C_l."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle


def scipy_ylm(l, m, theta, phi):
    if hasattr(sp, "sph_harm_y"):
        return sp.sph_harm_y(l, m, theta, phi)
    return sp.sph_harm(m, l, phi, theta)


@pytest.mark.parametrize("z", [-0.97, -0.4, 0.0, 0.31, 0.88])
def test_lambda_against_scipy(z):
    s = math.sqrt(1 - z * z)
    for m in (0, 1, 2, 7, 19, 40):
        lam = oracle.lambda_lm(60, m, z, s)
        ref = np.array([scipy_ylm(l, m, math.acos(z), 0.0).real for l in range(m, 61)])
        assert np.max(np.abs(lam - ref)) <= 1e-13, (z, m)


@pytest.mark.parametrize("lmax", [64, 700, 3000])
def test_addition_theorem(lmax):
    """sum_{m=-l}^{l} |Y_lm|^2 = (2l+1)/(4 pi) at any direction, for every l."""
    rng = np.random.default_rng(lmax)
    for z in list(rng.uniform(-1, 1, 3)) + [0.9999, -0.99999]:
        s = math.sqrt(1 - z * z)
        tot = np.zeros(lmax + 1)
        for m in range(lmax + 1):
            lam = oracle.lambda_lm(lmax, m, z, s)
            tot[m:] += (1.0 if m == 0 else 2.0) * lam * lam
        ref = (2 * np.arange(lmax + 1) + 1) / (4 * np.pi)
        assert np.max(np.abs(tot / ref - 1)) <= 1e-11, (lmax, z)


@pytest.mark.parametrize("l,m,theta", [(1500, 1000, 0.9), (3000, 2500, 1.2), (4000, 1500, 0.45),
                                       (3000, 1200, 0.4),
                                       (4000, 100, 0.05)])
def test_lambda_high_degree_against_40_digits(l, m, theta):
    """lambda_lm = (-1)^m sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta)
    evaluated with 40 digits; the start sin^m theta is far below 1e-308 in
    some of these cases."""
    mpmath.mp.dps = 40
    z = math.cos(theta)
    s = math.sin(theta)
    val = oracle.lambda_lm(l, m, z, s)[-1]
    zz = mpmath.mpf(z)
    pl = mpmath.legenp(l, m, zz, type=2, maxprec=100000)   # includes (-1)^m, |z| < 1
    norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) /
                       mpmath.factorial(l + m))
    ref = float(norm * pl)
    assert abs(val - ref) <= 1e-10 * max(abs(ref), 1e-30) + 1e-300, (val, ref)


def ring_perm(nside, op):
    """Pixel permutation of an exact grid symmetry: 'quarter' (phi + pi/2) or
    'mirror' (z -> -z)."""
    npix = 12 * nside * nside
    ring, pos = oracle.ring_of_pixel(nside, np.arange(npix))
    first = {}
    for p in range(npix):
        first.setdefault(int(ring[p]), p)
    n = 4 * nside
    length = lambda i: 4 * min(i, nside, n - i)
    out = np.empty(npix, dtype=np.int64)
    for p in range(npix):
        i, j = int(ring[p]), int(pos[p])
        if op == "quarter":
            L = length(i)
            out[p] = first[i] + (j + L // 4) % L
        else:
            out[p] = first[n - i] + j
    return out


def test_quarter_turn_and_mirror_symmetries():
    nside, lmax = 8, 20
    rng = np.random.default_rng(3)
    m0 = rng.standard_normal(12 * nside * nside)
    a = oracle.map2alm(nside, lmax, m0)
    q = ring_perm(nside, "quarter")
    rot = np.empty_like(m0)
    rot[q] = m0                      # the value at p moves to the pixel pi/2 further in phi
    ar = oracle.map2alm(nside, lmax, rot)
    mir = np.empty_like(m0)
    mir[ring_perm(nside, "mirror")] = m0
    am = oracle.map2alm(nside, lmax, mir)
    for l in range(lmax + 1):
        for m in range(l + 1):
            i = oracle.alm_index(lmax, l, m)
            assert abs(ar[i] - a[i] * np.exp(-1j * m * np.pi / 2)) <= 1e-13
            assert abs(am[i] - (-1) ** (l + m) * a[i]) <= 1e-13


def test_alm_index_and_real_map_structure():
    lmax = 9
    seen = sorted(oracle.alm_index(lmax, l, m) for l in range(lmax + 1) for m in range(l + 1))
    assert seen == list(range(oracle.alm_size(lmax)))
    a = oracle.map2alm(4, lmax, np.random.default_rng(2).standard_normal(192))
    for l in range(lmax + 1):
        assert a[oracle.alm_index(lmax, l, 0)].imag == 0.0


def test_constant_map_and_band_limited_recovery():
    nside = 32
    npix = 12 * nside * nside
    a = oracle.map2alm(nside, 8, np.full(npix, 2.5))
    assert abs(a[0] - 2.5 * math.sqrt(4 * math.pi)) <= 1e-13
    # A map synthesised from known a_lm (l <= 6) at the pixel centres is
    # analysed back to them within the pixel quadrature error.
    rng = np.random.default_rng(5)
    lmax = 6
    true = np.zeros(oracle.alm_size(lmax), dtype=complex)
    for l in range(lmax + 1):
        for m in range(l + 1):
            v = rng.standard_normal() + (1j * rng.standard_normal() if m else 0)
            true[oracle.alm_index(lmax, l, m)] = v
    v = oracle.pix2vec(nside, np.arange(npix))
    theta, phi = np.arccos(v[:, 2]), np.arctan2(v[:, 1], v[:, 0])
    hmap = np.zeros(npix)
    for l in range(lmax + 1):
        for m in range(l + 1):
            y = scipy_ylm(l, m, theta, phi)
            t = true[oracle.alm_index(lmax, l, m)] * y
            hmap += t.real if m == 0 else 2 * t.real
    got = oracle.map2alm(nside, lmax, hmap)
    assert np.max(np.abs(got - true)) <= 2e-3 * np.max(np.abs(true))
    cl = oracle.alm2cl(lmax, got)
    cl_true = oracle.alm2cl(lmax, true)
    assert np.allclose(cl, cl_true, rtol=5e-3)


def test_alm2cl_definition():
    lmax = 5
    rng = np.random.default_rng(9)
    a = rng.standard_normal(oracle.alm_size(lmax)) + 1j * rng.standard_normal(oracle.alm_size(lmax))
    cl = oracle.alm2cl(lmax, a)
    for l in range(lmax + 1):
        s = sum((1 if m == 0 else 2) * abs(a[oracle.alm_index(lmax, l, m)]) ** 2
                for m in range(l + 1))
        assert abs(cl[l] - s / (2 * l + 1)) <= 1e-14 * s


def test_ring_sparse_reference_matches_direct_sum():
    """The ring-by-ring reference that the full-size GPU test uses (numpy FFT
    of each ring times the oracle's lambda_lm) equals the oracle's direct
    sum over pixels on a whole map, at every (l, m)."""
    from helpers import ring_sparse_alm
    nside, lmax = 8, 24
    hmap = np.random.default_rng(31).standard_normal(12 * nside * nside)
    ref = oracle.map2alm(nside, lmax, hmap)
    got = ring_sparse_alm(nside, lmax, hmap, list(range(1, 4 * nside)))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
