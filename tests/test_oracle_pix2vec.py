"""Pins of the oracle's HEALPix RING pixel centres (the map directions of
the paper's Sec. II.D, following the published HEALPix definition).

Every check here is against something other than the oracle itself: a
brute-force enumeration of the ring layout, exact rational arithmetic for
z, 50-digit mpmath for the trigonometric part, the Nside=1 base-pixel
layout, and exact symmetries of the pixelisation."""
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "healpix_nside1.txt")
NSIDES = [1, 2, 3, 4, 5, 7, 8, 16, 32, 64]


def brute_force_layout(nside):
    """(ring, position) of every pixel, by walking the rings in order:
    4i pixels in north-cap ring i < N, 4N in each belt ring N..3N, and the
    south cap mirroring the north."""
    lens = [4 * i for i in range(1, nside)] + [4 * nside] * (2 * nside + 1) + \
           [4 * i for i in range(nside - 1, 0, -1)]
    ring, pos = [], []
    for r, L in enumerate(lens, start=1):
        ring += [r] * L
        pos += list(range(L))
    return np.array(ring), np.array(pos), lens


def exact_z(nside, ring):
    """z of a ring as an exact rational (HEALPix: 1 - i^2/(3N^2) in the
    north cap, (4N - 2i)/(3N) in the belt, mirrored in the south cap)."""
    n = nside
    if ring < n:
        return 1 - Fraction(ring * ring, 3 * n * n)
    if ring > 3 * n:
        k = 4 * n - ring
        return -(1 - Fraction(k * k, 3 * n * n))
    return Fraction(4 * n - 2 * ring, 3 * n)


def test_isqrt_exact():
    for x in list(range(0, 5000)) + [2**52 - 1, 2**52, 2**52 + 1, 4 * 8192**2 * 3 + 7,
                                     (2**31 - 1) ** 2, (2**31 - 1) ** 2 - 1]:
        r = oracle.isqrt(x)
        assert r * r <= x < (r + 1) * (r + 1), x


@pytest.mark.parametrize("nside", NSIDES + [128, 256])
def test_integer_stage_matches_brute_force(nside):
    ring_bf, pos_bf, lens = brute_force_layout(nside)
    assert len(ring_bf) == 12 * nside * nside
    assert len(lens) == 4 * nside - 1
    ring, pos = oracle.ring_of_pixel(nside, np.arange(12 * nside * nside))
    np.testing.assert_array_equal(ring, ring_bf)
    np.testing.assert_array_equal(pos, pos_bf)


def test_integer_stage_large_nside_samples():
    # Ring starts and ends at Nside = 8192, where isqrt works near 2^30.
    n = 8192
    starts = []
    acc = 0
    for i in range(1, 4 * n):
        L = 4 * i if i < n else (4 * n if i <= 3 * n else 4 * (4 * n - i))
        starts.append((i, acc, L))
        acc += L
    assert acc == 12 * n * n
    rng = np.random.default_rng(5)
    pick = [starts[k] for k in rng.choice(len(starts), 400, replace=False)]
    pix, exp_ring, exp_pos = [], [], []
    for i, s, L in pick:
        for off in (0, 1, L // 2, L - 2, L - 1):
            pix.append(s + off)
            exp_ring.append(i)
            exp_pos.append(off)
    ring, pos = oracle.ring_of_pixel(n, np.array(pix))
    np.testing.assert_array_equal(ring, exp_ring)
    np.testing.assert_array_equal(pos, exp_pos)


def test_nside1_base_pixels_golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    v = oracle.pix2vec(1, np.arange(12))
    for r in rows:
        p, zn, zd, q = int(r[0]), int(r[1]), int(r[2]), int(r[3])
        assert v[p, 2] == float(Fraction(zn, zd))
        phi = math.atan2(v[p, 1], v[p, 0]) % (2 * math.pi)
        assert abs(phi - q * math.pi / 4) < 1e-15 or abs(phi - q * math.pi / 4 - 2 * math.pi) < 1e-15
    # pixel 4 is exactly the +x axis
    assert tuple(v[4]) == (1.0, 0.0, 0.0)


@pytest.mark.parametrize("nside", NSIDES)
def test_z_is_correctly_rounded_rational(nside):
    ring, _ = oracle.ring_of_pixel(nside, np.arange(12 * nside * nside))
    v = oracle.pix2vec(nside, np.arange(12 * nside * nside))
    for r in range(1, 4 * nside):
        zs = v[ring == r, 2]
        assert np.all(zs == float(exact_z(nside, r))), (nside, r)


def _phi_expected(nside, ring, pos):
    """Azimuth of a pixel centre in quarter turns, as an exact rational:
    cap rings (and their mirrors) are offset by half a pixel; belt rings
    alternate, ring N carrying the same half-pixel offset as the cap."""
    n = nside
    if ring < n or ring > 3 * n:
        k = ring if ring < n else 4 * n - ring
        return Fraction(2 * pos + 1, 2 * k)
    half = 1 if (ring - n) % 2 == 0 else 0
    return Fraction(2 * pos + half, 2 * n)


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 13, 32])
def test_directions_against_mpmath(nside):
    mp.mp.dps = 50
    npx = 12 * nside * nside
    pix = np.arange(npx) if npx <= 3072 else np.random.default_rng(nside).choice(npx, 3072, replace=False)
    ring, pos = oracle.ring_of_pixel(nside, pix)
    v = oracle.pix2vec(nside, pix)
    worst = 0.0
    for k, p in enumerate(pix):
        z = exact_z(nside, int(ring[k]))
        st = mp.sqrt(1 - mp.mpf(z.numerator) ** 2 / mp.mpf(z.denominator) ** 2)
        phi = mp.pi / 2 * mp.mpf(_phi_expected(nside, int(ring[k]), int(pos[k])).numerator) / \
            _phi_expected(nside, int(ring[k]), int(pos[k])).denominator
        ex = (st * mp.cos(phi), st * mp.sin(phi))
        for c in range(2):
            err = abs(mp.mpf(v[k, c]) - ex[c])
            # error in units of the last place of a number of size 1/2..1
            worst = max(worst, float(err / mp.mpf(2) ** -53))
    # A few rounding steps (division, sqrt, polynomial, product): bounded by 4 ulp of 1.
    assert worst <= 4.0, worst


@pytest.mark.parametrize("nside", [1, 2, 4, 5, 16, 64])
def test_unit_norm_and_zero_sum(nside):
    v = oracle.pix2vec(nside, np.arange(12 * nside * nside))
    norm = np.sqrt(np.sum(v * v, axis=1))
    assert np.max(np.abs(norm - 1.0)) < 4e-16
    assert np.max(np.abs(v.sum(axis=0))) < 1e-12 * v.shape[0]


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 32])
def test_quarter_turn_and_mirror_symmetry_exact(nside):
    """Rotating by 90 degrees about z maps pixel j of a ring of length L to
    pixel j + L/4, bit for bit; mirroring z maps ring i to ring 4N - i."""
    npx = 12 * nside * nside
    v = oracle.pix2vec(nside, np.arange(npx))
    ring, pos = oracle.ring_of_pixel(nside, np.arange(npx))
    start = {}
    length = {}
    for p in range(npx):
        r = int(ring[p])
        start.setdefault(r, p)
        length[r] = length.get(r, 0) + 1
    for p in range(npx):
        r, j, L = int(ring[p]), int(pos[p]), length[int(ring[p])]
        q = start[r] + (j + L // 4) % L
        assert v[q, 0] == -v[p, 1] and v[q, 1] == v[p, 0] and v[q, 2] == v[p, 2]
        m = start[4 * nside - r] + j
        assert v[m, 0] == v[p, 0] and v[m, 1] == v[p, 1] and v[m, 2] == -v[p, 2]


def test_ring_spacing_uniform():
    nside = 16
    v = oracle.pix2vec(nside, np.arange(12 * nside * nside))
    ring, _ = oracle.ring_of_pixel(nside, np.arange(12 * nside * nside))
    for r in range(1, 4 * nside):
        phi = np.unwrap(np.arctan2(v[ring == r, 1], v[ring == r, 0]))
        d = np.diff(phi)
        assert np.allclose(d, 2 * np.pi / len(phi), atol=1e-13)
