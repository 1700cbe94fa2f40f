"""Pins of the oracle's direction -> HEALPix RING pixel map (ang2pix), which
decides which strings live inside a healpix cone when simulations are
stacked (Sec. II.C, Fig. 1).

Every check is against something other than ang2pix itself: the pixel
centres (pinned separately against exact rationals and mpmath), the Nside=1
base-pixel layout, brute-force nearest-centre search along ring-centre
latitudes, the diamond shape of belt pixels along their centre meridian,
exact symmetries of the grid, and the equal-area property."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "healpix_nside1.txt")


def ring_first(nside, ring):
    n = nside
    ring = np.asarray(ring)
    return np.where(ring < n, 2 * ring * (ring - 1),
                    np.where(ring <= 3 * n, 2 * n * (n - 1) + (ring - n) * 4 * n,
                             12 * n * n - 2 * (4 * n - ring) * (4 * n - ring + 1)))


def ring_len(nside, ring):
    n = nside
    ring = np.asarray(ring)
    return 4 * np.minimum(np.minimum(ring, n), 4 * n - ring)


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 5, 7, 8, 13, 16, 32, 64, 128])
def test_pixel_centres_map_to_their_pixel(nside):
    pix = np.arange(12 * nside * nside)
    np.testing.assert_array_equal(oracle.ang2pix(nside, oracle.pix2vec(nside, pix)), pix)


@pytest.mark.parametrize("nside", [1024, 2048, 4096, 8192])
def test_pixel_centres_large_nside(nside):
    npx = 12 * nside * nside
    rng = np.random.default_rng(nside)
    pix = np.concatenate([rng.integers(0, npx, 200_000), np.arange(64), npx - 1 - np.arange(64),
                          2 * nside * (nside - 1) + np.arange(-8, 8)])
    np.testing.assert_array_equal(oracle.ang2pix(nside, oracle.pix2vec(nside, pix)), pix)


def test_nside1_golden_directions():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for r in rows:
        p, zn, zd, q = int(r[0]), int(r[1]), int(r[2]), int(r[3])
        z = zn / zd
        phi = q * math.pi / 4
        s = math.sqrt(1 - z * z)
        v = np.array([[s * math.cos(phi), s * math.sin(phi), z]])
        assert oracle.ang2pix(1, v)[0] == p
        # any positive length
        assert oracle.ang2pix(1, 1e-3 * v)[0] == p and oracle.ang2pix(1, 7e5 * v)[0] == p


def test_poles_and_axes():
    for n in (1, 2, 16, 1024, 8192):
        assert oracle.ang2pix(n, np.array([[0.0, 0.0, 1.0]]))[0] == 0
        assert oracle.ang2pix(n, np.array([[0.0, 0.0, -3.0]]))[0] == 12 * n * n - 4
        # a direction a hair off the north pole at azimuth just below 2 pi
        assert oracle.ang2pix(n, np.array([[1e-9, -1e-15, 1.0]]))[0] == 3


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 16, 32])
def test_ring_centre_latitude_is_nearest_centre_in_azimuth(nside):
    """On the latitude of a ring's centres, pixel edges cross only at the
    east and west corners, which sit half-way between centres: the pixel of
    a direction there is the ring's pixel with the nearest centre azimuth."""
    rng = np.random.default_rng(40 + nside)
    npx = 12 * nside * nside
    ring, _ = oracle.ring_of_pixel(nside, np.arange(npx))
    cen = oracle.pix2vec(nside, np.arange(npx))
    cen_phi = np.arctan2(cen[:, 1], cen[:, 0]) % (2 * np.pi)
    for r in range(1, 4 * nside):
        members = np.nonzero(ring == r)[0]
        z = cen[members[0], 2]
        phi = rng.uniform(0, 2 * np.pi, 64)
        s = math.sqrt(1 - z * z)
        v = np.stack([s * np.cos(phi), s * np.sin(phi), np.full_like(phi, z)], 1)
        got = oracle.ang2pix(nside, v)
        d = np.abs((phi[:, None] - cen_phi[members][None, :] + np.pi) % (2 * np.pi) - np.pi)
        np.testing.assert_array_equal(got, members[np.argmin(d, 1)])


@pytest.mark.parametrize("nside", [2, 4, 8, 16])
def test_belt_pixels_span_neighbour_ring_latitudes_on_their_meridian(nside):
    """Belt pixels are diamonds whose north and south corners lie on their
    centre meridian at the latitudes of the rings above and below."""
    n = nside
    rng = np.random.default_rng(n)
    for r in range(n + 1, 3 * n):
        first = ring_first(n, r)
        for p in first + rng.choice(4 * n, 6, replace=False):
            c = oracle.pix2vec(n, [p])[0]
            phi = math.atan2(c[1], c[0])
            z_hi = (4 * n - 2 * (r - 1)) / (3 * n)
            z_lo = (4 * n - 2 * (r + 1)) / (3 * n)
            z = z_lo + (z_hi - z_lo) * rng.uniform(0.001, 0.999, 32)
            s = np.sqrt(1 - z * z)
            v = np.stack([s * math.cos(phi), s * math.sin(phi), z], 1)
            assert np.all(oracle.ang2pix(n, v) == p), (n, r, p)


@pytest.mark.parametrize("nside", [1, 4, 16, 64])
def test_quarter_turn_and_mirror_symmetry(nside):
    n = nside
    rng = np.random.default_rng(90 + n)
    d = rng.standard_normal((50_000, 3))
    p = oracle.ang2pix(n, d)
    ring, pos = oracle.ring_of_pixel(n, p)
    L = ring_len(n, ring)
    quarter = ring_first(n, ring) + (pos + L // 4) % L
    rot = np.stack([-d[:, 1], d[:, 0], d[:, 2]], 1)
    np.testing.assert_array_equal(oracle.ang2pix(n, rot), quarter)
    mir = ring_first(n, 4 * n - ring) + pos
    np.testing.assert_array_equal(oracle.ang2pix(n, d * np.array([1.0, 1.0, -1.0])), mir)


@pytest.mark.parametrize("nside", [2, 8])
def test_equal_area(nside):
    """Isotropic directions land in the 12 Nside^2 pixels with equal
    probability (HEALPix pixels have equal areas)."""
    npx = 12 * nside * nside
    rng = np.random.default_rng(7 + nside)
    counts = np.zeros(npx, dtype=np.int64)
    for _ in range(4):
        counts += np.bincount(oracle.ang2pix(nside, rng.standard_normal((1_000_000, 3))),
                              minlength=npx)
    chi2 = np.sum((counts - counts.mean()) ** 2 / counts.mean())
    pval = stats.chi2.sf(chi2, npx - 1)
    assert pval > 1e-4, (chi2, pval)
    # An area error of 2% in one ring would give chi2 far beyond that.
    assert np.max(np.abs(counts / counts.mean() - 1)) < 6 * math.sqrt(npx / 4e6)


def test_polar_accuracy_near_the_pole():
    """Directions 1e-9 rad from either pole at Nside 8192 land in the four
    pixels of the first (last) ring, chosen by their quarter of azimuth."""
    n = 8192
    for k in range(4):
        phi = (k + 0.5) * math.pi / 2
        v = np.array([[1e-9 * math.cos(phi), 1e-9 * math.sin(phi), 1.0]])
        assert oracle.ang2pix(n, v)[0] == k
        assert oracle.ang2pix(n, v * np.array([1, 1, -1]))[0] == 12 * n * n - 4 + k


def test_quarter_turns_recipe_against_mpmath():
    """The fixed arctangent recipe (quadrant fold, one ratio, a fold at
    tan(pi/8), a Maclaurin series) against atan2 at 40 digits: within 3 ulp
    of phi/(pi/2) over random directions, the axes, the diagonals, both sides
    of the tan(pi/8) fold, and tiny components."""
    import mpmath
    mpmath.mp.dps = 40
    rng = np.random.default_rng(77)
    xy = [rng.standard_normal((20000, 2)),
          rng.standard_normal((2000, 2)) * np.array([1.0, 1e-12]),
          rng.standard_normal((2000, 2)) * np.array([1e-12, 1.0])]
    t8 = 0.41421356237309503
    fold = []
    for r in (t8, np.nextafter(t8, 0), np.nextafter(t8, 1), 0.5, 1.0, 1e-300, 0.0):
        for sx in (1, -1):
            for sy in (1, -1):
                fold += [(sx * 1.0, sy * r), (sx * r, sy * 1.0)]
    xy.append(np.array(fold))
    xy.append(np.array([(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1),
                        (3e-310, 1.0), (-5.0, -0.0), (2.0, -0.0)], dtype=float))
    xy = np.concatenate(xy)
    got = oracle.quarter_turns(xy)
    assert np.all((got >= 0.0) & (got < 4.0))
    worst = 0.0
    for (x, y), t in zip(xy, got):
        ref = mpmath.atan2(mpmath.mpf(float(y)), mpmath.mpf(float(x))) / (mpmath.pi / 2)
        if ref < 0:
            ref += 4
        d = abs(mpmath.mpf(float(t)) - ref)
        d = min(d, abs(d - 4))            # 4 and 0 are the same azimuth
        ulp = float(np.spacing(max(float(ref), 1e-300)))
        worst = max(worst, float(d) / max(ulp, np.spacing(1.0) / 4))
    assert worst <= 3.0, worst
    # exact values at the axes
    axes = oracle.quarter_turns(np.array([(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]))
    assert list(axes) == [0.0, 1.0, 2.0, 3.0]
