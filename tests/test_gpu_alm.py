"""GPU spherical-harmonic analysis of RING maps (csmap_map2alm,
csmap_alm2cl) against the oracle's direct sum over pixels.  Bars: every
a_lm within 1e-11 of max |a_lm| (1e-10 at Nside 256, lmax 1024, where the
Legendre recursion runs thousands of steps), C_l within 1e-10 relative;
at full size (Nside 2048, lmax 4096), where the oracle is out of reach, the
exact symmetries of the HEALPix grid: a quarter turn in azimuth multiplies
a_lm by e^{-i m pi/2} and the north-south mirror by (-1)^(l+m)."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    return binding


def gpu_alm(B, hmap, lmax):
    return B.map2alm(torch.from_numpy(np.ascontiguousarray(hmap)).cuda(), lmax).cpu().numpy()


# Powers of two take the FFT of the belt rings, other Nside the direct sums.
# Nside 2 and 3 take the smallest transforms (a one-point chirp transform for
# the first cap ring, a radix-4 belt FFT at Nside 2), lmax 0 the shortest
# recursion.
@pytest.mark.parametrize("nside,lmax", [(1, 4), (4, 12), (8, 16), (16, 64), (32, 64), (64, 128),
                                        (12, 48), (48, 96), (64, 256), (2, 8), (3, 11), (2, 0),
                                        (8, 0)])
def test_map2alm_matches_oracle(B, nside, lmax):
    rng = np.random.default_rng(100 + nside)
    hmap = rng.standard_normal(12 * nside * nside) + 0.3
    say(f"map2alm nside={nside} lmax={lmax}")
    got = gpu_alm(B, hmap, lmax)
    ref = oracle.map2alm(nside, lmax, hmap)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"  max |da| / max |a| = {err:.3e}")
    assert err <= 1e-11
    cl = B.alm2cl(torch.from_numpy(got).cuda(), lmax).cpu().numpy()
    cl_ref = oracle.alm2cl(lmax, ref)
    assert np.max(np.abs(cl - cl_ref) / cl_ref) <= 1e-10


def test_map2alm_high_degree_sampled_m(B):
    """Nside 256, lmax 1024 (= 4 Nside): m = 0, 7, 500 and 1000, the last two
    starting far below the double range near the poles."""
    nside, lmax = 256, 1024
    hmap = np.random.default_rng(7).standard_normal(12 * nside * nside)
    say("map2alm nside=256 lmax=1024")
    got = gpu_alm(B, hmap, lmax)
    ms = (0, 7, 500, 1000)
    with ThreadPoolExecutor(max_workers=len(ms)) as ex:
        refs = list(ex.map(lambda m: oracle.map2alm_m(nside, lmax, m, hmap), ms))
    for m, ref in zip(ms, refs):
        idx = [oracle.alm_index(lmax, l, m) for l in range(m, lmax + 1)]
        err = np.max(np.abs(got[idx] - ref)) / np.max(np.abs(ref))
        say(f"  m={m}: max |da| / max |a_m| = {err:.3e}")
        assert err <= 1e-10, (m, err)


def test_power_spectrum_of_a_string_map(B):
    """The FP64-form map of the plain workload (Nside 64, 2,000 segments)
    analysed on the device against the oracle's analysis of the oracle's map."""
    from helpers import sky_from_workload
    w = synth.config0()
    lmax = 128
    ref_map = oracle.theta_pixels(w.nside, np.arange(w.npix), w.eta0, w.boxes)
    sky = sky_from_workload(w, B.CSMAP_FORM_FP64)
    m = sky.render()
    alm = B.map2alm(m, lmax)
    cl = B.alm2cl(alm, lmax).cpu().numpy()
    sky.close()
    cl_ref = oracle.alm2cl(lmax, oracle.map2alm(w.nside, lmax, ref_map))
    err = np.max(np.abs(cl - cl_ref) / cl_ref)
    say(f"string map C_l max rel err {err:.3e}; C_2 = {cl[2]:.6e}, C_100 = {cl[100]:.6e}")
    assert err <= 1e-9


def symmetry_perms(nside):
    """Pixel permutations of the quarter turn phi -> phi + pi/2 and of the
    mirror z -> -z, from the ring structure (vectorised)."""
    npix = 12 * nside * nside
    ring, pos = oracle.ring_of_pixel(nside, np.arange(npix))
    N = nside
    L = 4 * np.minimum(np.minimum(ring, N), 4 * N - ring)
    first = np.where(ring < N, 2 * ring * (ring - 1),
                     np.where(ring <= 3 * N, 2 * N * (N - 1) + (ring - N) * 4 * N,
                              npix - 2 * (4 * N - ring) * (4 * N - ring + 1)))
    quarter = first + (pos + L // 4) % L
    mir_ring = 4 * N - ring
    mfirst = np.where(mir_ring < N, 2 * mir_ring * (mir_ring - 1),
                      np.where(mir_ring <= 3 * N, 2 * N * (N - 1) + (mir_ring - N) * 4 * N,
                               npix - 2 * (4 * N - mir_ring) * (4 * N - mir_ring + 1)))
    mirror = mfirst + pos
    return quarter, mirror


def test_full_size_grid_symmetries(B):
    nside, lmax = 2048, 4096
    npix = 12 * nside * nside
    hmap = np.random.default_rng(11).standard_normal(npix)
    quarter, mirror = symmetry_perms(nside)
    assert np.array_equal(np.sort(quarter), np.arange(npix))
    rot = np.empty(npix)
    rot[quarter] = hmap
    mir = np.empty(npix)
    mir[mirror] = hmap
    say("map2alm nside=2048 lmax=4096, three maps")
    a = gpu_alm(B, hmap, lmax)
    ar = gpu_alm(B, rot, lmax)
    am = gpu_alm(B, mir, lmax)
    l = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    m = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
    order = np.array([oracle.alm_index(lmax, 0, 0)])   # index layout check
    assert order[0] == 0
    scale = np.max(np.abs(a))
    e_rot = np.max(np.abs(ar - a * np.exp(-1j * m * np.pi / 2))) / scale
    e_mir = np.max(np.abs(am - (-1.0) ** (l + m) * a)) / scale
    say(f"  quarter turn {e_rot:.3e}, mirror {e_mir:.3e}")
    assert e_rot <= 1e-10 and e_mir <= 1e-10
    # A white-noise map of unit variance has C_l close to 4 pi / Npix.
    cl = B.alm2cl(torch.from_numpy(a).cuda(), lmax).cpu().numpy()
    assert abs(np.mean(cl[2:]) / (4 * np.pi / npix) - 1) < 0.01


def test_full_size_ring_sparse_map(B):
    """Nside 2048, lmax 4096 on a map that is non-zero only on a few rings:
    cap rings whose quarter-length transforms take every chirp-transform
    size from 1 to 4096 points (i = 1, 2, 3, 5, 64, 65, 513, 1024, 1025,
    2047 in the north cap, 1, 700, 2047 in the south) and two belt rings."""
    nside, lmax = 2048, 4096
    N = nside
    npix = 12 * N * N
    rings = [1, 2, 3, 5, 64, 65, 513, 1024, 1025, 2047, N, 2 * N + 1,
             4 * N - 1, 4 * N - 700, 4 * N - 2047]
    rng = np.random.default_rng(29)
    hmap = np.zeros(npix)
    ref_rings = []
    for r in rings:
        if r < N:
            L, first = 4 * r, 2 * r * (r - 1)
        elif r <= 3 * N:
            L, first = 4 * N, 2 * N * (N - 1) + (r - N) * 4 * N
        else:
            k = 4 * N - r
            L, first = 4 * k, npix - 2 * k * (k + 1)
        hmap[first:first + L] = rng.standard_normal(L) + 0.2
        ref_rings.append(r)
    say("map2alm nside=2048 lmax=4096, ring-sparse map")
    got = gpu_alm(B, hmap, lmax)
    from helpers import ring_sparse_alm
    ref = ring_sparse_alm(nside, lmax, hmap, ref_rings)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    say(f"  max |da| / max |a| = {err:.3e}")
    assert err <= 1e-11
