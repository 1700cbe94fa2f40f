"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, rejects bad arguments before touching the device, and its
host-side tile planner never drops a pixel that can see a box."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csmap.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csmap_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("csmap_create_sky", "csmap_add_box", "csmap_render", "csmap_backward"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1204_5041_amd import binding as B
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTED) == declared_functions()


def test_invalid_arguments_rejected_on_host():
    from paper_1204_5041_amd import binding as B
    L = B.lib()
    out = ctypes.c_void_p()
    assert L.csmap_create_sky(0, 1.0, 1, None, ctypes.byref(out)) == B.CSMAP_E_INVALID
    assert L.csmap_create_sky(8193, 1.0, 1, None, ctypes.byref(out)) == B.CSMAP_E_INVALID
    assert L.csmap_create_sky(64, float("nan"), 1, None, ctypes.byref(out)) == B.CSMAP_E_INVALID
    assert L.csmap_create_sky(64, 1.0, 7, None, ctypes.byref(out)) == B.CSMAP_E_INVALID
    assert L.csmap_create_sky(64, 1.0, 1, None, None) == B.CSMAP_E_INVALID
    assert "nside" in B.csmap_last_error() or B.csmap_last_error()
    assert L.csmap_add_box(None, None, None) == B.CSMAP_E_INVALID
    assert L.csmap_render(None, None) == B.CSMAP_E_INVALID
    assert L.csmap_destroy_sky(None) == B.CSMAP_OK
    assert L.csmap_npix(1) == 12 and L.csmap_npix(8192) == 12 * 8192 ** 2 and L.csmap_npix(0) == -1
    assert L.csmap_pix2vec_ring(16, 0, 10**9, None, None) == B.CSMAP_E_INVALID
    assert L.csmap_pix2vec_ring(16, -1, 1, None, None) == B.CSMAP_E_INVALID


@pytest.mark.parametrize("nside,tile", [(16, 64), (64, 256), (128, 512), (37, 128)])
def test_cap_tiles_cover_every_visible_pixel(nside, tile):
    from paper_1204_5041_amd import binding as B
    rng = np.random.default_rng(nside)
    npx = 12 * nside * nside
    pix = np.arange(npx)
    for trial in range(12):
        c = synth.uniform_directions(1, 1000 + trial + nside)[0]
        if trial == 0:
            c = np.array([0.0, 0.0, 1.0])           # cap on a pole
        if trial == 1:
            c = np.array([1.0, 0.0, 0.0])           # on the equator at phi = 0 (wrap)
        rho = float(np.exp(rng.uniform(np.log(1e-3), np.log(2.5))))
        box = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=0, eta_hi=1,
                        x_rel=np.zeros((0, 3)), xdot=np.zeros((0, 3)), xprime=np.zeros((0, 3)),
                        dsigma=np.zeros(0), vis=synth.VIS_CAP, cap_dir=c, cap_cos=math.cos(rho))
        vis = oracle.visible(nside, pix, 1.0, box)
        ranges = B.csmap_cap_tiles(nside, tile, c, rho)
        covered = np.zeros((npx + tile - 1) // tile, dtype=bool)
        for a, b in ranges:
            covered[a:b + 1] = True
        need = np.unique(pix[vis] // tile)
        assert covered[need].all(), (trial, rho)
        # ranges are sorted and disjoint
        for (a0, b0), (a1, b1) in zip(ranges, ranges[1:]):
            assert b0 + 1 < a1
        # and not wildly larger than needed for small caps
        if rho < 0.3 and vis.any():
            assert covered.sum() <= 8 * max(len(need), 1) + 64


def _ring_of(nside, pix):
    return oracle.ring_of_pixel(nside, np.asarray(pix, dtype=np.int64))[0]


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 13, 64])
@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_ring_blocks_cover_every_pixel_once(nside, k):
    """Rows of the ring-block tiling: every RING pixel in exactly one row, each
    row inside one ring, the rows of a tile on k consecutive rings of one
    block, and at most 64 pixels a row."""
    from paper_1204_5041_amd import binding as B
    rows = B.csmap_ring_block_rows(nside, k)
    npx = 12 * nside * nside
    first = rows >> 7
    cnt = rows & 127
    assert (cnt <= 64).all() and (cnt >= 0).all()
    assert (first[cnt == 0] == 0).all()
    pix = np.concatenate([np.arange(f, f + c) for f, c in zip(first.ravel(), cnt.ravel()) if c])
    assert np.array_equal(np.sort(pix), np.arange(npx))
    nz = cnt > 0
    ring_a = np.zeros_like(first)
    ring_b = np.zeros_like(first)
    ring_a[nz] = _ring_of(nside, first[nz])
    ring_b[nz] = _ring_of(nside, first[nz] + cnt[nz] - 1)
    assert np.array_equal(ring_a[nz], ring_b[nz])
    # Row j of every tile lies on ring (block * k + j + 1): the rings of a tile
    # are consecutive and in order.
    t_idx, j_idx = np.nonzero(nz)
    blocks = (ring_a[nz] - 1 - j_idx) // k
    assert ((ring_a[nz] - 1 - j_idx) % k == 0).all()
    assert (np.diff(blocks[np.argsort(t_idx, kind="stable")]) >= 0).all()


@pytest.mark.parametrize("nside,k", [(8, 4), (16, 8), (32, 2), (64, 8)])
def test_ring_block_tiles_are_azimuth_aligned(nside, k):
    """Chunk c of a block covers azimuths [2 pi 64 c / L, 2 pi 64 (c+1) / L] in
    every ring of the block (L = longest ring), up to one pixel spacing of
    the ring: tiles are compact patches, not strips."""
    from paper_1204_5041_amd import binding as B
    rows = B.csmap_ring_block_rows(nside, k)
    first = rows >> 7
    cnt = rows & 127
    nring = 4 * nside - 1
    ringlen = lambda i: 4 * min(i, nside, 4 * nside - i)
    tile = 0
    for blk in range((nring + k - 1) // k):
        rings = list(range(1 + blk * k, min(nring, (blk + 1) * k) + 1))
        L = max(ringlen(i) for i in rings)
        for c in range((L + 63) // 64):
            lo, hi = 2 * math.pi * 64 * c / L, 2 * math.pi * 64 * (c + 1) / L
            for j, i in enumerate(rings):
                if cnt[tile, j] == 0:
                    continue
                px = np.arange(first[tile, j], first[tile, j] + cnt[tile, j])
                v = oracle.pix2vec(nside, px)
                phi = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * math.pi)
                step = 2 * math.pi / ringlen(i)
                assert phi.min() >= lo - step - 1e-12 and phi.max() <= hi + step + 1e-12
            tile += 1
    assert tile == rows.shape[0]


@pytest.mark.parametrize("nside,k", [(16, 4), (64, 8), (37, 2), (128, 4)])
def test_cap_block_tiles_cover_every_visible_pixel(nside, k):
    from paper_1204_5041_amd import binding as B
    rng = np.random.default_rng(7 * nside + k)
    rows = B.csmap_ring_block_rows(nside, k)
    npx = 12 * nside * nside
    tile_of_pix = np.empty(npx, dtype=np.int64)
    first = rows >> 7
    cnt = rows & 127
    for t in range(rows.shape[0]):
        for j in range(k):
            if cnt[t, j]:
                tile_of_pix[first[t, j]:first[t, j] + cnt[t, j]] = t
    pix = np.arange(npx)
    for trial in range(12):
        c = synth.uniform_directions(1, 2000 + trial + nside)[0]
        if trial == 0:
            c = np.array([0.0, 0.0, -1.0])
        if trial == 1:
            c = np.array([1.0, 0.0, 0.0])
        rho = float(np.exp(rng.uniform(np.log(1e-3), np.log(2.5))))
        box = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=0, eta_hi=1,
                        x_rel=np.zeros((0, 3)), xdot=np.zeros((0, 3)), xprime=np.zeros((0, 3)),
                        dsigma=np.zeros(0), vis=synth.VIS_CAP, cap_dir=c, cap_cos=math.cos(rho))
        vis = oracle.visible(nside, pix, 1.0, box)
        ranges = B.csmap_cap_block_tiles(nside, k, c, rho)
        covered = np.zeros(rows.shape[0], dtype=bool)
        for a, b in ranges:
            covered[a:b + 1] = True
        assert covered[np.unique(tile_of_pix[vis])].all(), (trial, rho)
        for (a0, b0), (a1, b1) in zip(ranges, ranges[1:]):
            assert b0 + 1 < a1


def test_ring_blocks_carry_fewer_idle_lanes_than_strips():
    """At Nside 4096, caps of 0.1%-5% of the sky: the tiles listed for a cap
    hold fewer pixels with ring blocks (4 rings x 64) than with strips of 256
    consecutive pixels, and not many more than the cap itself."""
    from paper_1204_5041_amd import binding as B
    nside, k = 4096, 4
    npx = 12 * nside * nside
    cnt = B.csmap_ring_block_rows(nside, k) & 127
    tile_px = cnt.sum(axis=1)
    cum = np.concatenate([[0], np.cumsum(tile_px)])
    for i, frac in enumerate((0.001, 0.005, 0.05)):
        c = synth.uniform_directions(1, 3000 + i)[0]
        rho = math.acos(1.0 - 2.0 * frac)
        blocks = sum(int(cum[b + 1] - cum[a]) for a, b in B.csmap_cap_block_tiles(nside, k, c, rho))
        strips = sum(min(npx, 64 * k * (b + 1)) - 64 * k * a
                     for a, b in B.csmap_cap_tiles(nside, 64 * k, c, rho))
        assert blocks < strips, (frac, blocks, strips)
        assert blocks < 1.3 * frac * npx, (frac, blocks / (frac * npx))
