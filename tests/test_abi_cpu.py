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
    assert L.csmap_add_snapshot_box(None, None, None) == B.CSMAP_E_INVALID
    assert L.csmap_cone_events(None, 1.0, None, None, None, None) == B.CSMAP_E_INVALID
    bx = B.csmap_box()
    bx.n, bx.dtype, bx.eta_lo, bx.eta_hi = 5, B.CSMAP_F32, 1.0, 0.5   # empty slab
    assert L.csmap_cone_events(ctypes.byref(bx), 2.0, None, None, None, None) == B.CSMAP_E_INVALID
    bx.eta_hi = 2.0                                                   # arrays missing
    assert L.csmap_cone_events(ctypes.byref(bx), 2.0, None, None, None, None) == B.CSMAP_E_INVALID
    bx.n = 0                                                          # nothing to do
    assert L.csmap_cone_events(ctypes.byref(bx), 2.0, None, None, None, None) == B.CSMAP_OK
    # The allocation-free map2alm validates (and refuses scratch needs above
    # its fixed array) before any device call.
    fake = ctypes.c_void_p(0x1000)
    assert L.csmap_map2alm_noalloc(0, 0, fake, fake, None) == B.CSMAP_E_INVALID
    assert L.csmap_map2alm_noalloc(64, 257, fake, fake, None) == B.CSMAP_E_INVALID
    assert L.csmap_map2alm_noalloc(64, 8, None, fake, None) == B.CSMAP_E_INVALID
    assert L.csmap_map2alm_noalloc(1024, 1024, fake, fake, None) == B.CSMAP_E_INVALID
    assert "scratch" in B.csmap_last_error()
    assert L.csmap_map2alm_noalloc(2048, 4096, fake, fake, None) == B.CSMAP_E_INVALID


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


def _split(rows):
    from paper_1204_5041_amd import binding as B
    return rows >> B.ROW_COUNT_BITS, rows & ((1 << B.ROW_COUNT_BITS) - 1)


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 13, 64])
@pytest.mark.parametrize("rings,width", [(1, 64), (2, 64), (4, 64), (8, 64), (4, 128), (16, 16),
                                         (8, 32), (64, 8), (1, 512)])
def test_ring_blocks_cover_every_pixel_once(nside, rings, width):
    """Rows of the ring-block tiling: every RING pixel in exactly one row, each
    row inside one ring, row g of every tile on ring (block * rings + g + 1),
    and at most `width` pixels a row."""
    from paper_1204_5041_amd import binding as B
    rows = B.csmap_ring_block_rows(nside, rings, width)
    npx = 12 * nside * nside
    first, cnt = _split(rows)
    assert (cnt <= width).all() and (cnt >= 0).all()
    assert (first[cnt == 0] == 0).all()
    pix = np.concatenate([np.arange(f, f + c) for f, c in zip(first.ravel(), cnt.ravel()) if c])
    assert np.array_equal(np.sort(pix), np.arange(npx))
    nz = cnt > 0
    ring_a = _ring_of(nside, first[nz])
    ring_b = _ring_of(nside, first[nz] + cnt[nz] - 1)
    assert np.array_equal(ring_a, ring_b)
    t_idx, g_idx = np.nonzero(nz)
    assert ((ring_a - 1 - g_idx) % rings == 0).all()
    blocks = (ring_a - 1 - g_idx) // rings
    assert (np.diff(blocks[np.argsort(t_idx, kind="stable")]) >= 0).all()


@pytest.mark.parametrize("nside,rings,width", [(8, 4, 64), (16, 8, 64), (32, 2, 64),
                                               (64, 8, 64), (64, 4, 128), (64, 16, 16)])
def test_ring_block_tiles_are_azimuth_aligned(nside, rings, width):
    """Chunk c of a block covers azimuths [2 pi w c / L, 2 pi w (c+1) / L] in
    every ring of the block (w = width, L = longest ring), up to one pixel
    spacing of the ring: tiles are compact patches, not strips."""
    from paper_1204_5041_amd import binding as B
    rows = B.csmap_ring_block_rows(nside, rings, width)
    first, cnt = _split(rows)
    nring = 4 * nside - 1
    ringlen = lambda i: 4 * min(i, nside, 4 * nside - i)
    tile = 0
    for blk in range((nring + rings - 1) // rings):
        rs = list(range(1 + blk * rings, min(nring, (blk + 1) * rings) + 1))
        L = max(ringlen(i) for i in rs)
        for c in range((L + width - 1) // width):
            lo, hi = 2 * math.pi * width * c / L, 2 * math.pi * width * (c + 1) / L
            for g, i in enumerate(rs):
                if cnt[tile, g] == 0:
                    continue
                px = np.arange(first[tile, g], first[tile, g] + cnt[tile, g])
                v = oracle.pix2vec(nside, px)
                phi = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * math.pi)
                step = 2 * math.pi / ringlen(i)
                assert phi.min() >= lo - step - 1e-12 and phi.max() <= hi + step + 1e-12
            tile += 1
    assert tile == rows.shape[0]


@pytest.mark.parametrize("nside,rings,width", [(16, 4, 64), (64, 8, 64), (37, 2, 64),
                                               (128, 4, 64), (128, 16, 16), (64, 4, 128)])
def test_cap_block_tiles_cover_every_visible_pixel(nside, rings, width):
    from paper_1204_5041_amd import binding as B
    rng = np.random.default_rng(7 * nside + rings)
    rows = B.csmap_ring_block_rows(nside, rings, width)
    npx = 12 * nside * nside
    tile_of_pix = np.empty(npx, dtype=np.int64)
    first, cnt = _split(rows)
    for t in range(rows.shape[0]):
        for g in range(rings):
            if cnt[t, g]:
                tile_of_pix[first[t, g]:first[t, g] + cnt[t, g]] = t
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
        ranges = B.csmap_cap_block_tiles(nside, rings, width, c, rho)
        covered = np.zeros(rows.shape[0], dtype=bool)
        for a, b in ranges:
            covered[a:b + 1] = True
        assert covered[np.unique(tile_of_pix[vis])].all(), (trial, rho)
        for (a0, b0), (a1, b1) in zip(ranges, ranges[1:]):
            assert b0 + 1 < a1


@pytest.mark.parametrize("rings,width", [(4, 64), (8, 32), (16, 16)])
def test_ring_blocks_carry_fewer_idle_lanes_than_strips(rings, width):
    """At Nside 4096, caps of 0.1%-5% of the sky: the tiles listed for a cap
    hold fewer pixels with ring blocks of 256 pixels than with strips of 256
    consecutive pixels, and not many more than the cap itself."""
    from paper_1204_5041_amd import binding as B
    nside = 4096
    npx = 12 * nside * nside
    _, cnt = _split(B.csmap_ring_block_rows(nside, rings, width))
    cum = np.concatenate([[0], np.cumsum(cnt.sum(axis=1))])
    for i, frac in enumerate((0.001, 0.005, 0.05)):
        c = synth.uniform_directions(1, 3000 + i)[0]
        rho = math.acos(1.0 - 2.0 * frac)
        blocks = sum(int(cum[b + 1] - cum[a])
                     for a, b in B.csmap_cap_block_tiles(nside, rings, width, c, rho))
        strips = sum(min(npx, 256 * (b + 1)) - 256 * a
                     for a, b in B.csmap_cap_tiles(nside, 256, c, rho))
        assert blocks < strips, (frac, blocks, strips)
        assert blocks < 1.3 * frac * npx, (frac, blocks / (frac * npx))


@pytest.mark.parametrize("nside", [3, 16, 40])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
@pytest.mark.parametrize("rings", [1, 2, 4, 16, 64])
def test_ring_block_lane_mapping_covers_map_once(nside, K, rings):
    """The forward kernels' reading of a ring-block tile (rows of
    64 K / rings pixels): lane l serves row l >> s of its tile, with
    s = log2(64 / rings), and holds slots pos0 + j (64 / rings) of that row.
    Every table read stays inside the table, every pixel load inside the
    map, a lane's present slots lie on one ring, and the present slots of
    all tiles cover each pixel exactly once."""
    from paper_1204_5041_amd import binding as B
    width = 64 * K // rings
    rows = B.csmap_ring_block_rows(nside, rings, width).ravel()
    ntiles = rows.size // rings
    npx = 12 * nside * nside
    shift = int(math.log2(64 // rings))
    assert (1 << shift) * rings == 64
    lane = np.arange(64)
    g = lane >> shift
    pos0 = lane - (g << shift)
    step = 1 << shift
    seen = np.zeros(npx, dtype=np.int64)
    for t in range(ntiles):
        idx = t * rings + g
        assert idx.max() < rows.size
        e = rows[idx]
        first, cnt = e >> B.ROW_COUNT_BITS, e & ((1 << B.ROW_COUNT_BITS) - 1)
        ring_of_lane = None
        for j in range(K):
            pos = pos0 + j * step
            present = pos < cnt
            off = np.where(present, pos, np.maximum(cnt - 1, 0))
            pix = first + off
            assert pix.min() >= 0 and pix.max() < npx
            np.add.at(seen, pix[present], 1)
            r = _ring_of(nside, pix)
            ring_of_lane = r if ring_of_lane is None else ring_of_lane
            assert np.array_equal(r[present], ring_of_lane[present])
    assert (seen == 1).all()
