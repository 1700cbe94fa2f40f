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
