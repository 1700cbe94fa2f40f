"""FP64 CPU oracle for the all-sky string ISW map (test infrastructure only).

This package is the independent reference that the HIP library is checked
against.  It is used by the test-suite, by ``__graft_entry__.smoke()`` and by
the CPU-baseline leg of ``bench.py``; the product library never imports,
links or executes it.  The arithmetic lives in ``csmap_oracle.c`` (plain C,
IEEE double, no floating-point contraction); this module only builds it and
marshals numpy arrays through ``ctypes``.

Inputs follow the shapes the workload generator produces: per box an origin,
an extent, a conformal-time slab, a visibility rule, and segment arrays
``x_rel (n,3)``, ``xdot (n,3)``, ``xprime (n,3)``, ``dsigma (n,)``.  Values
stored in float32 are widened to float64 exactly before they reach the C code,
so the oracle sees the very numbers the GPU sees.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csmap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

VIS_ALL, VIS_BOX, VIS_CAP = 0, 1, 2
BOX_STRIDE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        i64, f64p, i64p, u8p = (ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint8))
        _lib.oracle_isqrt.argtypes = [i64]
        _lib.oracle_isqrt.restype = i64
        _lib.oracle_pix2vec_many.argtypes = [i64, i64, i64p, f64p]
        _lib.oracle_ring_many.argtypes = [i64, i64, i64p, i64p, i64p]
        _lib.oracle_lambda_lm.argtypes = [i64, i64, ctypes.c_double, ctypes.c_double, f64p]
        _lib.oracle_alm_index.argtypes = [i64, i64, i64]
        _lib.oracle_alm_index.restype = i64
        _lib.oracle_map2alm.argtypes = [i64, i64, f64p, f64p, f64p]
        _lib.oracle_map2alm_m.argtypes = [i64, i64, i64, f64p, f64p, f64p]
        _lib.oracle_alm2cl.argtypes = [i64, f64p, f64p, f64p]
        _lib.oracle_ang2pix_many.argtypes = [i64, i64, f64p, i64p]
        _lib.oracle_quarter_turns_many.argtypes = [i64, f64p, f64p]
        _lib.oracle_flat_theta.argtypes = [i64, i64, ctypes.c_double, f64p, ctypes.c_double,
                                           ctypes.c_double, i64, f64p, i64p, f64p, f64p, f64p,
                                           f64p, f64p]
        _lib.oracle_flat_points.argtypes = [i64, f64p, f64p, ctypes.c_double, ctypes.c_double,
                                            i64, f64p, i64p, f64p, f64p, f64p, f64p, f64p]
        _lib.oracle_cone_events.argtypes = [i64, f64p, f64p, f64p, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, f64p, f64p, u8p]
        _lib.oracle_theta_dirs.argtypes = [i64, f64p, ctypes.c_double, i64, f64p, i64p,
                                           f64p, f64p, f64p, f64p, ctypes.c_int, f64p]
        _lib.oracle_theta_pixels.argtypes = [i64, i64, i64p, ctypes.c_double, i64, f64p, i64p,
                                             f64p, f64p, f64p, f64p, f64p]
        _lib.oracle_visible_many.argtypes = [i64, i64, i64p, ctypes.c_double, f64p, u8p]
        _lib.oracle_kept_many.argtypes = [i64, f64p, ctypes.c_double, f64p, f64p, f64p, f64p,
                                          u8p]
        _lib.oracle_grad.argtypes = [i64, i64, i64p, f64p, ctypes.c_double, i64, f64p, i64p,
                                     f64p, f64p, f64p, f64p, i64, i64p, f64p]
        _lib.oracle_grad_abs.argtypes = _lib.oracle_grad.argtypes
        _lib.oracle_num_threads.restype = ctypes.c_int
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ----------------------------------------------------------------------------
# HEALPix RING geometry (Gorski et al. 2005, the pixelisation of Sec. II.D)
# ----------------------------------------------------------------------------

def npix(nside: int) -> int:
    return 12 * nside * nside


def isqrt(x: int) -> int:
    return int(lib().oracle_isqrt(int(x)))


def ring_of_pixel(nside: int, pix) -> tuple[np.ndarray, np.ndarray]:
    """(ring 1..4N-1, 0-based position in the ring) of each RING pixel."""
    p = _i64(pix).ravel()
    ring = np.empty_like(p)
    pos = np.empty_like(p)
    lib().oracle_ring_many(nside, p.size, _p(p, ctypes.c_int64), _p(ring, ctypes.c_int64),
                           _p(pos, ctypes.c_int64))
    return ring, pos


def pix2vec(nside: int, pix) -> np.ndarray:
    """Unit vectors (n,3) of RING pixel centres."""
    p = _i64(pix).ravel()
    out = np.empty((p.size, 3), dtype=np.float64)
    lib().oracle_pix2vec_many(nside, p.size, _p(p, ctypes.c_int64), _p(out, ctypes.c_double))
    return out


# ----------------------------------------------------------------------------
# Boxes and segments
# ----------------------------------------------------------------------------

def box_record(box) -> np.ndarray:
    """Pack one box (an object with origin, ext, eta_lo, eta_hi, vis, cap_dir,
    cap_cos attributes) into the 16-double record the C code reads."""
    r = np.zeros(BOX_STRIDE, dtype=np.float64)
    r[0:3] = np.asarray(box.origin, dtype=np.float64)
    r[3:6] = np.asarray(box.ext, dtype=np.float64)
    r[6] = box.eta_lo
    r[7] = box.eta_hi
    r[8] = int(box.vis)
    if box.cap_dir is not None:
        r[9:12] = np.asarray(box.cap_dir, dtype=np.float64)
    r[12] = box.cap_cos if box.cap_cos is not None else 0.0
    return r


class _Packed:
    def __init__(self, boxes: Sequence):
        self.nbox = len(boxes)
        self.boxes = np.ascontiguousarray(np.stack([box_record(b) for b in boxes]) if boxes
                                          else np.zeros((0, BOX_STRIDE)))
        counts = [len(b.dsigma) for b in boxes]
        self.seg_off = _i64(np.concatenate([[0], np.cumsum(counts)]))
        cat = (lambda name, shape: _f64(np.concatenate([getattr(b, name) for b in boxes]))
               if boxes else np.zeros(shape))
        self.x = cat("x_rel", (0, 3)).reshape(-1, 3)
        self.xd = cat("xdot", (0, 3)).reshape(-1, 3)
        self.xp = cat("xprime", (0, 3)).reshape(-1, 3)
        self.ds = cat("dsigma", (0,)).ravel()

    def args(self):
        c = ctypes.c_double
        return (self.nbox, _p(self.boxes, c), _p(self.seg_off, ctypes.c_int64),
                _p(self.x, c), _p(self.xd, c), _p(self.xp, c), _p(self.ds, c))


def theta_dirs(dirs, eta0: float, boxes: Sequence, use_vis: bool = False) -> np.ndarray:
    """Theta/GU (Eq. 1) at arbitrary unit directions (n,3)."""
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty(d.shape[0], dtype=np.float64)
    pk = _Packed(boxes)
    lib().oracle_theta_dirs(d.shape[0], _p(d, ctypes.c_double), float(eta0), *pk.args(),
                            int(bool(use_vis)), _p(out, ctypes.c_double))
    return out


def theta_pixels(nside: int, pix, eta0: float, boxes: Sequence) -> np.ndarray:
    """Theta/GU at RING pixel centres, each pixel summing the boxes it sees."""
    p = _i64(pix).ravel()
    out = np.empty(p.size, dtype=np.float64)
    pk = _Packed(boxes)
    lib().oracle_theta_pixels(nside, p.size, _p(p, ctypes.c_int64), float(eta0), *pk.args(),
                              _p(out, ctypes.c_double))
    return out


def visible(nside: int, pix, eta0: float, box) -> np.ndarray:
    p = _i64(pix).ravel()
    out = np.empty(p.size, dtype=np.uint8)
    rec = box_record(box)
    lib().oracle_visible_many(nside, p.size, _p(p, ctypes.c_int64), float(eta0),
                              _p(rec, ctypes.c_double), _p(out, ctypes.c_uint8))
    return out.astype(bool)


def kept(eta0: float, box) -> np.ndarray:
    """Light-cone selection flag of every segment of one box."""
    rec = box_record(box)
    x, xd, xp, ds = (_f64(box.x_rel).reshape(-1, 3), _f64(box.xdot).reshape(-1, 3),
                     _f64(box.xprime).reshape(-1, 3), _f64(box.dsigma).ravel())
    out = np.empty(ds.size, dtype=np.uint8)
    c = ctypes.c_double
    lib().oracle_kept_many(ds.size, _p(rec, c), float(eta0), _p(x, c), _p(xd, c), _p(xp, c),
                           _p(ds, c), _p(out, ctypes.c_uint8))
    return out.astype(bool)


def grad(nside: int, pix, cotangent, eta0: float, boxes: Sequence, sel,
         absolute: bool = False) -> np.ndarray:
    """Gradient of sum_p g_p Theta_p/GU over the listed pixels with respect to
    (x_rel[3], xdot[3], xprime[3], dsigma) of the selected segments.

    ``sel`` holds global segment indices (box-major concatenation order).
    Returns an array (len(sel), 10).  With absolute=True, every pixel's
    contribution enters in absolute value: sum_p |g_p df_p/dtheta|, the scale
    of each component before its terms cancel."""
    p = _i64(pix).ravel()
    g = _f64(cotangent).ravel()
    if g.size != p.size:
        raise ValueError("cotangent must have one value per listed pixel")
    s = _i64(sel).ravel()
    pk = _Packed(boxes)
    if s.size and (s.min() < 0 or s.max() >= pk.seg_off[-1]):
        raise ValueError("segment index out of range")
    out = np.empty((s.size, 10), dtype=np.float64)
    fn = lib().oracle_grad_abs if absolute else lib().oracle_grad
    fn(nside, p.size, _p(p, ctypes.c_int64), _p(g, ctypes.c_double), float(eta0), *pk.args(),
       s.size, _p(s, ctypes.c_int64), _p(out, ctypes.c_double))
    return out


def cone_events(x_rel, xdot, origin, eta0: float, eta_lo: float, eta_hi: float):
    """Light-cone crossings of segments given at the slab start eta_lo
    (straight worldlines P0 + Xdot (eta - eta_lo), P0 = origin + x_rel).

    Returns (pos (n,3) observer-relative event positions, delta (n,) crossing
    time after eta_lo, keep (n,) bool); positions and delta are NaN where
    the crossing is outside [eta_lo, eta_hi)."""
    x = _f64(x_rel).reshape(-1, 3)
    v = _f64(xdot).reshape(-1, 3)
    o = _f64(origin).reshape(3)
    n = x.shape[0]
    pos = np.empty((n, 3), dtype=np.float64)
    delta = np.empty(n, dtype=np.float64)
    keep = np.empty(n, dtype=np.uint8)
    lib().oracle_cone_events(n, _p(x, ctypes.c_double), _p(v, ctypes.c_double),
                             _p(o, ctypes.c_double), float(eta0), float(eta_lo), float(eta_hi),
                             _p(pos, ctypes.c_double), _p(delta, ctypes.c_double),
                             _p(keep, ctypes.c_uint8))
    return pos, delta, keep.astype(bool)


def lambda_lm(lmax: int, m: int, z: float, s: float) -> np.ndarray:
    """Orthonormal associated Legendre functions lambda_lm(cos theta) for
    l = m .. lmax (Condon-Shortley phase), with z = cos theta, s = sin theta."""
    out = np.empty(lmax - m + 1, dtype=np.float64)
    lib().oracle_lambda_lm(lmax, m, float(z), float(s), _p(out, ctypes.c_double))
    return out


def alm_index(lmax: int, l: int, m: int) -> int:
    """Position of a_lm (0 <= m <= l <= lmax): m (2 lmax + 1 - m) / 2 + l."""
    return int(lib().oracle_alm_index(lmax, l, m))


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def map2alm(nside: int, lmax: int, hmap) -> np.ndarray:
    """a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(n_p)) (complex128, index
    alm_index), by direct summation over pixels."""
    m = _f64(hmap).ravel()
    if m.size != 12 * nside * nside:
        raise ValueError("map size does not match nside")
    re = np.empty(alm_size(lmax), dtype=np.float64)
    im = np.empty(alm_size(lmax), dtype=np.float64)
    lib().oracle_map2alm(nside, lmax, _p(m, ctypes.c_double), _p(re, ctypes.c_double),
                         _p(im, ctypes.c_double))
    return re + 1j * im


def alm2cl(lmax: int, alm) -> np.ndarray:
    """C_l = sum_{m=-l}^{l} |a_lm|^2 / (2l + 1) of a real map's a_lm (m >= 0 stored)."""
    a = np.asarray(alm, dtype=np.complex128)
    re = np.ascontiguousarray(a.real)
    im = np.ascontiguousarray(a.imag)
    cl = np.empty(lmax + 1, dtype=np.float64)
    lib().oracle_alm2cl(lmax, _p(re, ctypes.c_double), _p(im, ctypes.c_double),
                        _p(cl, ctypes.c_double))
    return cl


def map2alm_m(nside: int, lmax: int, m: int, hmap) -> np.ndarray:
    """a_lm for one m and l = m .. lmax (complex128), by the same direct sum
    as map2alm; single-threaded."""
    mp = _f64(hmap).ravel()
    re = np.empty(lmax - m + 1, dtype=np.float64)
    im = np.empty(lmax - m + 1, dtype=np.float64)
    lib().oracle_map2alm_m(nside, lmax, m, _p(mp, ctypes.c_double), _p(re, ctypes.c_double),
                           _p(im, ctypes.c_double))
    return re + 1j * im


def ang2pix(nside: int, vecs) -> np.ndarray:
    """HEALPix RING pixel of each direction (n,3) (any positive length)."""
    v = _f64(vecs).reshape(-1, 3)
    out = np.empty(v.shape[0], dtype=np.int64)
    lib().oracle_ang2pix_many(nside, v.shape[0], _p(v, ctypes.c_double), _p(out, ctypes.c_int64))
    return out


def quarter_turns(xy) -> np.ndarray:
    """Azimuth phi / (pi/2) in [0, 4) of directions (n, 2) by the fixed
    arctangent recipe that ang2pix uses."""
    v = _f64(xy).reshape(-1, 2)
    out = np.empty(v.shape[0], dtype=np.float64)
    lib().oracle_quarter_turns_many(v.shape[0], _p(v, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def place_segments(x_rel, xdot, xprime, rot, origin):
    """Segments of a rotated simulation box in the sky frame (Sec. II.C: a
    box is turned so that its photons travel towards the observer):
    P = origin + R x_rel, Xdot -> R Xdot, X' -> R X' (FP64; R row-major 3x3,
    box coordinates to sky coordinates)."""
    R = _f64(rot).reshape(3, 3)
    o = _f64(origin).reshape(3)

    def turn(a):
        # row k of R times a, summed left to right with separate roundings
        a = _f64(a).reshape(-1, 3)
        return np.stack([(R[k, 0] * a[:, 0] + R[k, 1] * a[:, 1]) + R[k, 2] * a[:, 2]
                         for k in range(3)], axis=1)

    return o[None, :] + turn(x_rel), turn(xdot), turn(xprime)


def in_cone(nside_c: int, cone: int, P) -> np.ndarray:
    """True where the position P lies inside the healpix cone `cone` of the
    Nside_c stacking grid (Sec. II.C: a box keeps only the strings inside
    its cone), i.e. where its direction falls in that RING pixel."""
    return ang2pix(nside_c, P) == cone


def cone_frame(nside_c: int, cone: int, axis: int, r_out: float, side: float):
    """Frame of a cubic box of side `side` placed in healpix cone `cone`
    (Sec. II.C, Fig. 1), as (R (3,3) box-to-sky, origin (3,)):
      * photons must travel towards the observer: box axis `axis` points out
        along the cone axis n (the pixel centre), photons moving along -axis;
      * the farthest pixel must fit in the farthest face: the far face
        x_axis = side is the plane n.P = r_out, centred on n;
      * the two other axes are (e_theta + e_phi)/sqrt(2) and
        (e_phi - e_theta)/sqrt(2) at n, in cyclic order after `axis`
        (right-handed), so the pixel's diamond lies across the face
        diagonals.  (The rotation about n is not fixed by the paper; this
        is the reading taken.)"""
    n = pix2vec(nside_c, [cone])[0]
    st = np.hypot(n[0], n[1])
    cp, sp = n[0] / st, n[1] / st
    e_th = np.array([n[2] * cp, n[2] * sp, -st])
    e_ph = np.array([-sp, cp, 0.0])
    e1 = (e_th + e_ph) / np.sqrt(2.0)
    e2 = (e_ph - e_th) / np.sqrt(2.0)
    R = np.empty((3, 3))
    R[:, axis] = n
    R[:, (axis + 1) % 3] = e1
    R[:, (axis + 2) % 3] = e2
    origin = (r_out - side) * n - 0.5 * side * (e1 + e2)
    return R, origin


def flat_theta(nx: int, ny: int, h: float, frame, accept_cos: float, eta0: float,
               boxes: Sequence) -> np.ndarray:
    """Flat-sky small-angle Theta/GU on an ny x nx patch (row-major, index
    j nx + i) of pixel size h (radians) around frame = (c, e1, e2) (rows of a
    3x3 array): the 2-D form of Eq. (1) with every photon path parallel to c
    (Sec. II.A, Fig. 3)."""
    fr = _f64(frame).reshape(3, 3)
    out = np.empty(ny * nx, dtype=np.float64)
    pk = _Packed(boxes)
    lib().oracle_flat_theta(nx, ny, float(h), _p(fr, ctypes.c_double), float(accept_cos),
                            float(eta0), *pk.args(), _p(out, ctypes.c_double))
    return out.reshape(ny, nx)


def flat_points(t, frame, accept_cos: float, eta0: float, boxes: Sequence) -> np.ndarray:
    """The flat-sky map of flat_theta at plane positions t (n, 2) in radians."""
    tt = _f64(t).reshape(-1, 2)
    fr = _f64(frame).reshape(3, 3)
    out = np.empty(tt.shape[0], dtype=np.float64)
    pk = _Packed(boxes)
    lib().oracle_flat_points(tt.shape[0], _p(tt, ctypes.c_double), _p(fr, ctypes.c_double),
                             float(accept_cos), float(eta0), *pk.args(), _p(out, ctypes.c_double))
    return out
