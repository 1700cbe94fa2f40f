"""ctypes binding of libcsmap (include/csmap.h).

Argument marshalling only: every step of the map computation runs in the HIP
library.  The functions ``csmap_*`` mirror the C entry points one to one;
:class:`Sky` is a small convenience wrapper that takes torch CUDA tensors
(PyTorch supplies device memory and the stream, nothing else).

Importing this module loads ``libcsmap.so`` built in-tree; it raises if the
library is missing.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsmap.so")

CSMAP_OK, CSMAP_E_INVALID, CSMAP_E_NOMEM, CSMAP_E_DEVICE, CSMAP_E_STATE, CSMAP_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
CSMAP_FORM_FP64, CSMAP_FORM_FP32C = 0, 1
CSMAP_F32, CSMAP_F64 = 0, 1
CSMAP_VIS_ALL, CSMAP_VIS_BOX, CSMAP_VIS_CAP = 0, 1, 2
(CSMAP_OPT_SCHEDULE, CSMAP_OPT_GRAPH, CSMAP_OPT_PIX_PER_LANE, CSMAP_OPT_WAVES, CSMAP_OPT_NEAR_W,
 CSMAP_OPT_CHUNK, CSMAP_OPT_ADJ_SPLIT, CSMAP_OPT_ACCUM, CSMAP_OPT_TILING, CSMAP_OPT_FAR_W,
 CSMAP_OPT_BLOCK_RINGS) = range(11)

_STATUS_NAMES = {0: "CSMAP_OK", -1: "CSMAP_E_INVALID", -2: "CSMAP_E_NOMEM", -3: "CSMAP_E_DEVICE",
                 -4: "CSMAP_E_STATE", -5: "CSMAP_E_UNSUPPORTED"}

EXPORTED = ["csmap_npix", "csmap_create_sky", "csmap_add_box", "csmap_add_snapshot_box",
            "csmap_cone_events", "csmap_map2alm", "csmap_alm2cl", "csmap_render", "csmap_backward", "csmap_reset",
            "csmap_destroy_sky", "csmap_last_error", "csmap_pix2vec_ring", "csmap_set_option",
            "csmap_get_stats", "csmap_autotune", "csmap_cap_tiles", "csmap_ring_block_rows",
            "csmap_cap_block_tiles", "csmap_add_cone_box", "csmap_precompute",
            "csmap_ang2pix_ring", "csmap_cone_place", "csmap_cone_min_nside",
            "csmap_render_flat", "csmap_render_dirs", "csmap_map2alm_noalloc",
            "csmap_valu_probe"]


class csmap_box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dtype", ctypes.c_int), ("x_rel", ctypes.c_void_p),
                ("xdot", ctypes.c_void_p), ("xprime", ctypes.c_void_p),
                ("dsigma", ctypes.c_void_p), ("origin", ctypes.c_double * 3),
                ("ext", ctypes.c_double * 3), ("eta_lo", ctypes.c_double),
                ("eta_hi", ctypes.c_double), ("vis", ctypes.c_int),
                ("cap_dir", ctypes.c_double * 3), ("cap_cos", ctypes.c_double)]


class csmap_cone(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int64), ("pix", ctypes.c_int64), ("rot", ctypes.c_double * 9)]


class csmap_patch(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double * 3), ("e1", ctypes.c_double * 3),
                ("e2", ctypes.c_double * 3), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("pix", ctypes.c_double), ("accept_cos", ctypes.c_double)]


class csmap_grad(ctypes.Structure):
    _fields_ = [("x_rel", ctypes.c_void_p), ("xdot", ctypes.c_void_p),
                ("xprime", ctypes.c_void_p), ("dsigma", ctypes.c_void_p)]


class csmap_stats(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int64), ("npix", ctypes.c_int64), ("nbox", ctypes.c_int64),
                ("segments", ctypes.c_int64), ("kept", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("near_steps", ctypes.c_int64), ("ms_precompute", ctypes.c_double),
                ("ms_forward", ctypes.c_double), ("ms_backward", ctypes.c_double),
                ("pix_per_lane", ctypes.c_int64), ("waves", ctypes.c_int64),
                ("schedule", ctypes.c_int64), ("graph", ctypes.c_int64), ("chunk", ctypes.c_int64),
                ("near_w", ctypes.c_double), ("tiling", ctypes.c_int64),
                ("mid_steps", ctypes.c_int64), ("far_w", ctypes.c_double),
                ("steps", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CsmapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libcsmap is not built ({path} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.csmap_npix.argtypes = [i64]
    lib.csmap_npix.restype = i64
    lib.csmap_create_sky.argtypes = [i64, dbl, i32, vp, ctypes.POINTER(vp)]
    lib.csmap_add_box.argtypes = [vp, ctypes.POINTER(csmap_box), ctypes.POINTER(i64)]
    lib.csmap_add_snapshot_box.argtypes = [vp, ctypes.POINTER(csmap_box), ctypes.POINTER(i64)]
    lib.csmap_cone_events.argtypes = [ctypes.POINTER(csmap_box), ctypes.c_double, vp, vp, vp, vp]
    lib.csmap_map2alm.argtypes = [i64, i64, vp, vp, vp]
    lib.csmap_map2alm_noalloc.argtypes = [i64, i64, vp, vp, vp]
    lib.csmap_valu_probe.argtypes = [i32, i64, i64, vp, vp, ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl)]
    lib.csmap_alm2cl.argtypes = [i64, vp, vp, vp]
    lib.csmap_render.argtypes = [vp, vp]
    lib.csmap_backward.argtypes = [vp, vp, ctypes.POINTER(csmap_grad), i64]
    lib.csmap_reset.argtypes = [vp]
    lib.csmap_destroy_sky.argtypes = [vp]
    lib.csmap_last_error.restype = ctypes.c_char_p
    lib.csmap_pix2vec_ring.argtypes = [i64, i64, i64, vp, vp]
    lib.csmap_set_option.argtypes = [vp, i32, dbl]
    lib.csmap_get_stats.argtypes = [vp, ctypes.POINTER(csmap_stats)]
    lib.csmap_autotune.argtypes = [vp, ctypes.c_char_p]
    lib.csmap_cap_tiles.argtypes = [i64, i64, dbl, dbl, dbl, dbl, ctypes.POINTER(i64), i64,
                                    ctypes.POINTER(i64)]
    lib.csmap_cap_block_tiles.argtypes = [i64, i64, i64, dbl, dbl, dbl, dbl, ctypes.POINTER(i64),
                                          i64, ctypes.POINTER(i64)]
    lib.csmap_ring_block_rows.argtypes = [i64, i64, i64, ctypes.POINTER(i64), i64,
                                          ctypes.POINTER(i64)]
    lib.csmap_add_cone_box.argtypes = [vp, ctypes.POINTER(csmap_box), ctypes.POINTER(csmap_cone),
                                       i32, ctypes.POINTER(i64)]
    lib.csmap_precompute.argtypes = [vp]
    lib.csmap_ang2pix_ring.argtypes = [i64, i64, vp, vp, vp]
    lib.csmap_cone_place.argtypes = [i64, i64, i32, dbl, dbl, dbl, ctypes.POINTER(csmap_cone),
                                     ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.csmap_cone_min_nside.argtypes = [dbl, dbl, dbl, ctypes.POINTER(i64)]
    lib.csmap_render_flat.argtypes = [vp, ctypes.POINTER(csmap_patch), vp]
    lib.csmap_render_dirs.argtypes = [vp, i64, vp, vp]
    for name in EXPORTED:
        if name not in ("csmap_npix", "csmap_last_error"):
            getattr(lib, name).restype = i32
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(status: int):
    if status != CSMAP_OK:
        raise CsmapError(status, lib().csmap_last_error().decode())


# ---- one-to-one wrappers of the C entry points -------------------------------

def csmap_npix(nside: int) -> int:
    return int(lib().csmap_npix(nside))


def csmap_create_sky(nside: int, eta0: float, form: int, stream: int | None) -> int:
    out = ctypes.c_void_p()
    _check(lib().csmap_create_sky(nside, eta0, form, stream or None, ctypes.byref(out)))
    return out.value


def csmap_add_box(sky: int, box: csmap_box) -> int:
    bid = ctypes.c_int64()
    _check(lib().csmap_add_box(sky, ctypes.byref(box), ctypes.byref(bid)))
    return bid.value


def csmap_add_snapshot_box(sky: int, box: csmap_box) -> int:
    bid = ctypes.c_int64()
    _check(lib().csmap_add_snapshot_box(sky, ctypes.byref(box), ctypes.byref(bid)))
    return bid.value


def csmap_add_cone_box(sky: int, box: csmap_box, cone: csmap_cone, snapshot: bool) -> int:
    bid = ctypes.c_int64()
    _check(lib().csmap_add_cone_box(sky, ctypes.byref(box), ctypes.byref(cone), int(bool(snapshot)),
                                    ctypes.byref(bid)))
    return bid.value


def csmap_precompute(sky: int):
    _check(lib().csmap_precompute(sky))


def csmap_cone_place(nside: int, pix: int, axis: int, r_in: float, r_out: float, side: float):
    """(cone, origin (3,), slack) of a box placed in a healpix cone."""
    cone = csmap_cone()
    origin = (ctypes.c_double * 3)()
    slack = ctypes.c_double()
    _check(lib().csmap_cone_place(nside, pix, axis, float(r_in), float(r_out), float(side),
                                  ctypes.byref(cone), origin, ctypes.byref(slack)))
    return cone, np.array(origin[:]), slack.value


def csmap_cone_min_nside(r_in: float, r_out: float, side: float) -> int:
    out = ctypes.c_int64()
    _check(lib().csmap_cone_min_nside(float(r_in), float(r_out), float(side), ctypes.byref(out)))
    return out.value


def csmap_cone_events(box: csmap_box, eta0: float, pos_ptr: int, delta_ptr: int, keep_ptr: int,
                      stream: int = 0):
    _check(lib().csmap_cone_events(ctypes.byref(box), float(eta0), pos_ptr, delta_ptr, keep_ptr,
                                   stream))


def csmap_render(sky: int, map_ptr: int):
    _check(lib().csmap_render(sky, map_ptr))


def csmap_backward(sky: int, dmap_ptr: int, grads: list):
    arr = (csmap_grad * max(len(grads), 1))(*grads)
    _check(lib().csmap_backward(sky, dmap_ptr, arr, len(grads)))


def csmap_reset(sky: int):
    _check(lib().csmap_reset(sky))


def csmap_destroy_sky(sky: int):
    _check(lib().csmap_destroy_sky(sky))


def csmap_last_error() -> str:
    return lib().csmap_last_error().decode()


def csmap_pix2vec_ring(nside: int, first: int, count: int, xyz_ptr: int, stream: int | None):
    _check(lib().csmap_pix2vec_ring(nside, first, count, xyz_ptr, stream or None))


def csmap_set_option(sky: int, opt: int, value: float):
    _check(lib().csmap_set_option(sky, opt, float(value)))


def csmap_get_stats(sky: int) -> dict:
    st = csmap_stats()
    _check(lib().csmap_get_stats(sky, ctypes.byref(st)))
    return st.as_dict()


def csmap_autotune(sky: int, cache_path: str | None):
    _check(lib().csmap_autotune(sky, cache_path.encode() if cache_path else None))


def csmap_cap_tiles(nside: int, tile: int, c, rho: float, max_ranges: int = 1 << 16):
    buf = (ctypes.c_int64 * (2 * max_ranges))()
    n = ctypes.c_int64()
    _check(lib().csmap_cap_tiles(nside, tile, float(c[0]), float(c[1]), float(c[2]), float(rho),
                                 buf, max_ranges, ctypes.byref(n)))
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]


def csmap_cap_block_tiles(nside: int, rings: int, width: int, c, rho: float,
                          max_ranges: int = 1 << 16):
    buf = (ctypes.c_int64 * (2 * max_ranges))()
    n = ctypes.c_int64()
    _check(lib().csmap_cap_block_tiles(nside, rings, width, float(c[0]), float(c[1]),
                                       float(c[2]), float(rho), buf, max_ranges, ctypes.byref(n)))
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]


ROW_COUNT_BITS = 10


def csmap_ring_block_rows(nside: int, rings: int, width: int):
    """Row table of the ring-block tiling as an (ntiles, rings) int64 numpy
    array of (first pixel << ROW_COUNT_BITS) | count entries."""
    import numpy as np
    n = ctypes.c_int64()
    st = lib().csmap_ring_block_rows(nside, rings, width, None, 0, ctypes.byref(n))
    if st != CSMAP_OK and n.value <= 0:
        _check(st)
    out = np.zeros((n.value, rings), dtype=np.int64)
    _check(lib().csmap_ring_block_rows(nside, rings, width,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       n.value, ctypes.byref(n)))
    return out


# ---- torch-facing convenience wrapper ---------------------------------------

def _torch():
    import torch
    return torch


def _dev_ptr(t) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Sky:
    """A HEALPix RING sky of Theta/GU owned by libcsmap.

    Segment tensors must be CUDA tensors of one dtype (float32 or float64):
    x_rel, xdot, xprime of shape (n, 3) and dsigma of shape (n,)."""

    def __init__(self, nside: int, eta0: float, form: int = CSMAP_FORM_FP32C, stream=None):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.nside = int(nside)
        self.npix = csmap_npix(self.nside)
        self.eta0 = float(eta0)
        self.form = form
        self.handle = csmap_create_sky(self.nside, self.eta0, form, self.stream.cuda_stream)
        self._keep = []           # tensors whose copy may still be in flight
        self.box_shapes = []
        self.box_dtypes = []

    def add_box(self, x_rel, xdot, xprime, dsigma, origin, eta_lo, eta_hi,
                vis=CSMAP_VIS_ALL, ext=(1.0, 1.0, 1.0), cap_dir=(0.0, 0.0, 1.0), cap_cos=-1.0,
                snapshot=False, cone=None):
        """Add a box of light-cone events (csmap_add_box), or with
        snapshot=True a box of segments at the slab start whose light-cone
        crossings the library records (csmap_add_snapshot_box).  With a
        `cone` (a csmap_cone, e.g. from cone_place) the arrays are in box
        coordinates and the box is a stacked simulation placed in that
        healpix cone (csmap_add_cone_box)."""
        torch = _torch()
        dt = x_rel.dtype
        if dt not in (torch.float32, torch.float64):
            raise TypeError("segment tensors must be float32 or float64")
        n = int(dsigma.shape[0])
        for t, shape in ((x_rel, (n, 3)), (xdot, (n, 3)), (xprime, (n, 3)), (dsigma, (n,))):
            if tuple(t.shape) != shape or t.dtype != dt:
                raise ValueError("segment tensors must share a dtype with shapes (n,3)x3 and (n,)")
        b = csmap_box()
        b.n = n
        b.dtype = CSMAP_F32 if dt == torch.float32 else CSMAP_F64
        if n:
            b.x_rel, b.xdot, b.xprime, b.dsigma = (_dev_ptr(x_rel), _dev_ptr(xdot),
                                                   _dev_ptr(xprime), _dev_ptr(dsigma))
        b.origin = (ctypes.c_double * 3)(*[float(v) for v in origin])
        b.ext = (ctypes.c_double * 3)(*[float(v) for v in ext])
        b.eta_lo, b.eta_hi = float(eta_lo), float(eta_hi)
        b.vis = int(vis)
        b.cap_dir = (ctypes.c_double * 3)(*[float(v) for v in cap_dir])
        b.cap_cos = float(cap_cos)
        if cone is not None:
            bid = csmap_add_cone_box(self.handle, b, cone, snapshot)
        else:
            bid = (csmap_add_snapshot_box if snapshot else csmap_add_box)(self.handle, b)
        self._keep.append((x_rel, xdot, xprime, dsigma))
        self.box_shapes.append(n)
        self.box_dtypes.append(dt)
        return bid

    def render(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.npix, dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or out.numel() != self.npix:
            raise ValueError("map must be a float64 tensor of npix elements")
        csmap_render(self.handle, _dev_ptr(out))
        return out

    def backward(self, dmap, grads=None):
        """dL/d(x_rel, xdot, xprime, dsigma) of every box (float64 tensors)."""
        torch = _torch()
        if dmap.dtype != torch.float64 or dmap.numel() != self.npix:
            raise ValueError("dmap must be a float64 tensor of npix elements")
        if grads is None:
            grads = []
            for n in self.box_shapes:
                grads.append(tuple(torch.empty(s, dtype=torch.float64, device="cuda")
                                   for s in ((n, 3), (n, 3), (n, 3), (n,))))
        gs = []
        for g in grads:
            gs.append(csmap_grad(*[(_dev_ptr(t) if t is not None and t.numel() else None)
                                   for t in g]))
        csmap_backward(self.handle, _dev_ptr(dmap.contiguous()), gs)
        return grads

    def render_flat(self, center, e1, e2, nx: int, ny: int, pix: float,
                    accept_cos: float, out=None):
        """Flat-sky small-angle map on a gnomonic patch (csmap_render_flat):
        a float64 CUDA tensor of shape (ny, nx).  accept_cos is the cosine of
        the acceptance cone around the patch axis, in (0, 1]."""
        torch = _torch()
        if out is None:
            out = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or out.numel() != nx * ny:
            raise ValueError("map must be a float64 tensor of nx * ny elements")
        p = csmap_patch()
        p.center = (ctypes.c_double * 3)(*[float(v) for v in center])
        p.e1 = (ctypes.c_double * 3)(*[float(v) for v in e1])
        p.e2 = (ctypes.c_double * 3)(*[float(v) for v in e2])
        p.nx, p.ny, p.pix, p.accept_cos = int(nx), int(ny), float(pix), float(accept_cos)
        _check(lib().csmap_render_flat(self.handle, ctypes.byref(p), _dev_ptr(out)))
        return out

    def render_dirs(self, xyz, out=None):
        """Theta/GU at arbitrary directions (csmap_render_dirs): xyz is an
        (n, 3) float64 CUDA tensor; returns an (n,) float64 tensor."""
        torch = _torch()
        if xyz.dtype != torch.float64 or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must be a float64 tensor of shape (n, 3)")
        xyz = xyz.contiguous()
        n = int(xyz.shape[0])
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or out.numel() != n:
            raise ValueError("out must be a float64 tensor of n elements")
        _check(lib().csmap_render_dirs(self.handle, n, _dev_ptr(xyz) if n else None,
                                       _dev_ptr(out) if n else None))
        return out

    def precompute(self):
        """Run the light-cone stage alone (csmap_precompute)."""
        csmap_precompute(self.handle)

    def set_option(self, opt, value):
        csmap_set_option(self.handle, opt, value)

    def stats(self) -> dict:
        return csmap_get_stats(self.handle)

    def autotune(self, cache_path=None):
        csmap_autotune(self.handle, cache_path)

    def reset(self):
        csmap_reset(self.handle)
        self._keep.clear()
        self.box_shapes.clear()
        self.box_dtypes.clear()

    def synchronize(self):
        self.stream.synchronize()
        self._keep.clear()

    def close(self):
        if self.handle:
            csmap_destroy_sky(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cone_events(x_rel, xdot, origin, eta0: float, eta_lo: float, eta_hi: float, stream=None):
    """Light-cone events of slab-start segments (csmap_cone_events): returns
    (pos (n,3) float64, delta (n,) float64, keep (n,) bool) CUDA tensors."""
    torch = _torch()
    n = int(x_rel.shape[0])
    if x_rel.dtype not in (torch.float32, torch.float64) or xdot.dtype != x_rel.dtype:
        raise TypeError("x_rel and xdot must share a float32 or float64 dtype")
    if tuple(x_rel.shape) != (n, 3) or tuple(xdot.shape) != (n, 3):
        raise ValueError("x_rel and xdot must have shape (n, 3)")
    pos = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    delta = torch.empty(n, dtype=torch.float64, device="cuda")
    keep = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = csmap_box()
    b.n = n
    b.dtype = CSMAP_F32 if x_rel.dtype == torch.float32 else CSMAP_F64
    if n:
        b.x_rel, b.xdot = _dev_ptr(x_rel), _dev_ptr(xdot)
    b.origin = (ctypes.c_double * 3)(*[float(v) for v in origin])
    b.eta_lo, b.eta_hi = float(eta_lo), float(eta_hi)
    st = stream if stream is not None else torch.cuda.current_stream()
    csmap_cone_events(b, eta0, pos.data_ptr() if n else None, delta.data_ptr() if n else None,
                      keep.data_ptr() if n else None, st.cuda_stream)
    return pos, delta, keep.view(torch.bool)


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def map2alm(hmap, lmax: int, stream=None):
    """a_lm of a RING map (csmap_map2alm) as a complex128 CUDA tensor of
    alm_size(lmax) entries, a_lm at m (2 lmax + 1 - m) / 2 + l.  Enqueued on
    `stream` (default: the current stream) without synchronising."""
    torch = _torch()
    npix = int(hmap.numel())
    nside = int(round((npix / 12) ** 0.5))
    if 12 * nside * nside != npix or hmap.dtype != torch.float64:
        raise ValueError("map must be a float64 tensor of 12 Nside^2 pixels")
    alm = torch.empty(2 * alm_size(lmax), dtype=torch.float64, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    src = hmap.contiguous()
    _check(lib().csmap_map2alm(nside, lmax, _dev_ptr(src), _dev_ptr(alm), st.cuda_stream))
    # The work reads `src` and writes `alm` after this returns: tell torch's
    # allocator that both are in use on `st`.
    src.record_stream(st)
    alm.record_stream(st)
    return torch.view_as_complex(alm.view(-1, 2))


def map2alm_noalloc(hmap, lmax: int, alm, stream=None):
    """csmap_map2alm_noalloc into a caller-owned float64 CUDA tensor `alm` of
    2 alm_size(lmax) entries (real and imaginary parts interleaved); the
    library allocates nothing.  Enqueued on `stream` without synchronising."""
    torch = _torch()
    npix = int(hmap.numel())
    nside = int(round((npix / 12) ** 0.5))
    if 12 * nside * nside != npix or hmap.dtype != torch.float64 or not hmap.is_contiguous():
        raise ValueError("map must be a contiguous float64 tensor of 12 Nside^2 pixels")
    if alm.dtype != torch.float64 or alm.numel() != 2 * alm_size(lmax) or not alm.is_contiguous():
        raise ValueError("alm must be a contiguous float64 tensor of 2 alm_size(lmax) entries")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().csmap_map2alm_noalloc(nside, lmax, _dev_ptr(hmap), _dev_ptr(alm),
                                       st.cuda_stream))
    return alm


def valu_probe(kind: int, blocks: int, iters: int, stream=None):
    """csmap_valu_probe: (kernel ms, FMA instructions per wavefront count) of
    a launch of known FMA work: FP32 (kind 0), FP64 (kind 1), FP32 with a
    scalar-register multiplier (kind 2)."""
    torch = _torch()
    out = torch.empty(int(blocks) * 256, dtype=torch.float64 if kind == 1 else torch.float32,
                      device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    ms, n = ctypes.c_double(), ctypes.c_double()
    _check(lib().csmap_valu_probe(int(kind), int(blocks), int(iters), _dev_ptr(out),
                                  st.cuda_stream, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def alm2cl(alm, lmax: int, stream=None):
    """C_l, l = 0 .. lmax, of a real map's a_lm (csmap_alm2cl), float64 CUDA tensor."""
    torch = _torch()
    a = torch.view_as_real(alm).contiguous().view(-1)
    if a.numel() != 2 * alm_size(lmax):
        raise ValueError("alm size does not match lmax")
    cl = torch.empty(lmax + 1, dtype=torch.float64, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().csmap_alm2cl(lmax, _dev_ptr(a), _dev_ptr(cl), st.cuda_stream))
    return cl


def pix2vec_ring(nside: int, first: int = 0, count: int | None = None):
    """Pixel-centre unit vectors from the device routine (float64, (count, 3))."""
    torch = _torch()
    npix = csmap_npix(nside)
    if count is None:
        count = npix - first
    out = torch.empty((count, 3), dtype=torch.float64, device="cuda")
    csmap_pix2vec_ring(nside, first, count, _dev_ptr(out), torch.cuda.current_stream().cuda_stream)
    return out


def cone_place(nside: int, pix: int, axis: int, r_in: float, r_out: float, side: float):
    """Placement of a box of side `side` in healpix cone `pix` of the Nside
    stacking grid (csmap_cone_place): (cone, origin, slack), cone a
    csmap_cone for Sky.add_box, origin a (3,) array; slack >= 0 iff the
    truncated cone r_in .. r_out fits in the box."""
    return csmap_cone_place(nside, pix, axis, r_in, r_out, side)


def cone_rot(cone) -> np.ndarray:
    """The rotation of a csmap_cone as a (3, 3) array."""
    return np.array(cone.rot[:]).reshape(3, 3)


def make_cone(nside: int, pix: int, rot) -> csmap_cone:
    c = csmap_cone()
    c.nside, c.pix = int(nside), int(pix)
    c.rot = (ctypes.c_double * 9)(*[float(v) for v in np.asarray(rot, dtype=np.float64).ravel()])
    return c


def cone_min_nside(r_in: float, r_out: float, side: float) -> int:
    return csmap_cone_min_nside(r_in, r_out, side)


def ang2pix_ring(nside: int, xyz):
    """RING pixels (int64 CUDA tensor) of the directions xyz ((n, 3) float64
    CUDA tensor) from the device routine (csmap_ang2pix_ring)."""
    torch = _torch()
    if xyz.dtype != torch.float64 or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must be a float64 tensor of shape (n, 3)")
    xyz = xyz.contiguous()
    n = int(xyz.shape[0])
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    _check(lib().csmap_ang2pix_ring(nside, n, _dev_ptr(xyz) if n else None,
                                    _dev_ptr(out) if n else None,
                                    torch.cuda.current_stream().cuda_stream))
    return out
