"""Seeded synthetic workloads for the string-ISW map maker.

This module only draws inputs: random string segments in boxes, box
placements, conformal-time slabs and visibility rules.  It contains none of
the map arithmetic and is shared, as plain input data, by the HIP library's
tests and benchmark and by the CPU oracle.

The paper's own light-cone data (Nambu-Goto simulations, Sec. II.B-C) is not
available, so segments are drawn independently in each box, with the gauge
conditions of Eq. (1) (transverse temporal gauge, Xdot.X' = 0) and the
conformal normalisation Xdot^2 + X'^2 = 1, i.e. eps = 1:

    x_rel  ~ U[0, side)^3                 (position inside the box)
    s_hat  ~ uniform on S^2               (string tangent direction)
    v_hat  ~ uniform in the plane _|_ s   (velocity direction)
    v      ~ U(0.2, 0.8)                   (speed)
    dsigma ~ U(0.001, 0.01)               (segment length parameter)
    Xdot = v v_hat,   X' = sqrt(1 - v^2) s_hat

drawn in that order from ``numpy.random.Generator(PCG64(seed))``.  Values are
then stored in the precision of the workload (float64 or float32); every
consumer reads the stored values.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

VIS_ALL, VIS_BOX, VIS_CAP = 0, 1, 2


@dataclasses.dataclass
class Box:
    origin: np.ndarray            # (3,) float64, observer-relative corner of the box
    ext: np.ndarray               # (3,) float64, box extent
    eta_lo: float                 # conformal-time slab [eta_lo, eta_hi)
    eta_hi: float
    x_rel: np.ndarray             # (n,3) position relative to origin
    xdot: np.ndarray              # (n,3)
    xprime: np.ndarray            # (n,3)
    dsigma: np.ndarray            # (n,)
    vis: int = VIS_ALL
    cap_dir: Optional[np.ndarray] = None   # (3,) unit vector for VIS_CAP
    cap_cos: Optional[float] = None        # cosine of the cap radius for VIS_CAP
    seed: Optional[int] = None

    @property
    def n(self) -> int:
        return int(self.dsigma.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    nside: int
    eta0: float
    boxes: list
    gu: float = 1e-7

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside


def _unit_rows(a: np.ndarray) -> np.ndarray:
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def segments(n: int, seed: int, dtype=np.float64, side: float = 1.0):
    """Draw n segments with the recipe in the module docstring."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 3)) * side
    s_hat = _unit_rows(rng.standard_normal((n, 3)))
    g = rng.standard_normal((n, 3))
    g = g - np.sum(g * s_hat, axis=1, keepdims=True) * s_hat
    v_hat = _unit_rows(g)
    v = rng.uniform(0.2, 0.8, n)
    ds = rng.uniform(0.001, 0.01, n)
    xdot = v[:, None] * v_hat
    xprime = np.sqrt(1.0 - v * v)[:, None] * s_hat
    cast = lambda a: np.ascontiguousarray(a.astype(dtype))
    return cast(x), cast(xdot), cast(xprime), cast(ds)


def near_luminal_segments(n: int, seed: int, speeds, v_dirs=None, dtype=np.float32,
                          side: float = 1.0):
    """Segments moving close to the speed of light (cusps of Nambu-Goto
    strings): the recipe above with the speed taken cyclically from
    `speeds` and, when given, the velocity direction from the unit rows of
    v_dirs (n, 3); the tangent is drawn uniformly in the plane normal to it,
    so Xdot.X' = 0 and Xdot^2 + X'^2 = 1 still hold."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 3)) * side
    if v_dirs is None:
        v_hat = _unit_rows(rng.standard_normal((n, 3)))
    else:
        v_hat = _unit_rows(np.asarray(v_dirs, dtype=np.float64).reshape(n, 3))
    g = rng.standard_normal((n, 3))
    g = g - np.sum(g * v_hat, axis=1, keepdims=True) * v_hat
    s_hat = _unit_rows(g)
    v = np.resize(np.asarray(speeds, dtype=np.float64), n)
    ds = rng.uniform(0.001, 0.01, n)
    xdot = v[:, None] * v_hat
    xprime = np.sqrt(1.0 - v * v)[:, None] * s_hat
    cast = lambda a: np.ascontiguousarray(a.astype(dtype))
    return cast(x), cast(xdot), cast(xprime), cast(ds)


def make_box(n: int, seed: int, origin, eta_lo: float, eta_hi: float, dtype=np.float64,
             side: float = 1.0, vis: int = VIS_ALL, cap_dir=None, cap_cos=None) -> Box:
    x, xd, xp, ds = segments(n, seed, dtype, side)
    return Box(origin=np.asarray(origin, dtype=np.float64), ext=np.full(3, float(side)),
               eta_lo=float(eta_lo), eta_hi=float(eta_hi), x_rel=x, xdot=xd, xprime=xp,
               dsigma=ds, vis=vis,
               cap_dir=None if cap_dir is None else np.asarray(cap_dir, dtype=np.float64),
               cap_cos=None if cap_cos is None else float(cap_cos), seed=seed)


def uniform_directions(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return _unit_rows(rng.standard_normal((n, 3)))


def sample_pixels(npix: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct pixel indices drawn uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, npix)
    return np.sort(rng.choice(npix, size=count, replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------
# The five benchmark workloads.  Geometry the paper leaves open is
# fixed here once (box placement, slabs, eta0) so every consumer agrees.
# ----------------------------------------------------------------------------

def config0() -> Workload:
    """Plain FP64: Nside=64, one unit box centred on the observer, 2,000
    segments (seed 0), eta0 = 1 and slab [0, 1) so every segment is kept."""
    box = make_box(2000, 0, origin=(-0.5, -0.5, -0.5), eta_lo=0.0, eta_hi=1.0,
                   dtype=np.float64)
    return Workload("config0: Nside=64, 1 box x 2,000 segments, FP64", 64, 1.0, [box], 1e-7)


def shell24_centres() -> np.ndarray:
    """The 24 integer points whose coordinates are a permutation of (0, +-1, +-2)."""
    pts = set()
    for a in (1, -1):
        for b in (2, -2):
            for perm in ((0, a, b), (0, b, a), (a, 0, b), (a, b, 0), (b, 0, a), (b, a, 0)):
                pts.add(perm)
    return np.array(sorted(pts), dtype=np.float64)


def config1(nseg: int = 100_000, nside: int = 512) -> Workload:
    """Plain vs FP32: Nside=512, 24 unit boxes tiling a shell at distance
    sqrt(5) (centres = permutations of (0, +-1, +-2)), 100,000 FP32 segments
    each (box b uses seed b+1), eta0 = 3 with slab [0.4, 1.1) (radii
    (1.9, 2.6]); a pixel sees a box when its ray crosses it within the slab."""
    boxes = []
    for b, c in enumerate(shell24_centres()):
        boxes.append(make_box(nseg, b + 1, origin=c - 0.5, eta_lo=0.4, eta_hi=1.1,
                              dtype=np.float32, vis=VIS_BOX))
    return Workload(f"config1: Nside={nside}, 24 shell boxes x {nseg:,} segments, FP32",
                    nside, 3.0, boxes, 1e-7)


def config2_geometry(nbox: int = 64):
    """Box origins for the Nside=2048 throughput workload: box b's nearest
    distance is r_b = 0.1 * 140^(b/63) Gpc along a direction drawn uniformly
    (seed 99); its centre sits at (r_b + sqrt(3)/2) d_b."""
    dirs = uniform_directions(64, 99)
    out = []
    for b in range(nbox):
        r = 0.1 * 140.0 ** (b / 63.0)
        centre = (r + math.sqrt(3.0) / 2.0) * dirs[b]
        out.append(centre - 0.5)
    return out


def config2_box(b: int, nseg: int = 400_000) -> Box:
    origin = config2_geometry()[b]
    return make_box(nseg, 100 + b, origin=origin, eta_lo=0.0, eta_hi=16.0, dtype=np.float32)


def config2(boxes=range(64), nseg: int = 400_000, nside: int = 2048) -> Workload:
    """FP32 throughput: Nside=2048, 64 boxes of side 1 Gpc at 0.1-14 Gpc,
    400,000 FP32 segments each (seeds 100-163), eta0 = 16 Gpc, slab [0, 16)
    (every segment kept), every pixel sees every box."""
    bl = [config2_box(b, nseg) for b in boxes]
    return Workload(f"config2: Nside={nside}, boxes {list(boxes)[:4]}... x {nseg:,} segments",
                    nside, 16.0, bl, 1e-7)


def config3_geometry(nbox: int = 256):
    rng = np.random.Generator(np.random.PCG64(399))
    g = rng.standard_normal(nbox)
    counts = np.clip(np.round(50_000 * np.exp(1.0 * g)), 1_000, 2_000_000).astype(np.int64)
    r = np.exp(rng.uniform(math.log(0.1), math.log(14.0), nbox))
    dirs = _unit_rows(rng.standard_normal((nbox, 3)))
    frac = np.exp(rng.uniform(math.log(0.001), math.log(0.05), nbox))
    return counts, r, dirs, frac


def config3(nbox: int = 256, nside: int = 4096, count_scale: float = 1.0) -> Workload:
    """Batched uneven: 256 boxes, lognormal segment counts (median 50,000,
    sigma 1, clipped to [1,000, 2,000,000]), distances log-uniform in
    [0.1, 14] Gpc, each box seen by a cap of sky fraction f_b log-uniform in
    [0.1%, 5%] around its direction (cos rho = 1 - 2 f_b); FP32 segments
    (seeds 400-655)."""
    counts, r, dirs, frac = config3_geometry(256)
    boxes = []
    for b in range(nbox):
        n = max(1, int(round(counts[b] * count_scale)))
        centre = (r[b] + math.sqrt(3.0) / 2.0) * dirs[b]
        boxes.append(make_box(n, 400 + b, origin=centre - 0.5, eta_lo=0.0, eta_hi=16.0,
                              dtype=np.float32, vis=VIS_CAP, cap_dir=dirs[b],
                              cap_cos=1.0 - 2.0 * frac[b]))
    return Workload(f"config3: Nside={nside}, {nbox} uneven boxes, FP32", nside, 16.0, boxes,
                    1e-7)


def config4(nseg: int = 50_000, nside: int = 1024, nbox: int = 8) -> Workload:
    """Differentiation: Nside=1024, 8 boxes x 50,000 FP32 segments (seeds
    200-207) at 1..8 Gpc along directions drawn with seed 208."""
    dirs = uniform_directions(8, 208)
    boxes = []
    for b in range(nbox):
        centre = (float(b + 1) + math.sqrt(3.0) / 2.0) * dirs[b]
        boxes.append(make_box(nseg, 200 + b, origin=centre - 0.5, eta_lo=0.0, eta_hi=16.0,
                              dtype=np.float32))
    return Workload(f"config4: Nside={nside}, {nbox} boxes x {nseg:,} segments", nside, 16.0,
                    boxes, 1e-7)


def config4_weights(npix: int) -> np.ndarray:
    """Gaussian pixel weights w_p of the loss L = sum_p w_p Theta_p^2 (seed 209)."""
    rng = np.random.Generator(np.random.PCG64(209))
    return rng.standard_normal(npix)


# ----------------------------------------------------------------------------
# Healpix-cone stacking (Sec. II.C, Fig. 1).  The paper's cosmology (Eq. (3)
# parameters) is not given, so the shell radii are fixed here with
# eta0 = 16 Gpc and eta(z) = eta0 / sqrt(1 + z) (matter era), rounded:
# z = 1089 -> r = 15.5, z = 36 -> r = 13.4, z = 0.2 -> r = 1.4 Gpc.  Box
# sides are round values for which the paper's grids are the coarsest that
# fit: Nside 16 for the high-redshift shell with 2.4 Gpc boxes, Nside 1 for
# the low-redshift shell with 16 Gpc boxes.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class StackPlan:
    """Which simulation run fills which healpix cone, and how."""
    name: str
    nside_c: int            # stacking grid
    r_in: float             # shell radii (observer-relative, Gpc)
    r_out: float
    side: float             # box side (Gpc)
    eta0: float
    seg_per_run: int
    run_seed0: int
    uses: list              # (cone pixel, run index, box axis facing the observer)

    @property
    def eta_lo(self) -> float:
        return self.eta0 - self.r_out

    @property
    def eta_hi(self) -> float:
        return self.eta0 - self.r_in

    @property
    def nruns(self) -> int:
        return 1 + max(u[1] for u in self.uses)

    def run(self, r: int, dtype=np.float32):
        """Segments of run r in box coordinates, inside [0, side)^3."""
        return segments(self.seg_per_run, self.run_seed0 + r, dtype, self.side)


def stack_highz(seg_per_run: int = 200_000) -> StackPlan:
    """3072 cones of the Nside 16 grid between z = 1089 and z = 36, filled by
    1024 runs used three times each (cone c: run c // 3, axis c % 3), FP32
    segments, run seeds 1000-2023."""
    uses = [(c, c // 3, c % 3) for c in range(12 * 16 * 16)]
    return StackPlan("high-z cones: Nside_c=16, 1024 runs x 3 axes", 16, 13.4, 15.5, 2.4, 16.0,
                     seg_per_run, 1000, uses)


def stack_lowz(seg_per_run: int = 200_000) -> StackPlan:
    """12 cones of the Nside 1 grid between z = 36 and z = 0.2, one run each
    (axis 2), FP32 segments, run seeds 3000-3011."""
    uses = [(c, c, 2) for c in range(12)]
    return StackPlan("low-z cones: Nside_c=1, 12 runs", 1, 1.4, 13.4, 16.0, 16.0, seg_per_run,
                     3000, uses)


# ----------------------------------------------------------------------------
# Flat-sky patch (Sec. III.B, Fig. 3: a 7.2 degree patch at the north pole).
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class FlatPatch:
    center: np.ndarray
    e1: np.ndarray
    e2: np.ndarray
    nx: int
    ny: int
    pix: float              # radians
    accept_cos: float
    eta0: float
    boxes: list

    @property
    def frame(self) -> np.ndarray:
        return np.stack([self.center, self.e1, self.e2])


def flat_pencil(nseg: int = 2_000_000, npix: int = 1024, seed: int = 800,
                dtype=np.float32) -> FlatPatch:
    """A 7.2 x 7.2 degree patch at the north pole (axes x, y), npix x npix
    pixels, and one box of nseg segments whose directions are uniform in the
    cap of radius 6 degrees around the pole (the patch's corners are 5.1
    degrees out) and whose radii are uniform in volume between 1.4 and
    15.5 Gpc (the stacked shells); eta0 = 16 Gpc, slab [0.5, 14.6).
    Velocities, tangents and dsigma follow the module recipe (seed), the
    positions are drawn with seed + 1."""
    x, xd, xp, ds = segments(nseg, seed, np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    rho = math.radians(6.0)
    cz = rng.uniform(math.cos(rho), 1.0, nseg)
    ph = rng.uniform(0.0, 2 * math.pi, nseg)
    r = np.cbrt(rng.uniform(1.4 ** 3, 15.5 ** 3, nseg))
    st = np.sqrt(1.0 - cz * cz)
    P = np.stack([st * np.cos(ph), st * np.sin(ph), cz], 1) * r[:, None]
    cast = lambda a: np.ascontiguousarray(a.astype(dtype))
    box = Box(origin=np.zeros(3), ext=np.full(3, 32.0), eta_lo=0.5, eta_hi=14.6, x_rel=cast(P),
              xdot=cast(xd), xprime=cast(xp), dsigma=cast(ds), seed=seed)
    return FlatPatch(center=np.array([0.0, 0.0, 1.0]), e1=np.array([1.0, 0.0, 0.0]),
                     e2=np.array([0.0, 1.0, 0.0]), nx=npix, ny=npix,
                     pix=math.radians(7.2) / npix, accept_cos=math.cos(rho), eta0=16.0,
                     boxes=[box])


def straight_strings(nstr: int = 40, seg_per: int = 3000, seed: int = 880,
                     cap_deg: float = 4.0, arc_deg: float = 12.0, dtype=np.float64) -> Box:
    """Long straight moving strings seen near the north pole, for comparing
    flat-sky and full-sky maps on coherent structures (Sec. III.B, Fig. 3):
    string k has its centre at a direction uniform in the cap of radius
    cap_deg and a distance uniform in [3, 15] Gpc, a tangent s uniform on
    S^2, a velocity direction uniform in s_perp and a speed U(0.2, 0.8); its
    seg_per segments (X' = s/gamma, Xdot = v v_hat, equal dsigma) span
    arc_deg of arc at that distance.  One box at the observer, slab
    [-100, 100) (every segment kept); values stored as `dtype`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P, V, T, DS = [], [], [], []
    for _ in range(nstr):
        th = math.radians(cap_deg) * math.sqrt(rng.uniform())
        ph = rng.uniform(0.0, 2 * math.pi)
        c = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        dist = rng.uniform(3.0, 15.0)
        sh = rng.standard_normal(3)
        sh /= np.linalg.norm(sh)
        g = rng.standard_normal(3)
        g -= (g @ sh) * sh
        vh = g / np.linalg.norm(g)
        v = rng.uniform(0.2, 0.8)
        gam = 1.0 / math.sqrt(1.0 - v * v)
        ds = dist * math.radians(arc_deg) * gam / seg_per
        sig = (np.arange(seg_per) + 0.5 - seg_per / 2) * ds
        P.append(dist * c[None, :] + (sig / gam)[:, None] * sh[None, :])
        V.append(np.tile(v * vh, (seg_per, 1)))
        T.append(np.tile(sh / gam, (seg_per, 1)))
        DS.append(np.full(seg_per, ds))
    cast = lambda a: np.ascontiguousarray(np.concatenate(a).astype(dtype))
    return Box(origin=np.zeros(3), ext=np.full(3, 32.0), eta_lo=-100.0, eta_hi=100.0,
               x_rel=cast(P), xdot=cast(V), xprime=cast(T), dsigma=cast(DS), seed=seed)
