"""More pins of the oracle against what the mathematics fixes.

* The dsigma derivative of Eq. (1): the sum is linear in each dsigma, so its
  derivative is the summand per unit dsigma, finite at dsigma = 0 and equal
  at every dsigma (central differences are exact up to rounding).
* Scale invariance (Sec. II.A, Eq. (1) is dimensionless): positions, slab,
  eta0 and dsigma multiplied by one factor leave the map unchanged; by a
  power of two, bit for bit.
* Mirror symmetry: reflecting every input vector in the plane z = 0 maps
  RING ring i onto ring 4 Nside - i at the same azimuth, and Eq. (1) (built
  from scalar products only) is unchanged there.
* Box placement (Sec. II.C): the frame of a cone box puts the far face on
  the plane n.P = r_out and the near face on n.P = r_out - side, centred on
  the cone axis, and turns vectors along the facing axis onto n; a
  transposed rotation fails these.
* Cap visibility: a pixel sees a cap box when its angle to the cap axis is
  at most the cap radius, decided against an independent angle formula.
* Absolute gradient sums: the triangle inequality against the gradient,
  equality for one pixel, additivity over pixels.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Box


def _box(x, xd, xp, ds, origin=(0.0, 0.0, 0.0), eta_lo=-1e9, eta_hi=1e9, vis=synth.VIS_ALL,
         ext=(1.0, 1.0, 1.0), cap_dir=None, cap_cos=None):
    return Box(origin=np.asarray(origin, float), ext=np.asarray(ext, float), eta_lo=eta_lo,
               eta_hi=eta_hi, x_rel=np.asarray(x, float).reshape(-1, 3),
               xdot=np.asarray(xd, float).reshape(-1, 3), xprime=np.asarray(xp, float).reshape(-1, 3),
               dsigma=np.asarray(ds, float).ravel(), vis=vis,
               cap_dir=None if cap_dir is None else np.asarray(cap_dir, float), cap_cos=cap_cos)


def _with(box, **kw):
    d = dict(vars(box))
    d.update(kw)
    return Box(**d)


def _segments_eps_not_one(n, seed):
    """Generated segments with X' rescaled by factors in [0.5, 1.5], so that
    eps = |X'|/sqrt(1 - Xdot^2) differs from 1 (a dropped eps shows)."""
    x, xd, xp, ds = synth.segments(n, seed, np.float64)
    f = np.random.default_rng(seed + 1000).uniform(0.5, 1.5, n)
    return x, xd, xp * f[:, None], ds


# ---------------------------------------------------------------------------
# dsigma derivative
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ds0", [0.0, 1e-300, 4e-3])
def test_dsigma_derivative_is_finite_and_matches_differences(ds0):
    nside = 4
    pix = np.arange(12 * nside * nside)
    x, xd, xp, ds = _segments_eps_not_one(6, 21)
    ds = ds.copy()
    ds[2] = ds0
    box = _box(x, xd, xp, ds, origin=(-0.5, -0.5, -0.5), eta_lo=0.0, eta_hi=2.0)
    eta0 = 2.0
    g = np.random.default_rng(5).standard_normal(len(pix))
    G = oracle.grad(nside, pix, g, eta0, [box], np.arange(6))
    assert np.all(np.isfinite(G))
    # L is linear in dsigma_2: the central difference is exact up to rounding.
    h = 1e-3
    vals = []
    for sgn in (1.0, -1.0):
        d2 = ds.copy()
        d2[2] = ds0 + sgn * h
        vals.append(np.dot(g, oracle.theta_pixels(nside, pix, eta0, [_with(box, dsigma=d2)])))
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(G[2, 9] - fd) <= 1e-10 * abs(fd), (G[2, 9], fd)
    # At dsigma = 0 every other component vanishes (each carries dsigma).
    if ds0 == 0.0:
        assert np.all(G[2, :9] == 0.0)
    # The derivative does not depend on dsigma: compare with dsigma = 1.
    d1 = ds.copy()
    d1[2] = 1.0
    G1 = oracle.grad(nside, pix, g, eta0, [_with(box, dsigma=d1)], np.array([2]))
    assert abs(G1[0, 9] - G[2, 9]) <= 1e-13 * abs(G1[0, 9])
    # and at dsigma = 1 it is the map sum of that segment alone.
    single = _box(x[2:3], xd[2:3], xp[2:3], [1.0], origin=box.origin, eta_lo=0.0, eta_hi=2.0)
    alone = np.dot(g, oracle.theta_pixels(nside, pix, eta0, [single]))
    assert abs(G1[0, 9] - alone) <= 1e-12 * abs(alone)


# ---------------------------------------------------------------------------
# Scale invariance and mirror symmetry
# ---------------------------------------------------------------------------

def _scaled(box, lam):
    return _box(box.x_rel * lam, box.xdot, box.xprime, box.dsigma * lam,
                origin=box.origin * lam, eta_lo=box.eta_lo * lam, eta_hi=box.eta_hi * lam,
                ext=box.ext * lam, vis=box.vis, cap_dir=box.cap_dir, cap_cos=box.cap_cos)


def _scale_workload():
    x, xd, xp, ds = _segments_eps_not_one(40, 31)
    b1 = _box(x[:20], xd[:20], xp[:20], ds[:20], origin=(-0.5, -0.5, -0.5), eta_lo=1.3,
              eta_hi=2.0)
    b2 = _box(x[20:], xd[20:], xp[20:], ds[20:], origin=(0.6, -0.9, 0.2), eta_lo=0.4,
              eta_hi=1.5, vis=synth.VIS_BOX)
    return [b1, b2], 2.0


def test_scale_invariance_power_of_two_is_bitwise():
    boxes, eta0 = _scale_workload()
    nside = 8
    pix = np.arange(12 * nside * nside)
    m = oracle.theta_pixels(nside, pix, eta0, boxes)
    assert np.count_nonzero(m) > len(pix) // 2
    for lam in (4.0, 0.125, 2.0 ** 40):
        ms = oracle.theta_pixels(nside, pix, eta0 * lam, [_scaled(b, lam) for b in boxes])
        assert np.array_equal(ms, m), lam


@pytest.mark.parametrize("lam", [3.0, 0.37, 1.7e4])
def test_scale_invariance_to_rounding(lam):
    boxes, eta0 = _scale_workload()
    nside = 8
    pix = np.arange(12 * nside * nside)
    m = oracle.theta_pixels(nside, pix, eta0, boxes)
    ms = oracle.theta_pixels(nside, pix, eta0 * lam, [_scaled(b, lam) for b in boxes])
    # Rounding of the scaled inputs can move an event across a slab edge or a
    # pixel across the box's ray test; none of these inputs sits that close.
    assert np.max(np.abs(ms - m)) <= 1e-12 * np.max(np.abs(m))


def _mirror_z(a):
    a = np.array(a, float, copy=True)
    a[..., 2] = -a[..., 2]
    return a


def test_mirror_in_the_equator_maps_ring_i_to_ring_4n_minus_i():
    nside = 8
    x, xd, xp, ds = _segments_eps_not_one(30, 41)
    origin = np.array([-0.3, -0.6, -0.45])
    ext = np.array([1.0, 1.0, 1.0])
    b = _box(x, xd, xp, ds, origin=origin, eta_lo=0.0, eta_hi=2.0, vis=synth.VIS_BOX, ext=ext)
    # The mirrored box has min corner z' = -(z0 + ext_z); its segments are
    # given relative to it, so x_rel_z' = ext_z - x_rel_z.
    om = _mirror_z(origin)
    om[2] -= ext[2]
    xm = np.array(x, copy=True)
    xm[:, 2] = ext[2] - x[:, 2]
    bm = _box(xm, _mirror_z(xd), _mirror_z(xp), ds, origin=om, eta_lo=0.0, eta_hi=2.0,
              vis=synth.VIS_BOX, ext=ext)
    pix = np.arange(12 * nside * nside)
    m = oracle.theta_pixels(nside, pix, 2.0, [b])
    mm = oracle.theta_pixels(nside, pix, 2.0, [bm])
    ring, pos = oracle.ring_of_pixel(nside, pix)
    start = {int(r): int(np.argmax(ring == r)) for r in np.unique(ring)}
    q = np.array([start[4 * nside - int(r)] + int(j) for r, j in zip(ring, pos)])
    # Mirrored pixel directions are exact negations of z.
    assert np.array_equal(oracle.pix2vec(nside, q), _mirror_z(oracle.pix2vec(nside, pix)))
    assert np.count_nonzero(m) > len(pix) // 4
    assert np.allclose(mm[q], m, rtol=0, atol=1e-12 * np.max(np.abs(m)))
    # It is not the identity: the map itself is not mirror symmetric.
    assert np.max(np.abs(m[q] - m)) > 1e-3 * np.max(np.abs(m))


# ---------------------------------------------------------------------------
# Box placement
# ---------------------------------------------------------------------------

def _corners(side):
    return np.array([[i, j, k] for i in (0.0, side) for j in (0.0, side) for k in (0.0, side)])


@pytest.mark.parametrize("nside,cone,axis", [(1, 0, 2), (1, 7, 0), (2, 21, 1), (16, 100, 0),
                                             (16, 3000, 2), (4, 95, 1)])
def test_placed_box_faces_lie_on_their_planes(nside, cone, axis):
    side, r_out = 2.4, 15.5
    R, origin = oracle.cone_frame(nside, cone, axis, r_out, side)
    n = oracle.pix2vec(nside, [cone])[0]
    c = _corners(side)
    zeros = np.zeros_like(c)
    P, V, T = oracle.place_segments(c, zeros, zeros, R, origin)
    far = c[:, axis] == side
    assert np.allclose(P[far] @ n, r_out, rtol=0, atol=1e-12 * r_out)
    assert np.allclose(P[~far] @ n, r_out - side, rtol=0, atol=1e-12 * r_out)
    # The far face's centre is the point r_out n.
    centre = np.full((1, 3), 0.5 * side)
    centre[0, axis] = side
    Pc, _, _ = oracle.place_segments(centre, zeros[:1], zeros[:1], R, origin)
    assert np.allclose(Pc[0], r_out * n, rtol=0, atol=1e-12 * r_out)
    # Distances between placed points equal those in the box (a rotation),
    # and vectors along the facing axis turn onto n.
    assert np.allclose(np.linalg.norm(P[:, None] - P[None], axis=2),
                       np.linalg.norm(c[:, None] - c[None], axis=2), atol=1e-12 * r_out)
    e = np.zeros((1, 3))
    e[0, axis] = 1.0
    _, Ve, Te = oracle.place_segments(zeros[:1], e, 0.5 * e, R, origin)
    assert np.allclose(Ve[0], n, atol=1e-15) and np.allclose(Te[0], 0.5 * n, atol=1e-15)
    # A transposed rotation (sky to box instead of box to sky) breaks the
    # face planes, so the test above would catch it.
    Pt, _, _ = oracle.place_segments(c, zeros, zeros, R.T, origin)
    assert np.max(np.abs(Pt[far] @ n - r_out)) > 1e-3 * side


def test_placement_is_the_linear_map_on_all_three_vectors():
    rng = np.random.default_rng(3)
    R, origin = oracle.cone_frame(16, 1234, 1, 15.5, 2.4)
    x = rng.random((50, 3)) * 2.4
    xd = rng.standard_normal((50, 3))
    xp = rng.standard_normal((50, 3))
    P, V, T = oracle.place_segments(x, xd, xp, R, origin)
    # column k of R is where box axis k goes
    for k in range(3):
        ek = np.zeros(3)
        ek[k] = 1.0
        Pk, Vk, _ = oracle.place_segments(ek[None], ek[None], ek[None], R, np.zeros(3))
        assert np.array_equal(Vk[0], R[:, k])
    lin = origin + x[:, 0:1] * R[:, 0] + x[:, 1:2] * R[:, 1] + x[:, 2:3] * R[:, 2]
    assert np.allclose(P, lin, rtol=0, atol=1e-14 * 20)
    assert np.allclose(V, xd[:, 0:1] * R[:, 0] + xd[:, 1:2] * R[:, 1] + xd[:, 2:3] * R[:, 2],
                       atol=1e-14)
    assert np.allclose(T, xp[:, 0:1] * R[:, 0] + xp[:, 1:2] * R[:, 1] + xp[:, 2:3] * R[:, 2],
                       atol=1e-14)
    # Dot products, hence Eq. (1), are preserved: Xdot.X' and norms.
    assert np.allclose(np.sum(V * T, 1), np.sum(xd * xp, 1), atol=1e-13)


# ---------------------------------------------------------------------------
# Cap visibility
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("frac", [0.001, 0.02, 0.3])
def test_cap_visibility_is_the_angular_disc(frac):
    nside = 64
    pix = np.arange(12 * nside * nside)
    rng = np.random.default_rng(int(frac * 1e4))
    c = rng.standard_normal(3)
    c /= np.linalg.norm(c)
    cap_cos = 1.0 - 2.0 * frac
    b = _box(np.zeros((1, 3)), np.zeros((1, 3)), np.ones((1, 3)), np.ones(1),
             vis=synth.VIS_CAP, cap_dir=c, cap_cos=cap_cos)
    vis = oracle.visible(nside, pix, 1.0, b)
    n = oracle.pix2vec(nside, pix)
    # Independent angle: atan2(|n x c|, n.c), accurate at every angle.
    ang = np.arctan2(np.linalg.norm(np.cross(n, c), axis=1), n @ c)
    rho = math.acos(cap_cos)
    clear = np.abs(ang - rho) > 1e-9
    assert np.array_equal(vis[clear], (ang <= rho)[clear])
    # The disc holds the cap's share of the sky up to its boundary pixels.
    pix_rad = math.sqrt(4 * math.pi / len(pix))
    boundary = 2 * math.pi * math.sin(rho) / pix_rad
    assert abs(vis.sum() - frac * len(pix)) <= 2 * boundary + 2
    # Only pixels of the cap enter the map of a cap box.
    x, xd, xp, ds = synth.segments(20, 17, np.float64)
    bb = _box(x, xd, xp, ds, origin=(-0.5, -0.5, -0.5), vis=synth.VIS_CAP, cap_dir=c,
              cap_cos=cap_cos)
    ball = _with(bb, vis=synth.VIS_ALL, cap_dir=None, cap_cos=None)
    mc = oracle.theta_pixels(nside, pix, 1.0, [bb])
    ma = oracle.theta_pixels(nside, pix, 1.0, [ball])
    assert np.array_equal(mc, np.where(vis, ma, 0.0))


# ---------------------------------------------------------------------------
# Absolute gradient sums (the scale a gradient's terms have before cancelling)
# ---------------------------------------------------------------------------

def test_absolute_gradient_sums():
    nside = 4
    pix = np.arange(12 * nside * nside)
    x, xd, xp, ds = _segments_eps_not_one(8, 51)
    box = _box(x, xd, xp, ds, origin=(-0.5, -0.5, -0.5), eta_lo=0.0, eta_hi=2.0)
    g = np.random.default_rng(8).standard_normal(len(pix))
    sel = np.arange(8)
    G = oracle.grad(nside, pix, g, 2.0, [box], sel)
    A = oracle.grad(nside, pix, g, 2.0, [box], sel, absolute=True)
    # triangle inequality, strict somewhere (terms of both signs cancel)
    assert np.all(A >= np.abs(G) * (1 - 1e-14))
    assert np.any(A > 1.5 * np.abs(G))
    # invariant under the cotangent's sign, linear in its magnitude
    assert np.allclose(oracle.grad(nside, pix, -2.0 * g, 2.0, [box], sel, absolute=True), 2 * A,
                       rtol=1e-14, atol=0)
    # one pixel: the absolute sum is the absolute gradient
    for p in (0, 77, 191):
        G1 = oracle.grad(nside, pix[p:p + 1], g[p:p + 1], 2.0, [box], sel)
        A1 = oracle.grad(nside, pix[p:p + 1], g[p:p + 1], 2.0, [box], sel, absolute=True)
        assert np.array_equal(A1, np.abs(G1))
    # and the sum over pixels of those
    A_parts = sum(oracle.grad(nside, pix[p:p + 1], g[p:p + 1], 2.0, [box], sel, absolute=True)
                  for p in range(len(pix)))
    assert np.allclose(A, A_parts, rtol=1e-13, atol=0)
