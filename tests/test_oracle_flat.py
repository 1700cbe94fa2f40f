"""Pins of the oracle's flat-sky small-angle map (Sec. II.A: the limit
X n -> X with parallel photon paths; Sec. III.B, Fig. 3).

* Kaiser-Stebbins step: a long straight string at one depth, moving with
  any velocity, makes the flat map jump by 8 pi gamma v c.(v_hat x s_hat)
  across its image (the line integral of the 2-D Lorentzian kernel).
* Small-angle limit of the full-sky oracle: for a compact group of segments
  near the axis the flat map and Eq. (1) at the gnomonic directions agree to
  O(theta), the difference shrinking linearly with the group's angular size.
* Grid layout: a segment at the patch centre moving along e1 gives a map
  odd under i -> nx-1-i and even under j -> ny-1-j; along e2, the reverse.
* Selection: the slab test and the acceptance cone decide which segments
  enter; the map is linear in the segment set."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Box


def box_of(P, V, T, ds, eta_lo=-1e9, eta_hi=1e9):
    return Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=eta_lo, eta_hi=eta_hi,
               x_rel=np.asarray(P, float).reshape(-1, 3), xdot=np.asarray(V, float).reshape(-1, 3),
               xprime=np.asarray(T, float).reshape(-1, 3), dsigma=np.asarray(ds, float).ravel())


def frame_z():
    return np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


def probe(nx, ny, h, fr, boxes, eta0=100.0, accept=-1.0):
    return oracle.flat_theta(nx, ny, h, fr, accept, eta0, boxes)


@pytest.mark.parametrize("phi_s,v_dir,v", [(0.3, (0.2, 0.9, 0.3), 0.5),
                                           (1.1, (-0.7, 0.1, -0.6), 0.8),
                                           (2.0, (0.0, 0.0, 1.0), 0.6)])
def test_kaiser_stebbins_step_flat(phi_s, v_dir, v):
    """String through the patch centre at depth D = 2 along
    s = (cos phi_s, sin phi_s, 0); a 1-pixel-wide 2 x 1 patch straddles it
    at distance +-d along the image normal c x s; Richardson in d."""
    c = np.array([0.0, 0.0, 1.0])
    s_hat = np.array([math.cos(phi_s), math.sin(phi_s), 0.0])
    v_hat = np.asarray(v_dir, float)
    v_hat /= np.linalg.norm(v_hat)
    gamma = 1 / math.sqrt(1 - v * v)
    D, dsig = 2.0, 2e-4
    sig = np.arange(-4.0, 4.0 + dsig / 2, dsig)
    sig -= 0.5 * (sig[0] + sig[-1])
    P = D * c[None, :] + (sig / gamma)[:, None] * s_hat[None, :]
    n = len(sig)
    bx = box_of(P, np.tile(v * v_hat, (n, 1)), np.tile(s_hat / gamma, (n, 1)), np.full(n, dsig))
    nrm = np.cross(c, s_hat)
    # frame whose e1 is the image normal: pixel i = 0, 1 at t = -h/2, +h/2 along e1
    fr = np.stack([c, nrm, s_hat])

    def step(d):
        m = probe(2, 1, 2 * d, fr, [bx])
        return m[0, 1] - m[0, 0]

    d = 2e-3
    s1, s2, s4 = step(d), step(d / 2), step(d / 4)
    r1, r2 = 2 * s2 - s1, 2 * s4 - s2
    rich = (4 * r2 - r1) / 3
    expected = 8 * math.pi * gamma * v * float(c @ np.cross(v_hat, s_hat))
    if abs(expected) < 1e-12:
        assert abs(rich) < 1e-6
    else:
        assert abs(rich - expected) <= 1e-4 * abs(expected), (rich, expected)


@pytest.mark.parametrize("size", [1e-2, 1e-3])
def test_small_angle_limit_of_full_sky(size):
    """Segments in a box of width `size` at distance 10 on the z axis;
    pixels of a 24 x 24 patch spanning 4 box widths: the flat map agrees with
    the full-sky oracle at the gnomonic pixel directions to O(size/10)."""
    x, xd, xp, ds = synth.segments(30, 5, np.float64, side=size)
    P = x + np.array([-size / 2, -size / 2, 10.0])
    bx = box_of(P, xd, xp, ds)
    nx = 24
    h = 4 * size / 10 / nx
    fr = frame_z()
    flat = probe(nx, nx, h, fr, [bx])
    t = (np.arange(nx) + 0.5 - nx / 2) * h
    tx, ty = np.meshgrid(t, t)
    dirs = np.stack([tx.ravel(), ty.ravel(), np.ones(nx * nx)], 1)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    full = oracle.theta_dirs(dirs, 100.0, [bx]).reshape(nx, nx)
    rel = np.max(np.abs(full - flat)) / np.max(np.abs(full))
    assert rel < 3 * size / 10 + 1e-9, rel
    assert rel > 1e-3 * size / 10      # not identical: the two forms differ at O(theta)


def test_limit_difference_shrinks_linearly():
    def diff(size):
        x, xd, xp, ds = synth.segments(30, 6, np.float64, side=size)
        P = x + np.array([-size / 2, -size / 2, 10.0])
        bx = box_of(P, xd, xp, ds)
        nx, h = 16, 3 * size / 10 / 16
        flat = probe(nx, nx, h, frame_z(), [bx])
        t = (np.arange(nx) + 0.5 - nx / 2) * h
        tx, ty = np.meshgrid(t, t)
        dirs = np.stack([tx.ravel(), ty.ravel(), np.ones(nx * nx)], 1)
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        full = oracle.theta_dirs(dirs, 100.0, [bx]).reshape(nx, nx)
        return np.max(np.abs(full - flat)) / np.max(np.abs(full))
    d1, d2 = diff(4e-2), diff(4e-3)
    assert 4 < d1 / d2 < 25, (d1, d2)


def test_grid_orientation_and_centre():
    V = np.array([[0.6, 0.0, 0.0]])
    T = np.array([[0.0, 0.0, 0.8]])
    for nx, ny in ((8, 6), (7, 5)):
        # segment on the axis at depth 3: the patch centre
        bx = box_of([[0.0, 0.0, 3.0]], V, T, [0.01])
        m = probe(nx, ny, 1e-3, frame_z(), [bx])
        np.testing.assert_allclose(m, -m[:, ::-1], rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(m, m[::-1, :], rtol=1e-13)
        assert m[0, -1] < 0 < m[0, 0]          # -u.(t - s): u along +e1
        bx2 = box_of([[0.0, 0.0, 3.0]], [[0.0, 0.6, 0.0]], T, [0.01])
        m2 = probe(nx, ny, 1e-3, frame_z(), [bx2])
        np.testing.assert_allclose(m2, -m2[::-1, :], rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(m2, m2[:, ::-1], rtol=1e-13)
        if nx % 2 == 1 and ny % 2 == 1:
            # the centre pixel sits on the segment: it receives 0
            assert m[ny // 2, nx // 2] == 0.0


def test_selection_and_linearity():
    x, xd, xp, ds = synth.segments(200, 9, np.float64, side=0.4)
    P = x + np.array([-0.2, -0.2, 3.0])
    a = box_of(P[:100], xd[:100], xp[:100], ds[:100])
    b = box_of(P[100:], xd[100:], xp[100:], ds[100:])
    fr = frame_z()
    ma = probe(12, 10, 2e-2, fr, [a])
    mb = probe(12, 10, 2e-2, fr, [b])
    mab = probe(12, 10, 2e-2, fr, [a, b])
    np.testing.assert_allclose(mab, ma + mb, rtol=1e-12, atol=1e-12 * np.max(np.abs(mab)))
    # slab: eta0 = 10, radii in (6.9, 7.1] only -> nothing here (radii ~3)
    empty = oracle.flat_theta(12, 10, 2e-2, fr, -1.0, 10.0,
                              [box_of(P, xd, xp, ds, eta_lo=2.9, eta_hi=3.1)])
    assert np.all(empty == 0.0)
    # acceptance cone: a box far off axis is excluded, one on axis kept
    off = box_of(P + np.array([5.0, 0.0, 0.0]), xd, xp, ds)
    m_off = oracle.flat_theta(12, 10, 2e-2, fr, math.cos(0.5), 100.0, [a, off])
    np.testing.assert_array_equal(m_off, ma)
    # segments behind the observer never enter, even with accept_cos = -1
    behind = box_of(P * np.array([1.0, 1.0, -1.0]), xd, xp, ds)
    np.testing.assert_array_equal(oracle.flat_theta(12, 10, 2e-2, fr, -1.0, 100.0, [a, behind]),
                                  ma)


def test_points_agree_with_the_grid():
    x, xd, xp, ds = synth.segments(300, 12, np.float64, side=0.5)
    bx = box_of(x + np.array([-0.25, -0.25, 4.0]), xd, xp, ds)
    nx, ny, h = 9, 7, 0.01
    g = oracle.flat_theta(nx, ny, h, frame_z(), -1.0, 100.0, [bx])
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    t = np.stack([(ii.ravel() + 0.5 - nx / 2) * h, (jj.ravel() + 0.5 - ny / 2) * h], 1)
    p = oracle.flat_points(t, frame_z(), -1.0, 100.0, [bx]).reshape(ny, nx)
    np.testing.assert_array_equal(p, g)
