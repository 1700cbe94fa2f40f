"""Pins of the oracle's light-cone event recording (the step before the sum,
Sec. II.B): a segment known at the slab start eta_lo moves on a straight
worldline P0 + Xdot (eta - eta_lo) and is recorded where that worldline
meets the past light cone |P| = eta0 - eta, if this happens inside the slab.
The oracle finds the crossing by bisection; these tests fix it against
closed forms (rest, radial and tangential motion), the defining identity
|P| = eta0 - eta at the event, exact slab edges, and a brute-force scan."""
import math

import mpmath
import numpy as np
import pytest

import oracle

EPS = np.finfo(np.float64).eps


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_segment_at_rest_crosses_at_its_distance():
    rng = np.random.default_rng(1)
    eta0, eta_lo, eta_hi = 16.0, 4.0, 9.0
    R0 = eta0 - eta_lo
    r = rng.uniform(R0 - 4.9, R0 - 0.1, 200)
    u = np.array([unit(x) for x in rng.standard_normal((200, 3))])
    x = r[:, None] * u
    pos, d, keep = oracle.cone_events(x, np.zeros_like(x), np.zeros(3), eta0, eta_lo, eta_hi)
    assert keep.all()
    exact = R0 - np.linalg.norm(x, axis=1)
    assert np.max(np.abs(d - exact)) <= 8 * EPS * R0
    assert np.array_equal(pos, x)


@pytest.mark.parametrize("v", [-0.9, -0.5, -0.1, 0.0, 0.3, 0.8, 0.99])
def test_radial_motion(v):
    """P0 = r0 u, Xdot = v u: |P0 + Xdot D| = |r0 + v D|, so
    D = (R0 - r0)/(1 + v) while the segment has not passed the observer, and
    D = (R0 + r0)/(1 - v) once it has (r0 + v D < 0)."""
    eta0, eta_lo, eta_hi = 14.0, 2.0, 12.0
    R0 = eta0 - eta_lo
    u = unit([0.3, -0.5, 0.8])
    for r0 in (3.0, 7.5, 11.9):
        D_exact = (R0 - r0) / (1.0 + v)
        if r0 + v * D_exact < 0:
            D_exact = (R0 + r0) / (1.0 - v)
        pos, d, keep = oracle.cone_events((r0 * u)[None], (v * u)[None], np.zeros(3), eta0,
                                          eta_lo, eta_hi)
        if D_exact < eta_hi - eta_lo:
            assert keep[0]
            assert abs(d[0] - D_exact) <= 16 * EPS * R0 / (1.0 - abs(v)), (r0, d[0], D_exact)
        else:
            assert not keep[0]


@pytest.mark.parametrize("v", [0.1, 0.5, 0.9])
def test_tangential_motion_against_high_precision(v):
    """P0 = r0 u, Xdot = v w with w perpendicular to u:
    (R0 - D)^2 = r0^2 + v^2 D^2, smaller root, evaluated with 50 digits."""
    mpmath.mp.dps = 50
    eta0, eta_lo, eta_hi = 10.0, 1.0, 9.0
    R0 = eta0 - eta_lo
    u = np.array([1.0, 0.0, 0.0])
    w = np.array([0.0, 0.6, 0.8])
    for r0 in (2.0, 5.25, 8.5):
        a = 1 - mpmath.mpf(v) ** 2
        R = mpmath.mpf(R0)
        D = (R - mpmath.sqrt(R * R - a * (R * R - mpmath.mpf(r0) ** 2))) / a
        pos, d, keep = oracle.cone_events((r0 * u)[None], (v * w)[None], np.zeros(3), eta0,
                                          eta_lo, eta_hi)
        assert keep[0]
        assert abs(d[0] - float(D)) <= 16 * EPS * R0 / (1 - v), (r0, d[0], float(D))


def test_event_lies_on_the_past_light_cone():
    rng = np.random.default_rng(7)
    n = 5000
    eta0, eta_lo, eta_hi = 16.0, 10.0, 11.0
    origin = np.array([5.1, -1.2, 0.7])
    x = rng.random((n, 3)) * 1.0
    vd = np.array([unit(t) for t in rng.standard_normal((n, 3))]) * rng.uniform(0.0, 0.95,
                                                                                  n)[:, None]
    pos, d, keep = oracle.cone_events(x, vd, origin, eta0, eta_lo, eta_hi)
    assert keep.any() and (~keep).any()
    k = keep
    # |P| = eta0 - eta with eta = eta_lo + D, to rounding of R0.
    R = np.linalg.norm(pos[k], axis=1)
    assert np.max(np.abs(R - (eta0 - eta_lo - d[k]))) <= 64 * EPS * (eta0 - eta_lo)
    # The event is on the worldline.
    P0 = origin + x
    assert np.allclose(pos[k], P0[k] + vd[k] * d[k][:, None], rtol=0, atol=1e-14)
    assert ((d[k] >= 0) & (d[k] < eta_hi - eta_lo)).all()
    assert np.isnan(d[~k]).all() and np.isnan(pos[~k]).all()


def test_exact_slab_edges_and_fast_segments():
    eta0, eta_lo, eta_hi = 16.0, 4.0, 6.0
    R0 = eta0 - eta_lo                        # 12
    x = np.array([[R0, 0.0, 0.0],             # at rest on the cone at eta_lo: kept, D = 0
                  [R0 - 2.0, 0.0, 0.0],       # crosses exactly at eta_hi: not kept
                  [R0 - 1.0, 0.0, 0.0],       # crosses at D = 1: kept
                  [R0 + 0.5, 0.0, 0.0],       # outside the cone already: no event
                  [5.0, 0.0, 0.0],            # |Xdot| = 1: no event
                  [5.0, 0.0, 0.0]])           # |Xdot| > 1: no event
    v = np.zeros_like(x)
    v[4] = [0.0, 1.0, 0.0]
    v[5] = [0.0, 0.0, 1.5]
    pos, d, keep = oracle.cone_events(x, v, np.zeros(3), eta0, eta_lo, eta_hi)
    assert keep.tolist() == [True, False, True, False, False, False]
    # to the rounding of h = |P| + D - R0 near R0
    assert abs(d[0]) <= 0.5 * np.spacing(R0) and abs(d[2] - 1.0) <= np.spacing(R0)


def test_brute_force_scan_of_the_gap_function():
    """The crossing is where |P0 + Xdot D| + D - R0 changes sign on a fine
    grid of D over the slab; kept iff it changes sign inside the slab."""
    rng = np.random.default_rng(11)
    n = 60
    eta0, eta_lo, eta_hi = 12.0, 6.0, 7.0
    R0, width = eta0 - eta_lo, eta_hi - eta_lo
    origin = np.array([-3.0, 2.0, 3.5])
    x = rng.random((n, 3)) * 1.2
    vd = np.array([unit(t) for t in rng.standard_normal((n, 3))]) * rng.uniform(0, 0.9, n)[:, None]
    pos, d, keep = oracle.cone_events(x, vd, origin, eta0, eta_lo, eta_hi)
    grid = np.linspace(0.0, width, 200_001)
    for i in range(n):
        P = origin + x[i]
        h = np.linalg.norm(P[None] + vd[i][None] * grid[:, None], axis=1) + grid - R0
        inside = h[0] <= 0 < h[-1]
        assert keep[i] == inside, i
        if inside:
            j = np.argmax(h > 0)
            assert grid[j - 1] - 1e-12 <= d[i] <= grid[j] + 1e-12
    assert keep.sum() > 5 and (~keep).sum() > 5
