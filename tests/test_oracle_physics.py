"""Pins of the oracle's Eq. (1)-(2) sum against results the physics fixes.

* Kaiser-Stebbins step: across the image of a long straight moving string
  Eq. (1) must jump by 8 pi GU gamma v n.(v_hat x s_hat) (closed form
  obtained from Eq. (1)-(2) by integrating the Lorentzian along the string;
  it holds for every orientation of n relative to s_hat and v_hat).
* Flat-sky limit (the paper's Sec. II.A: X n -> X, parallel photon paths):
  for a small distant box, the full-sky sum tends to the 2-D form.
* Brute-force quadrature of Eq. (1) along a circular loop: the segment sum is
  the periodic trapezoid rule of the integral.
* Linearity in dsigma, superposition of segments and boxes (the paper adds
  full-sky maps of subsets of cones, Sec. III.A), segment-order invariance,
  rotation covariance, and the exact-coincidence rule (q = 0 contributes 0).
* The gradient against central finite differences of the forward sum.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from synth import Box


def _box(x, xd, xp, ds, origin=(0.0, 0.0, 0.0), eta_lo=-1e9, eta_hi=1e9, vis=synth.VIS_ALL,
         ext=(1.0, 1.0, 1.0), cap_dir=None, cap_cos=None):
    return Box(origin=np.asarray(origin, float), ext=np.asarray(ext, float), eta_lo=eta_lo,
               eta_hi=eta_hi, x_rel=np.asarray(x, float).reshape(-1, 3),
               xdot=np.asarray(xd, float).reshape(-1, 3), xprime=np.asarray(xp, float).reshape(-1, 3),
               dsigma=np.asarray(ds, float).ravel(), vis=vis, cap_dir=cap_dir, cap_cos=cap_cos)


def _orthonormal(seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return q[:, 0], q[:, 1], q[:, 2]


def straight_string_on_light_cone(n0, s_hat, v_hat, v, dist, eta0, half_len, dsig):
    """Segments of X(sigma, tau) = X0 + sigma s_hat/gamma + tau v v_hat
    (Xdot.X' = 0, Xdot^2 + X'^2 = 1) at the events where |X| = eta0 - tau,
    with the sigma = 0 event at distance `dist` along n0."""
    gamma = 1.0 / math.sqrt(1.0 - v * v)
    tau0 = eta0 - dist
    B = v * v_hat
    X0 = dist * n0 - tau0 * B
    sig = np.arange(-half_len, half_len + 0.5 * dsig, dsig)
    sig = sig - 0.5 * (sig[0] + sig[-1])           # symmetric about 0
    A = X0[None, :] + sig[:, None] * (s_hat / gamma)[None, :]
    # (v^2 - 1) tau^2 + 2 (A.B + eta0) tau + (A.A - eta0^2) = 0, past root.
    a2 = v * v - 1.0
    a1 = 2.0 * (A @ B + eta0)
    a0 = np.sum(A * A, axis=1) - eta0 ** 2
    disc = np.sqrt(a1 * a1 - 4 * a2 * a0)
    r1 = (-a1 + disc) / (2 * a2)
    r2 = (-a1 - disc) / (2 * a2)
    tau = np.where(r1 < eta0, r1, r2)
    tau = np.where((r1 < eta0) & (r2 < eta0), np.maximum(r1, r2), tau)
    X = A + tau[:, None] * B[None, :]
    assert np.allclose(np.linalg.norm(X, axis=1), eta0 - tau, rtol=1e-13, atol=1e-13)
    n = len(sig)
    xd = np.tile(B, (n, 1))
    xp = np.tile(s_hat / gamma, (n, 1))
    return X, xd, xp, np.full(n, dsig), gamma


ORIENTATIONS = [
    # (n.s, n.v) of the line of sight; the remaining component is along s x v
    (0.0, 0.0),
    (0.4, 0.0),
    (0.0, -0.5),
    (0.3, 0.45),
    (-0.6, 0.2),
]


@pytest.mark.parametrize("cs,cv", ORIENTATIONS)
@pytest.mark.parametrize("v", [0.3, 0.7])
def test_kaiser_stebbins_step(cs, cv, v):
    s_hat, v_hat, w_hat = _orthonormal(11)
    cw = math.sqrt(1.0 - cs * cs - cv * cv)
    n0 = cs * s_hat + cv * v_hat + cw * w_hat
    eta0, dist = 3.0, 1.0
    X, xd, xp, ds, gamma = straight_string_on_light_cone(n0, s_hat, v_hat, v, dist, eta0,
                                                       half_len=2.0, dsig=2.5e-5)
    box = _box(X, xd, xp, ds)
    # Image tangent at the sigma = 0 event and the unit normal e = n x t / |n x t|.
    a = n0 @ xp[0]
    b = 1.0 + n0 @ xd[0]
    t = xp[0] - xd[0] * a / b
    e = np.cross(n0, t)
    e /= np.linalg.norm(e)

    def step(beta):
        dirs = np.stack([n0 + beta * e, n0 - beta * e])
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        th = oracle.theta_dirs(dirs, eta0, [box])
        return th[0] - th[1]

    beta = 2e-3
    s1, s2, s4 = step(beta), step(beta / 2), step(beta / 4)
    r1 = 2 * s2 - s1          # removes the O(beta) smooth-part and end corrections
    r2 = 2 * s4 - s2
    richardson = (4 * r2 - r1) / 3
    expected = 8 * math.pi * gamma * v * float(n0 @ np.cross(v_hat, s_hat))
    assert abs(richardson - expected) <= 2e-4 * abs(expected), (richardson, expected)


def test_kaiser_stebbins_sign_flips_with_velocity():
    s_hat, v_hat, w_hat = _orthonormal(3)
    n0 = w_hat
    res = []
    for vh in (v_hat, -v_hat):
        X, xd, xp, ds, gamma = straight_string_on_light_cone(n0, s_hat, vh, 0.5, 1.0, 3.0,
                                                           half_len=1.0, dsig=5e-5)
        box = _box(X, xd, xp, ds)
        t = xp[0] - xd[0] * (n0 @ xp[0]) / (1.0 + n0 @ xd[0])
        e = np.cross(n0, t)
        e /= np.linalg.norm(e)
        dirs = np.stack([n0 + 1e-3 * e, n0 - 1e-3 * e])
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        th = oracle.theta_dirs(dirs, 3.0, [box])
        res.append(th[0] - th[1])
    assert res[0] * res[1] < 0


def test_flat_sky_limit():
    """A 0.01-wide box at distance 10 around the z axis: the full-sky sum
    agrees with the 2-D small-angle form (n -> fixed axis, transverse
    separations) to O(theta^2)."""
    rng = np.random.default_rng(7)
    nseg = 40
    x, xd, xp, ds = synth.segments(nseg, 17, np.float64, side=0.01)
    origin = np.array([-0.005, -0.005, 10.0])
    box = _box(x, xd, xp, ds, origin=origin)
    eta0 = 20.0
    P = origin + x
    zhat = np.array([0.0, 0.0, 1.0])
    # Sky points within a few box widths of the axis, away from the segments.
    ang = rng.uniform(-2e-3, 2e-3, size=(60, 2))
    dirs = np.column_stack([ang[:, 0], ang[:, 1], np.ones(60)])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    full = oracle.theta_dirs(dirs, eta0, [box])
    # Flat-sky: theta-plane positions, u built with the fixed axis.
    flat = np.zeros(len(dirs))
    Xpar = P[:, 2]
    pos_s = P[:, :2] / Xpar[:, None]
    a = xp @ zhat
    b = 1.0 + xd @ zhat
    u = xd - (a / b)[:, None] * xp
    eps = np.sqrt(np.sum(xp * xp, 1) / (1 - np.sum(xd * xd, 1)))
    for k, n in enumerate(dirs):
        pos = n[:2] / n[2]
        sep = pos[None, :] - pos_s
        flat[k] = np.sum(-4.0 * np.sum(u[:, :2] * sep, 1) / (Xpar * np.sum(sep * sep, 1)) * eps * ds)
    rel = np.max(np.abs(full - flat)) / np.max(np.abs(flat))
    assert rel < 5e-3, rel        # O(theta) with theta ~ 1e-3 box angular size


def test_circular_loop_quadrature():
    """Eq. (1) along the events of a circular loop X = rho cos(tau/rho)
    (cos(sigma/rho), sin(sigma/rho), 0) + Xc on the past light cone: the
    segment sum (midpoints) equals adaptive quadrature of the integral."""
    rho, Xc, eta0 = 0.3, np.array([0.2, -0.1, 2.0]), 4.0
    n_dir = np.array([0.3, 0.2, 1.0])
    n_dir /= np.linalg.norm(n_dir)

    def event(sig):
        # Solve |X(sig, tau)| = eta0 - tau by bisection in FP64.
        def F(tau):
            c = math.cos(tau / rho)
            X = rho * c * np.array([math.cos(sig / rho), math.sin(sig / rho), 0.0]) + Xc
            return np.linalg.norm(X) - (eta0 - tau)
        lo, hi = 0.0, eta0
        flo = F(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = F(mid)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
        tau = 0.5 * (lo + hi)
        cs, sn = math.cos(sig / rho), math.sin(sig / rho)
        ct, st = math.cos(tau / rho), math.sin(tau / rho)
        X = rho * ct * np.array([cs, sn, 0.0]) + Xc
        Xd = -st * np.array([cs, sn, 0.0])
        Xp = ct * np.array([-sn, cs, 0.0])
        return X, Xd, Xp

    def integrand(sig):
        X, Xd, Xp = event(sig)
        R = np.linalg.norm(X)
        d = R * n_dir - X
        a = n_dir @ Xp
        b = 1 + n_dir @ Xd
        u = Xd - a / b * Xp
        eps = math.sqrt((Xp @ Xp) / (1 - Xd @ Xd))
        return -4.0 * (u @ d) / (d @ d) * eps

    L = 2 * math.pi * rho
    ref, err = integrate.quad(integrand, 0.0, L, limit=400, epsabs=1e-14, epsrel=1e-13)
    K = 512
    sig = (np.arange(K) + 0.5) * L / K
    ev = [event(s) for s in sig]
    box = _box([e[0] for e in ev], [e[1] for e in ev], [e[2] for e in ev], np.full(K, L / K))
    got = oracle.theta_dirs(n_dir[None, :], eta0, [box])[0]
    assert abs(got - ref) <= 1e-9 * abs(ref), (got, ref)


def _tiny_workload(seed=3, n=12, nside=4):
    rng = np.random.default_rng(seed)
    x, xd, xp, ds = synth.segments(n, seed, np.float64)
    b1 = _box(x[: n // 2], xd[: n // 2], xp[: n // 2], ds[: n // 2], origin=(-0.5, -0.5, -0.5),
              eta_lo=0.0, eta_hi=1.0)
    b2 = _box(x[n // 2:], xd[n // 2:], xp[n // 2:], ds[n // 2:], origin=(0.7, -0.2, 0.1),
              eta_lo=-0.45, eta_hi=0.2)
    return [b1, b2], 1.0, nside


def test_linearity_superposition_and_order():
    boxes, eta0, nside = _tiny_workload()
    pix = np.arange(12 * nside * nside)
    full = oracle.theta_pixels(nside, pix, eta0, boxes)
    parts = sum(oracle.theta_pixels(nside, pix, eta0, [b]) for b in boxes)
    assert np.allclose(full, parts, rtol=1e-14, atol=1e-14 * np.max(np.abs(full)))
    # segment-by-segment superposition
    b = boxes[0]
    singles = 0
    for i in range(b.n):
        bi = _box(b.x_rel[i:i + 1], b.xdot[i:i + 1], b.xprime[i:i + 1], b.dsigma[i:i + 1],
                  origin=b.origin, eta_lo=b.eta_lo, eta_hi=b.eta_hi)
        singles = singles + oracle.theta_pixels(nside, pix, eta0, [bi])
    one = oracle.theta_pixels(nside, pix, eta0, [b])
    assert np.allclose(one, singles, rtol=1e-13, atol=1e-13 * np.max(np.abs(one)))
    # linear in dsigma
    b3 = _box(b.x_rel, b.xdot, b.xprime, 3.0 * b.dsigma, origin=b.origin, eta_lo=b.eta_lo,
              eta_hi=b.eta_hi)
    assert np.allclose(oracle.theta_pixels(nside, pix, eta0, [b3]), 3.0 * one, rtol=1e-14,
                       atol=1e-14 * np.max(np.abs(one)))
    # order of segments does not matter
    perm = np.random.default_rng(1).permutation(b.n)
    bp = _box(b.x_rel[perm], b.xdot[perm], b.xprime[perm], b.dsigma[perm], origin=b.origin,
              eta_lo=b.eta_lo, eta_hi=b.eta_hi)
    assert np.allclose(oracle.theta_pixels(nside, pix, eta0, [bp]), one, rtol=1e-13,
                       atol=1e-13 * np.max(np.abs(one)))


def test_rotation_covariance_quarter_turn():
    """Rotating every input vector by 90 degrees about z permutes the RING
    map by a quarter of each ring."""
    nside = 8
    x, xd, xp, ds = synth.segments(30, 9, np.float64)
    origin = np.array([-0.3, -0.6, -0.45])
    rot = lambda a: np.column_stack([-a[:, 1], a[:, 0], a[:, 2]])
    P = origin + x
    b = _box(P, xd, xp, ds)
    br = _box(rot(P), rot(xd), rot(xp), ds)
    pix = np.arange(12 * nside * nside)
    m = oracle.theta_pixels(nside, pix, 2.0, [b])
    mr = oracle.theta_pixels(nside, pix, 2.0, [br])
    ring, pos = oracle.ring_of_pixel(nside, pix)
    start = {int(r): int(np.argmax(ring == r)) for r in np.unique(ring)}
    length = {int(r): int(np.sum(ring == r)) for r in np.unique(ring)}
    q = np.array([start[int(r)] + (int(j) + length[int(r)] // 4) % length[int(r)]
                  for r, j in zip(ring, pos)])
    assert np.allclose(mr[q], m, rtol=1e-12, atol=1e-12 * np.max(np.abs(m)))


def test_exact_coincidence_contributes_zero():
    # Nside=1 pixel 4 points exactly along +x; a segment at (0.5, 0, 0)
    # sits exactly on that ray, so |R n - P|^2 = 0 for that pixel.
    x = np.array([[0.5, 0.0, 0.0], [0.1, 0.3, -0.2]])
    xd = np.array([[0.0, 0.5, 0.0], [0.3, 0.0, 0.1]])
    xp = np.array([[0.0, 0.0, math.sqrt(0.75)], [0.0, 0.6, 0.0]])
    ds = np.array([0.01, 0.01])
    both = oracle.theta_pixels(1, np.arange(12), 1.0, [_box(x, xd, xp, ds)])
    second = oracle.theta_pixels(1, np.arange(12), 1.0, [_box(x[1:], xd[1:], xp[1:], ds[1:])])
    assert np.all(np.isfinite(both))
    assert both[4] == second[4]


def test_light_cone_selection():
    rng = np.random.default_rng(4)
    x, xd, xp, ds = synth.segments(4000, 4, np.float64)
    origin = np.array([0.6, -0.4, 0.9])
    b = _box(x, xd, xp, ds, origin=origin, eta_lo=0.7, eta_hi=1.5)
    eta0 = 3.0
    R = np.linalg.norm(origin + x, axis=1)
    expect = (eta0 - R >= 0.7) & (eta0 - R < 1.5)
    got = oracle.kept(eta0, b)
    near_edge = (np.abs(eta0 - R - 0.7) < 1e-12) | (np.abs(eta0 - R - 1.5) < 1e-12)
    assert np.array_equal(got[~near_edge], expect[~near_edge])
    assert 0 < got.sum() < len(got)


def test_ray_box_visibility_against_marching():
    """A pixel sees a VIS_BOX box when its ray crosses the box at a radius
    inside the slab: compare with dense sampling along each ray."""
    nside = 16
    pix = np.arange(12 * nside * nside)
    dirs = oracle.pix2vec(nside, pix)
    origin = np.array([0.8, -0.3, 0.4])
    b = _box(np.zeros((1, 3)), np.zeros((1, 3)), np.ones((1, 3)), np.ones(1), origin=origin,
             eta_lo=0.0, eta_hi=1.4, vis=synth.VIS_BOX)
    eta0 = 3.0          # radii (1.6, 3.0]
    vis = oracle.visible(nside, pix, eta0, b)
    t = np.linspace(1.6 + 1e-9, 3.0, 4000)
    margin = 2e-3
    for k in range(len(pix)):
        pts = t[:, None] * dirs[k][None, :]
        inside = np.all((pts >= origin - 1e-12) & (pts <= origin + 1 + 1e-12), axis=1)
        deep = np.all((pts >= origin + margin) & (pts <= origin + 1 - margin), axis=1)
        if deep.any():
            assert vis[k]
        elif not inside.any():
            assert not vis[k]
    assert 0 < vis.sum() < len(pix)


def test_gradient_against_finite_differences():
    boxes, eta0, nside = _tiny_workload(seed=8, n=10, nside=4)
    pix = np.arange(12 * nside * nside)
    rng = np.random.default_rng(2)
    g = rng.standard_normal(len(pix))
    nseg = sum(b.n for b in boxes)
    sel = np.arange(nseg)
    G = oracle.grad(nside, pix, g, eta0, boxes, sel)
    h = 1e-6
    fd = np.zeros_like(G)
    off = np.cumsum([0] + [b.n for b in boxes])
    for s in range(nseg):
        bi = int(np.searchsorted(off, s, side="right") - 1)
        li = s - off[bi]
        for c in range(10):
            vals = []
            for sgn in (1.0, -1.0):
                bb = [Box(**{**vars(b)}) for b in boxes]
                tgt = bb[bi]
                arrs = {"x_rel": tgt.x_rel.copy(), "xdot": tgt.xdot.copy(),
                        "xprime": tgt.xprime.copy(), "dsigma": tgt.dsigma.copy()}
                name = ["x_rel", "xdot", "xprime", "dsigma"][min(c // 3, 3)]
                if name == "dsigma":
                    arrs[name][li] += sgn * h
                else:
                    arrs[name][li, c % 3] += sgn * h
                for k2, val in arrs.items():
                    setattr(tgt, k2, val)
                vals.append(np.dot(g, oracle.theta_pixels(nside, pix, eta0, bb)))
            fd[s, c] = (vals[0] - vals[1]) / (2 * h)
    kept = np.concatenate([oracle.kept(eta0, b) for b in boxes])
    assert kept.any() and not kept.all()
    assert np.all(G[~kept] == 0.0)
    scale = np.max(np.abs(fd[kept]))
    assert np.max(np.abs(G[kept] - fd[kept])) <= 1e-6 * scale, np.max(np.abs(G - fd)) / scale


@pytest.mark.parametrize("theta", [1e-2, 1e-4, 1e-6, 1e-8, 1e-9])
def test_single_term_accuracy_near_line_of_sight(theta):
    """One term of Eq. (1)-(2) for an event at angle theta from the direction,
    against 50-digit arithmetic on the same FP64 inputs (P, and R formed as
    the FP64 root of the FP64 sum of squares): accurate to ~1e-14 for every
    theta."""
    import mpmath as mp
    mp.mp.dps = 50
    rng = np.random.default_rng(int(-math.log10(theta)))
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    perp = np.cross(n, rng.standard_normal(3))
    perp /= np.linalg.norm(perp)
    R0 = 1.7
    P = R0 * (math.cos(theta) * n + math.sin(theta) * perp)
    x, xd, xp, ds = synth.segments(1, 3, np.float64)
    box = _box(P[None, :], xd, xp, ds)
    got = oracle.theta_dirs(n[None, :], 10.0, [box])[0]
    R = math.sqrt((P[0] * P[0] + P[1] * P[1]) + P[2] * P[2])
    mn = [mp.mpf(float(v)) for v in n]
    mP = [mp.mpf(float(v)) for v in P]
    mR = mp.mpf(R)
    V = [mp.mpf(float(v)) for v in xd[0]]
    T = [mp.mpf(float(v)) for v in xp[0]]
    d = [mR * mn[k] - mP[k] for k in range(3)]
    q = sum(v * v for v in d)
    a = sum(mn[k] * T[k] for k in range(3))
    b = 1 + sum(mn[k] * V[k] for k in range(3))
    u = [V[k] - a / b * T[k] for k in range(3)]
    eps = mp.sqrt(sum(t * t for t in T) / (1 - sum(v * v for v in V)))
    exact = -4 * sum(u[k] * d[k] for k in range(3)) / q * eps * mp.mpf(float(ds[0]))
    assert abs(got - float(exact)) <= 1e-14 * abs(float(exact)), (got, float(exact))
