"""GPU parity of healpix-cone stacking (Sec. II.C, Fig. 1): the device
direction -> RING pixel map (csmap_ang2pix_ring) against the oracle, bit for
bit; skies of rotated cone boxes (csmap_add_cone_box: on-cone events and
slab-start segments, both forms) against the oracle's map of the oracle's
placed and cone-filtered segments; the adjoint of cone boxes in box
coordinates; and the full Nside_c = 16 + Nside_c = 1 stacking grid (3084
boxes) with kept counts equal to the oracle's and a sampled stacked map.
Bars: pixel indices and keep decisions identical; maps FP64 1e-12, FP32C
1e-5 rms / 1e-4 max relative; gradients 1e-4 relative."""
import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from helpers import err_metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    return binding


def gpu_pix(B, nside, v):
    return B.ang2pix_ring(nside, torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64))
                          .cuda()).cpu().numpy()


def check_pix(B, nside, v):
    """Device and oracle pixels identical: both take the azimuth from the same
    fixed arctangent recipe, so no direction is decided differently."""
    got = gpu_pix(B, nside, v)
    ref = oracle.ang2pix(nside, v)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("nside", [1, 2, 3, 16, 1024, 4096, 8192])
def test_device_ang2pix_matches_oracle(B, nside):
    say(f"ang2pix nside={nside}")
    rng = np.random.default_rng(500 + nside)
    v = rng.standard_normal((1_000_000, 3)) * rng.uniform(1e-3, 1e3, (1_000_000, 1))
    check_pix(B, nside, v)
    npx = 12 * nside * nside
    pix = np.arange(npx) if npx <= 200_000 else rng.integers(0, npx, 200_000)
    c = oracle.pix2vec(nside, pix)
    np.testing.assert_array_equal(gpu_pix(B, nside, c), pix)
    # directions on ring-centre latitudes and near the poles and the belt edge
    z = c[:, 2]
    phi = rng.uniform(0, 2 * np.pi, len(z))
    s = np.sqrt(1 - z * z)
    check_pix(B, nside, np.stack([s * np.cos(phi), s * np.sin(phi), z], 1))
    ph = rng.uniform(0, 2 * np.pi, 1000)
    for zz in (1.0, -1.0, 2.0 / 3.0, -2.0 / 3.0, 0.0):
        sz = math.sqrt(1 - zz * zz)
        w = np.stack([sz * np.cos(ph), sz * np.sin(ph), np.full(1000, zz)], 1)
        check_pix(B, nside, w)
    assert gpu_pix(B, nside, np.zeros((0, 3))).size == 0


def cone_sky_case(dtype, nside_c, cones, axes, side=3.0, seed=700, nseg=6000, speeds=None):
    """Cone boxes of a shell r in [1, 2] (eta0 = 3, slab [1, 2)): runs of
    segments in [0, side)^3, each placed in its cone by the oracle's frame."""
    r_in, r_out, eta0 = 1.0, 2.0, 3.0
    uses = []
    for k, (cone, axis) in enumerate(zip(cones, axes)):
        x, xd, xp, ds = synth.segments(nseg, seed + k, dtype, side)
        if speeds is not None:   # slab-start segments: wider speed range
            rng = np.random.default_rng(seed + 50 + k)
            v = rng.uniform(*speeds, nseg)
            xd64 = xd.astype(np.float64)
            xp64 = xp.astype(np.float64)
            xd = (xd64 / np.linalg.norm(xd64, axis=1, keepdims=True) * v[:, None]).astype(dtype)
            xp = (xp64 / np.linalg.norm(xp64, axis=1, keepdims=True) *
                  np.sqrt(1 - v * v)[:, None]).astype(dtype)
        R, origin = oracle.cone_frame(nside_c, cone, axis, r_out, side)
        uses.append(dict(cone=cone, axis=axis, R=R, origin=origin, x=x, xd=xd, xp=xp, ds=ds))
    return eta0, eta0 - r_out, eta0 - r_in, uses


def oracle_cone_boxes(eta0, lo, hi, nside_c, uses, snapshot):
    """The oracle's on-cone boxes of placed, cone-filtered segments, with
    the index of every kept segment inside its run."""
    out, idx = [], []
    for u in uses:
        P, V, T = oracle.place_segments(u["x"], u["xd"], u["xp"], u["R"], u["origin"])
        ds = u["ds"].astype(np.float64)
        if snapshot:
            pos, _, keep = oracle.cone_events(P, V, np.zeros(3), eta0, lo, hi)
            keep &= oracle.in_cone(nside_c, u["cone"], np.where(keep[:, None], pos, 1.0))
            P = pos
            width = hi - lo
            blo, bhi = lo - width, hi + width
        else:
            box = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=lo, eta_hi=hi, x_rel=P,
                            xdot=V, xprime=T, dsigma=ds)
            keep = oracle.kept(eta0, box) & oracle.in_cone(nside_c, u["cone"], P)
            blo, bhi = lo, hi
        out.append(synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=blo, eta_hi=bhi,
                             x_rel=P[keep], xdot=V[keep], xprime=T[keep], dsigma=ds[keep]))
        idx.append(np.nonzero(keep)[0])
    return out, idx


def gpu_cone_sky(B, nside, eta0, lo, hi, nside_c, uses, form, snapshot):
    sky = B.Sky(nside, eta0, form)
    for u in uses:
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
             for a in (u["x"], u["xd"], u["xp"], u["ds"])]
        sky.add_box(*t, origin=tuple(u["origin"]), eta_lo=lo, eta_hi=hi, snapshot=snapshot,
                    cone=B.make_cone(nside_c, u["cone"], u["R"]))
    return sky


@pytest.mark.parametrize("snapshot", [False, True])
@pytest.mark.parametrize("form", ["fp64", "fp32c"])
@pytest.mark.parametrize("nside_c,cones,axes", [(1, [0, 5, 7, 10], [0, 1, 2, 2]),
                                                (2, [3, 20, 30, 47], [2, 0, 1, 0])])
def test_cone_sky_matches_oracle(B, form, snapshot, nside_c, cones, axes):
    dtype = np.float64 if form == "fp64" else np.float32
    eta0, lo, hi, uses = cone_sky_case(dtype, nside_c, cones, axes,
                                       speeds=(0.0, 0.95) if snapshot else None)
    nside = 32
    boxes, idx = oracle_cone_boxes(eta0, lo, hi, nside_c, uses, snapshot)
    kept = sum(len(i) for i in idx)
    say(f"cone sky nside_c={nside_c} form={form} snapshot={snapshot}: kept {kept} of "
        f"{sum(len(u['ds']) for u in uses)}")
    assert kept > 300
    ref = oracle.theta_pixels(nside, np.arange(12 * nside * nside), eta0, boxes)
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    sky = gpu_cone_sky(B, nside, eta0, lo, hi, nside_c, uses, f, snapshot)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    sky.close()
    e = err_metrics(m, ref)
    say(f"  {e}")
    assert st["kept"] == kept
    if form == "fp64":
        assert e["rel_rms"] <= 1e-12 and e["rel_max"] <= 1e-12, e
    else:
        assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e


def test_cone_box_adjoint_in_box_coordinates(B):
    """dL/d(box-frame arrays) = R^T dL/d(sky-frame arrays); segments outside
    their cone get zero gradient."""
    eta0, lo, hi, uses = cone_sky_case(np.float32, 2, [3, 20, 30], [2, 0, 1], nseg=4000)
    nside = 16
    npix = 12 * nside * nside
    g = np.random.default_rng(3).standard_normal(npix)
    boxes, idx = oracle_cone_boxes(eta0, lo, hi, 2, uses, False)
    sky = gpu_cone_sky(B, nside, eta0, lo, hi, 2, uses, B.CSMAP_FORM_FP32C, False)
    sky.render()
    grads = sky.backward(torch.from_numpy(g).cuda())
    sky.close()
    off = np.concatenate([[0], np.cumsum([len(i) for i in idx])])
    gref_sky = oracle.grad(nside, np.arange(npix), g, eta0, boxes, np.arange(off[-1]))
    got_all, ref_all = [], []
    for b, u in enumerate(uses):
        got = np.concatenate([grads[b][0].cpu().numpy(), grads[b][1].cpu().numpy(),
                              grads[b][2].cpu().numpy(), grads[b][3].cpu().numpy()[:, None]], 1)
        ref = np.zeros_like(got)
        gs = gref_sky[off[b]:off[b + 1]]
        R = u["R"]
        for k in range(3):
            ref[idx[b], 3 * k:3 * k + 3] = gs[:, 3 * k:3 * k + 3] @ R
        ref[idx[b], 9] = gs[:, 9]
        outside = np.setdiff1d(np.arange(len(got)), idx[b])
        assert np.all(got[outside] == 0.0)
        got_all.append(got)
        ref_all.append(ref)
    got, ref = np.concatenate(got_all), np.concatenate(ref_all)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"cone adjoint: rel err {rel:.3e} over {off[-1]} kept segments")
    assert rel <= 1e-4


def test_cone_box_rejects_bad_rotations(B):
    sky = B.Sky(8, 3.0, B.CSMAP_FORM_FP32C)
    t = [torch.zeros((4, 3), dtype=torch.float32, device="cuda") for _ in range(3)]
    ds = torch.ones(4, dtype=torch.float32, device="cuda")
    for rot in (np.diag([1.0, 1.0, -1.0]), 2 * np.eye(3), np.full((3, 3), np.nan)):
        with pytest.raises(B.CsmapError):
            sky.add_box(*t, ds, origin=(0, 0, 0), eta_lo=0.0, eta_hi=1.0,
                        cone=B.make_cone(2, 0, rot))
    with pytest.raises(B.CsmapError):
        sky.add_box(*t, ds, origin=(0, 0, 0), eta_lo=0.0, eta_hi=1.0, cone=B.make_cone(2, 48, np.eye(3)))
    with pytest.raises(B.CsmapError):
        sky.add_box(*t, ds, origin=(0, 0, 0), eta_lo=0.0, eta_hi=1.0, vis=B.CSMAP_VIS_BOX,
                    cone=B.make_cone(2, 0, np.eye(3)))
    sky.close()


def stacked_sky(B, plans, nside):
    """Every cone of the plans as a cone box, placed by the library
    (csmap_cone_place), with the oracle's frames alongside."""
    sky = B.Sky(nside, plans[0].eta0, B.CSMAP_FORM_FP32C)
    runs, uses = {}, []
    for p in plans:
        with ThreadPoolExecutor(16) as ex:
            data = list(ex.map(lambda r: p.run(r), range(p.nruns)))
        for r, d in enumerate(data):
            runs[(p.name, r)] = d
        dev = {}
        for cone, r, axis in p.uses:
            if r not in dev:
                dev[r] = [torch.from_numpy(a).cuda() for a in runs[(p.name, r)]]
            c, origin, slack = B.cone_place(p.nside_c, cone, axis, p.r_in, p.r_out, p.side)
            assert slack >= 0
            sky.add_box(*dev[r], origin=tuple(origin), eta_lo=p.eta_lo, eta_hi=p.eta_hi, cone=c)
            uses.append((p, cone, r, axis, np.array(c.rot[:], dtype=np.float64).reshape(3, 3),
                         np.array(origin, dtype=np.float64)))
        torch.cuda.synchronize()
    return sky, runs, uses


def test_full_stacking_grid(B):
    """The Nside_c = 16 grid (3072 cones from 1024 runs x 3 axes) and the
    Nside_c = 1 grid (12 cones), 20,000 segments per run: total kept equals
    the oracle's count of placed segments inside their cone and slab, every
    cone gets about its share of the shell volume, and the stacked map at
    Nside 16 matches the oracle on 96 pixels."""
    plans = [synth.stack_highz(20_000), synth.stack_lowz(20_000)]
    say("stacking grid: building 3084 cone boxes")
    sky, runs, uses = stacked_sky(B, plans, 16)
    sky.precompute()
    st = sky.stats()
    say(f"  device kept {st['kept']} of {st['segments']}, precompute {st['ms_precompute']:.2f} ms")
    # oracle: place every use with the frame the library used, count what is kept
    def count(u):
        p, cone, r, axis, R, origin = u
        x, xd, xp, ds = runs[(p.name, r)]
        P, V, T = oracle.place_segments(x, xd, xp, R, origin)
        rr = np.sqrt((P[:, 0] * P[:, 0] + P[:, 1] * P[:, 1]) + P[:, 2] * P[:, 2])
        eta = p.eta0 - rr
        keep = (rr > 0) & (eta >= p.eta_lo) & (eta < p.eta_hi) & oracle.in_cone(p.nside_c, cone, P)
        return int(keep.sum()), (P[keep], V[keep], T[keep], ds[keep].astype(np.float64))
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(count, uses))
    ref_kept = sum(k for k, _ in res)
    say(f"  oracle kept {ref_kept}")
    # The oracle places each run with the frame the library used (the
    # library's frames are pinned against the oracle's own on the CPU), so
    # every keep decision is the same computation on both sides.
    assert st["kept"] == ref_kept
    hz = np.array([k for (k, _), u in zip(res, uses) if u[0].nside_c == 16])
    p = plans[0]
    expect = 20_000 * (4 * math.pi / 3072) * (p.r_out ** 3 - p.r_in ** 3) / 3 / p.side ** 3
    say(f"  high-z kept per cone: mean {hz.mean():.1f}, expected {expect:.1f}")
    assert abs(hz.mean() / expect - 1) < 0.01
    assert abs(hz.std() / math.sqrt(expect) - 1) < 0.15
    m = sky.render().cpu().numpy()
    sky.close()
    pix = synth.sample_pixels(12 * 16 * 16, 96, 5)
    boxes = [synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=u[0].eta_lo, eta_hi=u[0].eta_hi,
                       x_rel=a[0], xdot=a[1], xprime=a[2], dsigma=a[3])
             for u, (_, a) in zip(uses, res)]
    ref = oracle.theta_pixels(16, pix, 16.0, boxes)
    e = err_metrics(m[pix], ref)
    say(f"  stacked map vs oracle on {len(pix)} pixels: {e}")
    assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e


def test_rotation_only_and_empty_cone_boxes(B):
    """nside = 0 turns a box onto the sky without a cone test; an empty cone
    box contributes nothing; both in the FP64 form against the oracle."""
    eta0, lo, hi = 3.0, 1.0, 2.0
    rng = np.random.default_rng(41)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    x, xd, xp, ds = synth.segments(4000, 890, np.float64, 2.0)
    origin = np.array([-0.4, 0.7, 0.2])
    P, V, T = oracle.place_segments(x, xd, xp, q, origin)
    ref_box = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=lo, eta_hi=hi, x_rel=P,
                        xdot=V, xprime=T, dsigma=ds)
    nside = 16
    ref = oracle.theta_pixels(nside, np.arange(12 * nside * nside), eta0, [ref_box])
    sky = B.Sky(nside, eta0, B.CSMAP_FORM_FP64)
    t = [torch.from_numpy(a).cuda() for a in (x, xd, xp, ds)]
    sky.add_box(*t, origin=tuple(origin), eta_lo=lo, eta_hi=hi, cone=B.make_cone(0, 0, q))
    e = [torch.zeros((0, 3), dtype=torch.float64, device="cuda") for _ in range(3)]
    sky.add_box(*e, torch.zeros(0, dtype=torch.float64, device="cuda"), origin=(1.0, 2.0, 3.0),
                eta_lo=lo, eta_hi=hi, cone=B.make_cone(4, 7, np.eye(3)))
    got = sky.render().cpu().numpy()
    st = sky.stats()
    sky.close()
    err = err_metrics(got, ref)
    say(f"rotation-only cone box: kept {st['kept']}, {err}")
    assert st["kept"] == int(oracle.kept(eta0, ref_box).sum())
    assert err["rel_rms"] <= 1e-12 and err["rel_max"] <= 1e-12, err


def edge_points(nside_c, cone, center, rng, count):
    """Directions within 1e-9 .. 1e-3 rad of the boundary of pixel `cone`,
    on both sides: boundary points found by bisection with the oracle's
    ang2pix along great circles from the pixel centre, then moved along
    the circle by the offsets."""
    out = []
    size = 1.02 / nside_c
    nb = count // 8   # boundary points, eight offsets each
    while len(out) < count:
        u = rng.standard_normal((4 * count, 3))
        u -= (u @ center)[:, None] * center
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        far = np.cos(1.5 * size) * center + np.sin(1.5 * size) * u
        far_out = oracle.ang2pix(nside_c, far) != cone
        a = np.zeros(len(u))
        b = np.full(len(u), 1.5 * size)
        u, a, b = u[far_out][:nb], a[far_out][:nb], b[far_out][:nb]
        for _ in range(60):
            mid = 0.5 * (a + b)
            d = np.cos(mid)[:, None] * center + np.sin(mid)[:, None] * u
            inside = oracle.ang2pix(nside_c, d) == cone
            a = np.where(inside, mid, a)
            b = np.where(inside, b, mid)
        for off in (1e-9, 1e-7, 1e-5, 1e-3):
            for sgn in (-1.0, 1.0):
                ang = 0.5 * (a + b) + sgn * off
                out.extend(np.cos(ang)[:, None] * center + np.sin(ang)[:, None] * u)
    return np.array(out[:count])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nside_c,cones,axes", [(1, [0, 4, 9], [0, 1, 2]),
                                                (2, [0, 19, 44], [2, 0, 1]),
                                                (16, [0, 1000, 1536, 3071], [1, 2, 0, 2])])
def test_cone_membership_near_pixel_edges(B, dtype, nside_c, cones, axes):
    """Segments placed within 1e-9 .. 1e-3 rad of their cone pixel's
    boundary, on both sides: the GPU keeps exactly the segments the oracle
    keeps (the bounding caps and edge planes only decide where the decision
    is certain, the rest go to the pixel test), and renders the same map."""
    rng = np.random.default_rng(4100 + nside_c)
    r_in, r_out, eta0, side = 1.0, 2.0, 3.0, 3.0
    uses = []
    for k, (cone, axis) in enumerate(zip(cones, axes)):
        R, origin = oracle.cone_frame(nside_c, cone, axis, r_out, side)
        center = R[:, axis]
        d = edge_points(nside_c, cone, center, rng, 800)
        P = d * rng.uniform(1.1, 1.9, (len(d), 1))
        x = ((P - origin) @ R).astype(dtype)          # box coordinates: R^T (P - origin)
        _, xd, xp, ds = synth.segments(len(d), 4200 + k, dtype, side)
        uses.append(dict(cone=cone, axis=axis, R=R, origin=origin, x=x, xd=xd, xp=xp, ds=ds))
    lo, hi = eta0 - r_out, eta0 - r_in
    boxes, idx = oracle_cone_boxes(eta0, lo, hi, nside_c, uses, False)
    kept = sum(len(i) for i in idx)
    total = sum(len(u["ds"]) for u in uses)
    say(f"edge cones nside_c={nside_c} dtype={np.dtype(dtype).name}: kept {kept} of {total}")
    assert 0.3 * total < kept < 0.7 * total
    nside = 32
    sky = gpu_cone_sky(B, nside, eta0, lo, hi, nside_c, uses, B.CSMAP_FORM_FP64, False)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    sky.close()
    assert st["kept"] == kept
    ref = oracle.theta_pixels(nside, np.arange(12 * nside * nside), eta0, boxes)
    e = err_metrics(m, ref)
    say(f"  {e}")
    assert e["rel_rms"] <= 1e-12 and e["rel_max"] <= 1e-12, e
