"""GPU parity of the flat-sky small-angle map (csmap_render_flat; Sec. II.A,
Sec. III.B, Fig. 3) against the oracle's flat map.  Bars: rel_rms <= 1e-5
and rel_max <= 1e-4 (the FP32 pair sum against FP64), on whole grids that
span several tiles with ragged row ends, on skies of cone boxes and snapshot
boxes, and on sampled pixels of the full 1024 x 1024 patch with 2,000,000
segments."""
import math
import sys

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


def sky_of(B, fp, form):
    sky = B.Sky(64, fp.eta0, form)
    for bx in fp.boxes:
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
             for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
        sky.add_box(*t, origin=tuple(bx.origin), eta_lo=bx.eta_lo, eta_hi=bx.eta_hi)
    return sky


def gpu_flat(sky, fp):
    return sky.render_flat(fp.center, fp.e1, fp.e2, fp.nx, fp.ny, fp.pix,
                           fp.accept_cos).cpu().numpy()


@pytest.mark.parametrize("nx,ny", [(96, 64), (1100, 3), (513, 7), (1, 1), (2, 9)])
@pytest.mark.parametrize("form", ["fp32c", "fp64"])
def test_flat_matches_oracle(B, nx, ny, form):
    fp = synth.flat_pencil(20_001, 64, seed=810)
    fp.nx, fp.ny = nx, ny
    fp.pix = math.radians(7.2) / max(nx, ny)
    say(f"flat nx={nx} ny={ny} form={form}")
    f = B.CSMAP_FORM_FP32C if form == "fp32c" else B.CSMAP_FORM_FP64
    sky = sky_of(B, fp, f)
    got = gpu_flat(sky, fp)
    sky.close()
    ref = oracle.flat_theta(nx, ny, fp.pix, fp.frame, fp.accept_cos, fp.eta0, fp.boxes)
    e = err_metrics(got, ref)
    say(f"  {e}")
    assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e


def test_flat_tilted_patch_with_cone_and_snapshot_boxes(B):
    """A patch off the poles with a rotated frame; the sky holds a cone box
    (rotation and cone test of the light-cone stage), a snapshot box and a
    plain FP64 box."""
    c = np.array([0.3, -0.5, 0.8])
    c /= np.linalg.norm(c)
    e1 = np.cross(c, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(c, e1)
    nside_c = 2
    cone = int(oracle.ang2pix(nside_c, c[None])[0])
    R, origin = oracle.cone_frame(nside_c, cone, 1, 2.0, 3.0)
    x, xd, xp, ds = synth.segments(6000, 820, np.float32, 3.0)
    xs, vs, ps, dss = synth.segments(3000, 821, np.float64, 0.6)
    xs = xs + 1.5 * c - 0.3
    xq, vq, pq, dq = synth.segments(2000, 822, np.float64, 0.5)
    xq = xq + 1.2 * c - 0.25
    eta0, lo, hi = 3.0, 1.0, 2.0
    # oracle boxes in the sky frame
    P, V, T = oracle.place_segments(x, xd, xp, R, origin)
    keep = oracle.in_cone(nside_c, cone, P)
    b_cone = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=lo, eta_hi=hi, x_rel=P[keep],
                       xdot=V[keep], xprime=T[keep], dsigma=ds[keep].astype(np.float64))
    pos, _, k2 = oracle.cone_events(xs, vs, np.zeros(3), eta0, lo, hi)
    b_snap = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=0.0, eta_hi=3.0,
                       x_rel=pos[k2], xdot=vs[k2], xprime=ps[k2], dsigma=dss[k2])
    b_plain = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=lo, eta_hi=hi, x_rel=xq,
                        xdot=vq, xprime=pq, dsigma=dq)
    nx, ny, pix, acc = 200, 150, math.radians(20.0) / 200, math.cos(math.radians(25.0))
    ref = oracle.flat_theta(nx, ny, pix, np.stack([c, e1, e2]), acc, eta0,
                            [b_cone, b_snap, b_plain])
    sky = B.Sky(16, eta0, B.CSMAP_FORM_FP32C)
    t = [torch.from_numpy(a).cuda() for a in (x, xd, xp, ds)]
    sky.add_box(*t, origin=tuple(origin), eta_lo=lo, eta_hi=hi, cone=B.make_cone(nside_c, cone, R))
    t = [torch.from_numpy(a).cuda() for a in (xs, vs, ps, dss)]
    sky.add_box(*t, origin=(0.0, 0.0, 0.0), eta_lo=lo, eta_hi=hi, snapshot=True)
    t = [torch.from_numpy(a).cuda() for a in (xq, vq, pq, dq)]
    sky.add_box(*t, origin=(0.0, 0.0, 0.0), eta_lo=lo, eta_hi=hi)
    got = sky.render_flat(c, e1, e2, nx, ny, pix, acc).cpu().numpy()
    e = err_metrics(got, ref)
    say(f"tilted patch with cone/snapshot boxes: {e}")
    assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e
    sky.close()


def test_flat_leaves_render_unchanged_and_handles_empty(B):
    fp = synth.flat_pencil(5000, 32, seed=830)
    sky = sky_of(B, fp, B.CSMAP_FORM_FP32C)
    m1 = sky.render().cpu().numpy()
    gpu_flat(sky, fp)
    m2 = sky.render().cpu().numpy()
    np.testing.assert_array_equal(m1, m2)
    # accept_cos = 1 admits nothing: the map is zero
    z = sky.render_flat(fp.center, fp.e1, fp.e2, 40, 30, fp.pix, 1.0).cpu().numpy()
    assert np.all(z == 0.0)
    sky.close()
    empty = B.Sky(8, 16.0, B.CSMAP_FORM_FP32C)
    z = empty.render_flat(fp.center, fp.e1, fp.e2, 17, 5, fp.pix, fp.accept_cos).cpu().numpy()
    assert np.all(z == 0.0)
    # Rejected: bad sizes and axes, accept_cos outside (0, 1], and cones so
    # wide for the pixel size that plane offsets would exceed 2^30 pixels.
    for bad in (dict(nx=0), dict(pix=0.0), dict(accept_cos=2.0), dict(e1=(0.0, 0.0, 1.0)),
                dict(center=(0.0, 0.0, 2.0)), dict(accept_cos=-1.0), dict(accept_cos=0.0),
                dict(accept_cos=math.cos(math.radians(89.0)), pix=1e-11)):
        kw = dict(center=fp.center, e1=fp.e1, e2=fp.e2, nx=4, ny=4, pix=fp.pix,
                  accept_cos=fp.accept_cos)
        kw.update(bad)
        with pytest.raises(B.CsmapError):
            empty.render_flat(**kw)
    empty.close()


def test_flat_full_patch_sampled(B):
    """The bench patch: 1024 x 1024 pixels of 0.42', 2,000,000 segments."""
    fp = synth.flat_pencil()
    say("flat full patch")
    sky = sky_of(B, fp, B.CSMAP_FORM_FP32C)
    got = gpu_flat(sky, fp)
    sky.close()
    rng = np.random.default_rng(7)
    ii = np.concatenate([rng.integers(0, fp.nx, 1500), [0, fp.nx - 1, 511, 512]])
    jj = np.concatenate([rng.integers(0, fp.ny, 1500), [0, fp.ny - 1, 512, 511]])
    t = np.stack([(ii + 0.5 - fp.nx / 2) * fp.pix, (jj + 0.5 - fp.ny / 2) * fp.pix], 1)
    ref = oracle.flat_points(t, fp.frame, fp.accept_cos, fp.eta0, fp.boxes)
    e = err_metrics(got[jj, ii], ref)
    say(f"  sampled {len(ii)} pixels: {e}")
    assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e


def unit_dirs(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_render_dirs_matches_oracle(B, form):
    """Eq. (1) at caller directions (csmap_render_dirs): random directions,
    directions next to segments (close pairs) and a ragged count, over boxes
    with every visibility rule."""
    dtype = np.float64 if form == "fp64" else np.float32
    boxes = [synth.make_box(3000, 860, origin=(-0.5, -0.5, -0.5), eta_lo=0.0, eta_hi=1.0,
                            dtype=dtype),
             synth.make_box(2000, 861, origin=(0.6, -0.3, 0.2), eta_lo=0.0, eta_hi=3.0,
                            dtype=dtype, vis=synth.VIS_BOX),
             synth.make_box(2500, 862, origin=(-1.4, 0.9, 0.3), eta_lo=0.0, eta_hi=3.0,
                            dtype=dtype, vis=synth.VIS_CAP, cap_dir=np.array([-0.8, 0.6, 0.0]),
                            cap_cos=math.cos(0.5))]
    eta0 = 3.0
    P = boxes[0].origin + boxes[0].x_rel[:200].astype(np.float64)
    near = P / np.linalg.norm(P, axis=1, keepdims=True) + 1e-4 * unit_dirs(200, 3)
    raw = np.concatenate([3.0 * unit_dirs(5001, 2), 0.5 * near])
    # the directions the device forms from them: v / sqrt((x^2 + y^2) + z^2)
    r = np.sqrt((raw[:, 0] * raw[:, 0] + raw[:, 1] * raw[:, 1]) + raw[:, 2] * raw[:, 2])
    dirs = raw / r[:, None]
    ref = oracle.theta_dirs(dirs, eta0, boxes, use_vis=True)
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    sky = B.Sky(8, eta0, f)
    for bx in boxes:
        t = [torch.from_numpy(a).cuda() for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
        kw = {}
        if bx.cap_dir is not None:
            kw = dict(cap_dir=tuple(bx.cap_dir), cap_cos=bx.cap_cos)
        sky.add_box(*t, origin=tuple(bx.origin), eta_lo=bx.eta_lo, eta_hi=bx.eta_hi, vis=bx.vis,
                    ext=tuple(bx.ext), **kw)
    got = sky.render_dirs(torch.from_numpy(raw).cuda()).cpu().numpy()
    e = err_metrics(got, ref)
    say(f"render_dirs form={form}: {e}")
    if form == "fp64":
        assert e["rel_rms"] <= 1e-12 and e["rel_max"] <= 1e-12, e
    else:
        assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e
    # the pixel centres of the sky's own map give the map
    pc = B.pix2vec_ring(8)
    m = sky.render().cpu().numpy()
    g2 = sky.render_dirs(pc).cpu().numpy()
    tol = 1e-10 if form == "fp64" else 1e-5
    assert np.max(np.abs(g2 - m)) <= tol * np.max(np.abs(m))
    assert sky.render_dirs(torch.zeros((0, 3), dtype=torch.float64, device="cuda")).numel() == 0
    sky.close()


def test_flat_and_full_sky_on_straight_strings(B):
    """Fig. 3-style: the flat map and the full-sky sum at the same gnomonic
    directions, for long straight strings near the pole; the GPU profile of
    their difference (per annulus) equals the oracle's."""
    box = synth.straight_strings(12, 1500, seed=881)
    nx = 64
    pix = math.radians(7.2) / nx
    c, e1, e2 = np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    acc = math.cos(math.radians(20.0))
    t = (np.arange(nx) + 0.5 - nx / 2) * pix
    tx, ty = np.meshgrid(t, t)
    dirs = c[None, :] + tx.ravel()[:, None] * e1[None, :] + ty.ravel()[:, None] * e2[None, :]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    sky = B.Sky(8, 16.0, B.CSMAP_FORM_FP64)
    tt = [torch.from_numpy(a).cuda() for a in (box.x_rel, box.xdot, box.xprime, box.dsigma)]
    sky.add_box(*tt, origin=(0.0, 0.0, 0.0), eta_lo=box.eta_lo, eta_hi=box.eta_hi)
    full = sky.render_dirs(torch.from_numpy(dirs).cuda()).cpu().numpy().reshape(nx, nx)
    flat = sky.render_flat(c, e1, e2, nx, nx, pix, acc).cpu().numpy()
    sky.close()
    rfull = oracle.theta_dirs(dirs, 16.0, [box]).reshape(nx, nx)
    rflat = oracle.flat_theta(nx, nx, pix, np.stack([c, e1, e2]), acc, 16.0, [box])
    rad = np.degrees(np.hypot(tx, ty))
    for lo, hi in ((0.0, 1.2), (1.2, 2.4), (2.4, 6.0)):
        m = (rad >= lo) & (rad < hi)
        g = np.sqrt(np.mean((full - flat)[m] ** 2) / np.mean(full[m] ** 2))
        r = np.sqrt(np.mean((rfull - rflat)[m] ** 2) / np.mean(rfull[m] ** 2))
        say(f"  annulus {lo}-{hi} deg: flat vs full rel rms {g:.4f} (oracle {r:.4f})")
        assert abs(g - r) <= 1e-3 * r + 1e-6
