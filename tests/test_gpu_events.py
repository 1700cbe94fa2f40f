"""GPU parity of light-cone event recording from slab-start snapshots
(csmap_cone_events, csmap_add_snapshot_box) against the oracle, which finds
each crossing by bisection.  Bars: keep decisions identical; crossing time D
within 64 ulp of R0 / (1 - |Xdot|) and event positions within 64 ulp of R0
(two FP64 solutions of the same equation by different methods); maps of
snapshot skies within the forms' gates (FP64 1e-12, FP32C 1e-5 / 1e-4)
against the oracle's map of the oracle's events."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import err_metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    return binding


def snapshot_segments(n, seed, dtype):
    """Segments of a 1 Gpc box at the slab start: the synthetic recipe, with
    speeds up to 0.95 so that crossings span the slab."""
    rng = np.random.default_rng(seed)
    x, xd, xp, ds = synth.segments(n, seed, np.float64)
    v = rng.uniform(0.0, 0.95, n)
    xd = xd / np.linalg.norm(xd, axis=1, keepdims=True) * v[:, None]
    xp = xp / np.linalg.norm(xp, axis=1, keepdims=True) * np.sqrt(1 - v * v)[:, None]
    cast = lambda a: np.ascontiguousarray(a.astype(dtype))
    return cast(x), cast(xd), cast(xp), cast(ds)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_cone_events_match_oracle(B, dtype):
    n = 200_000
    x, xd, _, _ = snapshot_segments(n, 301, dtype)
    origin = np.array([3.7, -2.1, 1.4])
    eta0, eta_lo, eta_hi = 16.0, 11.0, 11.6
    say(f"cone events dtype={np.dtype(dtype).name}")
    pos, d, keep = B.cone_events(torch.from_numpy(x).cuda(), torch.from_numpy(xd).cuda(), origin,
                                 eta0, eta_lo, eta_hi)
    pos, d, keep = pos.cpu().numpy(), d.cpu().numpy(), keep.cpu().numpy()
    rpos, rd, rkeep = oracle.cone_events(x, xd, origin, eta0, eta_lo, eta_hi)
    say(f"kept {keep.sum()} of {n}")
    assert 0.2 * n < keep.sum() < 0.8 * n
    assert np.array_equal(keep, rkeep)
    R0 = eta0 - eta_lo
    speed = np.linalg.norm(xd.astype(np.float64), axis=1)
    tol = 64 * EPS * R0 / (1.0 - speed[keep])
    assert np.all(np.abs(d[keep] - rd[keep]) <= tol)
    assert np.max(np.abs(pos[keep] - rpos[keep])) <= 64 * EPS * R0
    assert np.isnan(d[~keep]).all() and np.isnan(pos[~keep]).all()


def test_cone_events_edges_and_fast_segments(B):
    eta0, eta_lo, eta_hi = 16.0, 4.0, 6.0
    R0 = eta0 - eta_lo
    x = np.array([[R0, 0.0, 0.0], [R0 - 2.0, 0.0, 0.0], [R0 - 1.0, 0.0, 0.0],
                  [R0 + 0.5, 0.0, 0.0], [5.0, 0.0, 0.0], [5.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    v = np.zeros_like(x)
    v[4] = [0.0, 1.0, 0.0]
    v[5] = [0.0, 0.0, 1.5]
    pos, d, keep = B.cone_events(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(),
                                 (0.0, 0.0, 0.0), eta0, eta_lo, eta_hi)
    rpos, rd, rkeep = oracle.cone_events(x, v, np.zeros(3), eta0, eta_lo, eta_hi)
    assert keep.cpu().numpy().tolist() == rkeep.tolist() == [True, False, True, False, False,
                                                             False, False]
    e = torch.empty(0, 3, dtype=torch.float64, device="cuda")
    p0, d0, k0 = B.cone_events(e, e, (0.0, 0.0, 0.0), eta0, eta_lo, eta_hi)
    assert p0.numel() == 0 and k0.numel() == 0


def snapshot_workload(nside, dtype):
    """Three snapshot boxes around a shell at ~2.7 (slab [0.4, 0.9) of
    eta0 = 3): one seen by every pixel, two seen through caps."""
    eta0 = 3.0
    boxes = []
    centres = [(2.2, 1.1, 0.6), (-1.3, 2.0, -1.0), (0.4, -1.6, 2.2)]
    for b, c in enumerate(centres):
        c = np.asarray(c)
        x, xd, xp, ds = snapshot_segments(400 + 150 * b, 320 + b, dtype)
        d = c / np.linalg.norm(c)
        kw = {}
        if b > 0:
            kw = dict(vis=synth.VIS_CAP, cap_dir=d, cap_cos=math.cos(0.6 + 0.2 * b))
        boxes.append(synth.Box(origin=c - 0.5, ext=np.ones(3), eta_lo=0.4, eta_hi=0.9, x_rel=x,
                               xdot=xd, xprime=xp, dsigma=ds, **kw))
    return synth.Workload("snapshot", nside, eta0, boxes)


def oracle_event_boxes(w):
    """The oracle's events of each snapshot box as on-cone boxes: origin 0,
    x_rel = event position, only the recorded segments, and a slab wide
    enough that the oracle's own slab test keeps every one of them."""
    out, kept = [], 0
    for bx in w.boxes:
        pos, d, keep = oracle.cone_events(bx.x_rel, bx.xdot, bx.origin, w.eta0, bx.eta_lo,
                                          bx.eta_hi)
        kept += int(keep.sum())
        width = bx.eta_hi - bx.eta_lo
        out.append(synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=bx.eta_lo - width,
                             eta_hi=bx.eta_hi + width, x_rel=pos[keep],
                             xdot=bx.xdot[keep].astype(np.float64),
                             xprime=bx.xprime[keep].astype(np.float64),
                             dsigma=bx.dsigma[keep].astype(np.float64), vis=bx.vis,
                             cap_dir=bx.cap_dir, cap_cos=bx.cap_cos))
    return out, kept


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_snapshot_sky_matches_oracle(B, form):
    dtype = np.float64 if form == "fp64" else np.float32
    w = snapshot_workload(48, dtype)
    ev, kept = oracle_event_boxes(w)
    pix = np.arange(w.npix)
    ref = oracle.theta_pixels(w.nside, pix, w.eta0, ev)
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    sky = B.Sky(w.nside, w.eta0, f)
    for bx in w.boxes:
        t = [torch.from_numpy(a).cuda() for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
        kw = {}
        if bx.cap_dir is not None:
            kw = dict(cap_dir=tuple(bx.cap_dir), cap_cos=bx.cap_cos)
        sky.add_box(*t, origin=tuple(bx.origin), eta_lo=bx.eta_lo, eta_hi=bx.eta_hi, vis=bx.vis,
                    snapshot=True, **kw)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    say(f"snapshot sky form={form} kept={st['kept']} (oracle {kept}) {e}")
    assert st["kept"] == kept
    if form == "fp64":
        assert e["rel_rms"] <= 1e-12 and e["rel_max"] <= 1e-12, e
    else:
        assert e["rel_rms"] <= 1e-5 and e["rel_max"] <= 1e-4, e
    if form == "fp32c":
        with pytest.raises(B.CsmapError):
            sky.backward(torch.zeros(w.npix, dtype=torch.float64, device="cuda"))
    sky.close()


def test_snapshot_box_rejects_the_ray_box_rule(B):
    sky = B.Sky(8, 3.0, B.CSMAP_FORM_FP32C)
    t = [torch.zeros((4, 3), dtype=torch.float32, device="cuda") for _ in range(3)]
    ds = torch.ones(4, dtype=torch.float32, device="cuda")
    with pytest.raises(B.CsmapError):
        sky.add_box(*t, ds, origin=(1.0, 1.0, 1.0), eta_lo=0.0, eta_hi=1.0, vis=B.CSMAP_VIS_BOX,
                    snapshot=True)
    sky.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [20_001, 20_002, 20_003])
def test_cone_events_odd_count_and_unaligned_arrays(B, dtype, n):
    """Odd and even counts (an odd one leaves the last thread of the
    two-segments-per-thread kernel one segment), and arrays offset by 0, 1
    or 2 elements: aligned for two segments per thread (0 and 2) or not
    (1: one segment per thread)."""
    x, xd, _, _ = snapshot_segments(n, 311, dtype)
    origin = np.array([1.2, -0.4, 2.1])
    eta0, eta_lo, eta_hi = 16.0, 12.0, 12.5
    rpos, rd, rkeep = oracle.cone_events(x, xd, origin, eta0, eta_lo, eta_hi)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    for off in (0, 1, 2):
        bx = torch.zeros(3 * n + 2, dtype=tdt, device="cuda")
        bv = torch.zeros(3 * n + 2, dtype=tdt, device="cuda")
        bx[off:off + 3 * n] = torch.from_numpy(x.ravel()).cuda()
        bv[off:off + 3 * n] = torch.from_numpy(xd.ravel()).cuda()
        xt, vt = bx[off:off + 3 * n].view(n, 3), bv[off:off + 3 * n].view(n, 3)
        say(f"cone events n={n} dtype={np.dtype(dtype).name} offset={off}")
        pos, d, keep = B.cone_events(xt, vt, origin, eta0, eta_lo, eta_hi)
        pos, d, keep = pos.cpu().numpy(), d.cpu().numpy(), keep.cpu().numpy()
        assert np.array_equal(keep, rkeep)
        R0 = eta0 - eta_lo
        speed = np.linalg.norm(xd.astype(np.float64), axis=1)
        assert np.all(np.abs(d[keep] - rd[keep]) <= 64 * EPS * R0 / (1.0 - speed[keep]))
        assert np.max(np.abs(pos[keep] - rpos[keep])) <= 64 * EPS * R0
        assert np.isnan(d[~keep]).all()
