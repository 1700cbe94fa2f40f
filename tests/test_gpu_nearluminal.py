"""GPU parity for segments moving close to the speed of light.

Eq. (2)'s denominator 1 + n.Xdot falls to 1 - |Xdot| for a pixel opposite
the velocity, and eps = sqrt(X'^2/(1 - Xdot^2)) (Sec. II.A) grows as
|Xdot| -> 1; cusps of Nambu-Goto strings reach such speeds.  The FP32C form
sends every segment with 1 - |Xdot| < 0.05 through its FP64-difference path.
Here speeds of 0.96, 0.99 and 0.999 move along the reverse of a pixel
centre's direction (so that pixel has b = 1 - |Xdot| up to the FP32 rounding
of the inputs), mixed with ordinary speeds.  Forward in both forms and the
adjoint against the oracle, at the usual bars; the flagged path must have
run."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import (SEG_REL, err_metrics, grad_group_errors, grad_segment_errors,
                     sky_from_workload)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
FP32_RMS, FP32_MAX = 1e-5, 1e-4
GRAD_TOL = 1e-4
SPEEDS = (0.96, 0.99, 0.999)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    assert torch.cuda.is_available()
    return binding


def _box(x, xd, xp, ds, origin, eta_lo, eta_hi, vis=synth.VIS_ALL):
    return synth.Box(origin=np.asarray(origin, float), ext=np.ones(3), eta_lo=eta_lo,
                     eta_hi=eta_hi, x_rel=x, xdot=xd, xprime=xp, dsigma=ds, vis=vis)


def workload(nside=64, n_fast=240, n_slow=120, seed=700):
    """Two boxes: one around the observer, one beside it seen through the
    ray-crosses-box rule; fast segments move away from a random pixel's
    direction."""
    npx = 12 * nside * nside
    rng = np.random.default_rng(seed)
    eta0 = 3.0
    boxes = []
    for k, (origin, lo, hi, vis) in enumerate((((-0.5, -0.5, -0.5), 2.2, 3.0, synth.VIS_ALL),
                                               ((0.8, -0.4, 0.2), 0.9, 1.8, synth.VIS_BOX))):
        opp = -oracle.pix2vec(nside, rng.integers(0, npx, n_fast))
        xf, vf, pf, df = synth.near_luminal_segments(n_fast, seed + 10 * k, SPEEDS, v_dirs=opp)
        xs, vs, ps, dss = synth.segments(n_slow, seed + 10 * k + 1, np.float32)
        cat = lambda a, b: np.ascontiguousarray(np.concatenate([a, b]))
        boxes.append(_box(cat(xf, xs), cat(vf, vs), cat(pf, ps), cat(df, dss), origin, lo, hi,
                          vis))
    return synth.Workload("near-luminal", nside, eta0, boxes)


@pytest.fixture(scope="module")
def nl():
    w = workload()
    pix = np.arange(w.npix)
    say("near-luminal oracle map")
    ref = oracle.theta_pixels(w.nside, pix, w.eta0, w.boxes)
    return w, ref


def test_inputs_are_near_luminal_and_on_the_gauge(nl):
    w, _ = nl
    for bx in w.boxes:
        v = np.linalg.norm(bx.xdot.astype(np.float64), axis=1)
        fast = v > 0.95
        assert fast.sum() == 240
        for s in SPEEDS:
            assert np.sum(np.abs(v - s) < 1e-6) == 80
        xd, xp = bx.xdot.astype(np.float64), bx.xprime.astype(np.float64)
        assert np.max(np.abs(np.sum(xd * xp, 1))) < 1e-6
        assert np.max(np.abs(np.sum(xd * xd + xp * xp, 1) - 1.0)) < 1e-6


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_near_luminal_forward(B, nl, form):
    w, ref = nl
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    say(f"near-luminal forward {form}")
    sky = sky_from_workload(w, f)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    fast_kept = sum(int(np.sum(oracle.kept(w.eta0, b)[:240])) for b in w.boxes)
    say(f"near-luminal {form} {e} near_steps={st['near_steps']} fast kept={fast_kept}")
    assert fast_kept >= 100
    if form == "fp64":
        assert e["rel_rms"] <= FP64_TOL and e["rel_max"] <= FP64_TOL, e
    else:
        # every kept fast segment is flagged: its steps take the FP64 path
        assert st["near_steps"] >= fast_kept
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def test_near_luminal_pixels_opposite_the_velocity(B, nl):
    """The pixels whose direction is opposite a fast segment's velocity
    (where b = 1 + n.Xdot is smallest): FP32C against the oracle on those
    pixels alone, with the bar taken relative to their own values."""
    w, ref = nl
    pix = []
    for bx in w.boxes:
        v = bx.xdot[:240].astype(np.float64)
        pix.append(oracle.ang2pix(w.nside, -v))
    pix = np.unique(np.concatenate(pix))
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    m = sky.render().cpu().numpy()
    e = err_metrics(m[pix], ref[pix])
    say(f"opposite-velocity pixels ({pix.size}): {e}")
    assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def test_near_luminal_adjoint(B, nl):
    w, _ = nl
    g = np.random.default_rng(9).standard_normal(w.npix)
    nseg = sum(b.n for b in w.boxes)
    say("near-luminal oracle gradient")
    ref = oracle.grad(w.nside, np.arange(w.npix), g, w.eta0, w.boxes, np.arange(nseg))
    absref = oracle.grad(w.nside, np.arange(w.npix), g, w.eta0, w.boxes, np.arange(nseg),
                         absolute=True)
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    grads = sky.backward(torch.from_numpy(g).cuda())
    got = np.concatenate([np.concatenate([a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy(),
                                          d.cpu().numpy()[:, None]], 1)
                          for a, b, c, d in grads])
    kept = np.concatenate([oracle.kept(w.eta0, b) for b in w.boxes])
    assert np.all(got[~kept] == 0.0)
    e = grad_group_errors(got[kept], ref[kept])
    es = grad_segment_errors(got[kept], ref[kept], absref[kept])
    say(f"near-luminal adjoint: group {e}; per segment (units of the bar) {es}")
    assert max(e.values()) <= GRAD_TOL, e
    assert max(es.values()) <= SEG_REL, es
    sky.close()
