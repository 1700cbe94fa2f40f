"""GPU parity of the hand-written adjoint against the oracle's gradient.

csmap_backward returns dL/d(x_rel, xdot, xprime, dsigma) of every segment for
a map cotangent dL/dTheta_p.  The oracle differentiates the same Eq. (1)-(2)
sum in FP64 (its gradient is itself pinned against finite differences in the
CPU suite).  Bars: relative L2 error <= 1e-4 per parameter group, and per
checked segment and group |got - ref| <= 1e-4 |ref| + 2e-5 |abs|, where abs
sums the pixels' contributions in absolute value (the sum's own scale before
its terms cancel; the FP32 form's per-term error is at most about 1.2e-5)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import SEG_REL, grad_group_errors, grad_segment_errors, sky_from_workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRAD_TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    return binding


def check_grads(got, ref, absref, what):
    """Both bars on the kept segments (rows of 10 components); returns the
    group errors."""
    e = grad_group_errors(got, ref)
    es = grad_segment_errors(got, ref, absref)
    say(f"{what}: group L2 {e}; per segment (units of the bar) {es}")
    assert np.all(np.isfinite(got))
    assert max(e.values()) <= GRAD_TOL, e
    assert max(es.values()) <= SEG_REL, es
    return e


def oracle_grads(w, pix, g, sel):
    return (oracle.grad(w.nside, pix, g, w.eta0, w.boxes, sel),
            oracle.grad(w.nside, pix, g, w.eta0, w.boxes, sel, absolute=True))


def gpu_grads(sky, g):
    grads = sky.backward(torch.from_numpy(g).cuda())
    rows = []
    for gx, gxd, gxp, gds in grads:
        rows.append(np.concatenate([gx.cpu().numpy(), gxd.cpu().numpy(), gxp.cpu().numpy(),
                                    gds.cpu().numpy()[:, None]], axis=1))
    return np.concatenate(rows, axis=0)


def mixed_small():
    eta0 = 3.0
    boxes = [
        synth.make_box(150, 41, origin=(-0.5, -0.5, -0.5), eta_lo=2.2, eta_hi=3.0, dtype=np.float32),
        synth.make_box(97, 42, origin=(0.8, -0.4, 0.2), eta_lo=0.9, eta_hi=1.6, dtype=np.float32,
                       vis=synth.VIS_BOX),
        synth.make_box(70, 43, origin=(-1.9, 0.4, -0.6), eta_lo=0.0, eta_hi=3.0, dtype=np.float32,
                       vis=synth.VIS_CAP, cap_dir=np.array([-0.8, 0.6, 0.0]), cap_cos=0.7),
    ]
    return synth.Workload("adj-mixed", 16, eta0, boxes)


@pytest.mark.parametrize("split", [0, 1, 3])
def test_adjoint_mixed_rules_random_cotangent(B, split):
    w = mixed_small()
    g = np.random.default_rng(5).standard_normal(w.npix)
    nseg = sum(b.n for b in w.boxes)
    say(f"adjoint mixed split={split}")
    ref, absref = oracle_grads(w, np.arange(w.npix), g, np.arange(nseg))
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C, {B.CSMAP_OPT_ADJ_SPLIT: split})
    got = gpu_grads(sky, g)
    kept = np.concatenate([oracle.kept(w.eta0, b) for b in w.boxes])
    assert np.all(got[~kept] == 0.0)
    check_grads(got[kept], ref[kept], absref[kept], f"adjoint mixed split={split}")
    sky.close()


def test_adjoint_of_quadratic_loss_reduced_config4(B):
    """L = sum_p w_p Theta_p^2 on a reduced copy of the differentiation
    workload (Nside=32, 2 boxes x 200 segments): cotangent 2 w Theta from the
    oracle's own map, gradient against the oracle's gradient."""
    full = synth.config4(nseg=200, nside=32, nbox=2)
    pix = np.arange(full.npix)
    theta = oracle.theta_pixels(full.nside, pix, full.eta0, full.boxes)
    wts = synth.config4_weights(full.npix)
    g = 2.0 * wts * theta
    ref, absref = oracle_grads(full, pix, g, np.arange(400))
    sky = sky_from_workload(full, B.CSMAP_FORM_FP32C)
    got = gpu_grads(sky, g)
    kept = np.concatenate([oracle.kept(full.eta0, b) for b in full.boxes])
    check_grads(got[kept], ref[kept], absref[kept], "reduced config4")
    sky.close()


def test_adjoint_config4_full_size_sampled(B):
    """Nside=1024, 8 boxes x 50,000 segments: the adjoint of every segment
    for a Gaussian cotangent, checked on 64 sampled segments against the
    oracle (each over all 12.6M pixels)."""
    w = synth.config4()
    g = synth.config4_weights(w.npix)
    sel = synth.sample_pixels(400_000, 64, seed=210)   # 64 distinct segment indices
    say("config4 gpu adjoint")
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    got = gpu_grads(sky, g)
    st = sky.stats()
    say(f"config4 adjoint ms={st['ms_backward']:.1f}")
    say("config4 oracle gradient on 64 segments")
    ref, absref = oracle_grads(w, np.arange(w.npix), g, sel)
    check_grads(got[sel], ref, absref, "config4 64 segments")
    sky.close()


@pytest.mark.parametrize("tiny", [0.0, 1e-30])
def test_adjoint_at_zero_and_tiny_dsigma(B, tiny):
    """Segments with dsigma = 0 (and 1e-30): Eq. (1) is linear in dsigma, so
    dL/d(dsigma) is the map sum per unit dsigma (finite), and every other
    component carries a factor dsigma (zero at 0)."""
    w = mixed_small()
    for k, bx in enumerate(w.boxes):
        ds = bx.dsigma.copy()
        ds[k::5] = np.float32(tiny)
        bx.dsigma = ds
    g = np.random.default_rng(6).standard_normal(w.npix)
    nseg = sum(b.n for b in w.boxes)
    ref, absref = oracle_grads(w, np.arange(w.npix), g, np.arange(nseg))
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    got = gpu_grads(sky, g)
    kept = np.concatenate([oracle.kept(w.eta0, b) for b in w.boxes])
    zero = np.concatenate([b.dsigma == np.float32(tiny) for b in w.boxes]) & kept
    assert zero.sum() >= 10
    assert np.all(np.abs(got[zero, 9]) > 0.0)
    if tiny == 0.0:
        assert np.all(got[zero, :9] == 0.0)
    check_grads(got[kept], ref[kept], absref[kept], f"dsigma={tiny}")
    sky.close()
