"""Shared helpers of the test-suite (no map arithmetic here)."""
import numpy as np


def err_metrics(got, ref):
    """Error norms over a set of pixels (Theta/GU units): relative rms and
    relative max (normalised by the reference's rms and max), and the plain
    max-abs and rms differences."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    nref2 = float(np.sqrt(np.sum(ref * ref)))
    mref = float(np.max(np.abs(ref))) if ref.size else 0.0
    return {
        "rel_rms": float(np.sqrt(np.sum(d * d))) / nref2 if nref2 > 0 else float(np.sqrt(np.sum(d * d))),
        "rel_max": float(np.max(np.abs(d))) / mref if mref > 0 else float(np.max(np.abs(d), initial=0.0)),
        "max_abs": float(np.max(np.abs(d), initial=0.0)),
        "rms": float(np.sqrt(np.mean(d * d))) if d.size else 0.0,
    }


def sky_from_workload(workload, form, options=None, boxes=None):
    """Create a libcsmap sky holding the workload's boxes (device copies)."""
    import torch
    from paper_1204_5041_amd import binding as B
    sky = B.Sky(workload.nside, workload.eta0, form)
    for opt, val in (options or {}).items():
        sky.set_option(opt, val)
    for bx in (workload.boxes if boxes is None else boxes):
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
             for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
        kw = {}
        if bx.cap_dir is not None:
            kw["cap_dir"] = tuple(float(v) for v in bx.cap_dir)
            kw["cap_cos"] = float(bx.cap_cos)
        sky.add_box(*t, origin=tuple(float(v) for v in bx.origin), eta_lo=bx.eta_lo,
                    eta_hi=bx.eta_hi, vis=bx.vis, ext=tuple(float(v) for v in bx.ext), **kw)
    return sky


GRAD_GROUPS = (("x_rel", slice(0, 3)), ("xdot", slice(3, 6)), ("xprime", slice(6, 9)),
               ("dsigma", slice(9, 10)))


def grad_group_errors(got, ref):
    """Relative L2 error of each parameter group (x_rel, xdot, xprime, dsigma)
    over all checked segments (rows of 10 gradient components)."""
    out = {}
    for name, sl in GRAD_GROUPS:
        d = got[:, sl] - ref[:, sl]
        out[name] = float(np.linalg.norm(d) / max(np.linalg.norm(ref[:, sl]), 1e-300))
    return out


# Per-segment bar: |got_s - ref_s| <= 1e-4 |ref_s| + 2e-5 |abs_s| per group,
# abs_s being the sum over pixels of each component's contributions in
# absolute value (oracle.grad(..., absolute=True)).  A segment's gradient is a
# sum over pixels whose terms can cancel to far below their size; the FP32
# form's terms each carry a relative error up to about 1.2e-5 (its far pair
# form rounds n.P/R against 1 - n.P/R >= 5e-3), so 2e-5 |abs_s| bounds what
# rounding of the terms alone can leave in such a sum.
SEG_REL, SEG_ABS = 1e-4, 2e-5


def grad_segment_errors(got, ref, absref):
    """Largest per-segment error of each parameter group in units of the
    per-segment bar, |got_s - ref_s| / (|ref_s| + (SEG_ABS/SEG_REL) |abs_s|),
    to be compared with SEG_REL."""
    out = {}
    k = SEG_ABS / SEG_REL
    for name, sl in GRAD_GROUPS:
        nref = np.linalg.norm(ref[:, sl], axis=1)
        nabs = np.linalg.norm(absref[:, sl], axis=1)
        nd = np.linalg.norm(got[:, sl] - ref[:, sl], axis=1)
        out[name] = float(np.max(nd / np.maximum(nref + k * nabs, 1e-300))) if nd.size else 0.0
    return out


def ring_sparse_alm(nside, lmax, hmap, rings):
    """a_lm of a map that is zero outside `rings` (1-based RING ring
    indices): (4 pi / Npix) sum_r lambda_lm(z_r) F_m(r), with the ring's
    Fourier sums F_m(r) = sum_j x_j e^{-i m phi_j} taken from numpy's FFT of
    the ring (phi_j = phi_0 + 2 pi j / L, phi_0 and z_r from the oracle's
    pixel direction of the ring's first pixel) and lambda from the oracle."""
    import oracle
    N = nside
    npix = 12 * N * N
    size = oracle.alm_size(lmax)
    mm = np.arange(lmax + 1)

    def one_ring(r):
        alm = np.zeros(size, dtype=np.complex128)
        if r < N:
            L, first = 4 * r, 2 * r * (r - 1)
        elif r <= 3 * N:
            L, first = 4 * N, 2 * N * (N - 1) + (r - N) * 4 * N
        else:
            k = 4 * N - r
            L, first = 4 * k, npix - 2 * k * (k + 1)
        x = hmap[first:first + L]
        v = oracle.pix2vec(nside, np.array([first]))[0]
        z, s, phi0 = v[2], float(np.hypot(v[0], v[1])), float(np.arctan2(v[1], v[0]))
        X = np.fft.fft(x)
        F = X[mm % L] * np.exp(-1j * mm * phi0)
        for m in range(lmax + 1):
            lam = oracle.lambda_lm(lmax, m, z, s)
            i0 = oracle.alm_index(lmax, m, m)
            alm[i0:i0 + lmax + 1 - m] = lam * F[m]
        return alm

    from concurrent.futures import ThreadPoolExecutor
    total = np.zeros(size, dtype=np.complex128)
    with ThreadPoolExecutor(max_workers=8) as ex:
        for part in ex.map(one_ring, rings):
            total += part
    return total * (4 * np.pi / npix)

