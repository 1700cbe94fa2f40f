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
