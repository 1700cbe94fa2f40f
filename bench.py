"""Benchmark of the all-sky string ISW map maker on one MI355X.

Workload (the Nside=2048 throughput case): HEALPix Nside=2048 (50,331,648
RING pixels), boxes of 400,000 FP32 segments (box b: seed 100+b, side 1 Gpc,
nearest distance 0.1 * 140^(b/63) Gpc, eta0 = 16 Gpc, every segment kept,
every pixel sees every box).  One step renders the full sky from one box
(2.01e13 pixel-segment pairs): the light-cone precompute kernels and the
pair kernel, FP32C form.  Step k uses box W+k (warm-up steps use boxes
0..W-1), so every timed step works on fresh data already resident in HBM.

Printed: one JSON line with pairs/s of the FP32C form, the FP64 form's
pairs/s on one box, the forward kernel's achieved FLOP/s against the FP32
vector peak (36 algorithmic FLOP per pair), the FP64 CPU oracle timed on a
sample of the same workload on this host, and the error of both GPU forms
against the oracle on that sample (the last timed box).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel-segment pairs/s (FP32 vs FP64, Nside=2048) + % of VALU peak"
FLOP_PER_PAIR = 36          # algorithmic count of one Eq. (1) term
# Algorithmic count of one pair's contribution to the adjoint's 14 sums (far
# form, FMA = 2): w, a, b (17), n - P/R (3), kappa-weighted dot products t1,
# t2 (4), m and the term f (4), the reciprocal of b w (2), the coefficients
# and updates of the 14 sums (37).
ADJ_FLOP_PER_PAIR = 67
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector peak
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector peak
NSIDE = 2048
NSEG = 400_000


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sky(B, torch, b, form, nseg, nside):
    import synth
    box = synth.config2_box(b, nseg)
    sky = B.Sky(nside, 16.0, form)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
         for a in (box.x_rel, box.xdot, box.xprime, box.dsigma)]
    sky.add_box(*t, origin=tuple(box.origin), eta_lo=box.eta_lo, eta_hi=box.eta_hi)
    return sky, box


def measured_traffic(kernel):
    """HBM bytes (per launch, or per step for the stacking stage) of a kernel
    from the committed rocprofv3 counter runs, if they were taken on the
    kernel's current sources (its record holds their SHA-256)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    k = json.load(open(path)).get("kernels", {}).get(kernel)
    if k is None or _sources_sha(k["sources"]) != k["sources_sha256"]:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def cpu_baseline(box, b, nside, pix):
    """The oracle on sampled pixels of one box: its rate, and its values."""
    import oracle
    t0 = time.perf_counter()
    ref = oracle.theta_pixels(nside, pix, 16.0, [box])
    dt = time.perf_counter() - t0
    pairs = len(pix) * box.n
    return {"value": pairs / dt, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{len(pix)} random pixels x box {b} ({box.n:,} segments) at Nside={nside}: "
                      f"{pairs:.3e} pairs in {dt:.1f} s"}, ref


def err_metrics(got, ref):
    """Errors in Theta/GU over the sampled pixels: relative rms and relative
    max (normalised by the reference's rms and max), max-abs and rms."""
    d = np.asarray(got, dtype=np.float64) - ref
    return {"rel_rms": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "rel_max": float(np.max(np.abs(d)) / np.max(np.abs(ref))),
            "max_abs": float(np.max(np.abs(d))), "rms": float(np.sqrt(np.mean(d * d)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nseg", type=int, default=NSEG)
    ap.add_argument("--nside", type=int, default=NSIDE)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="config2: leave out the batched 256-box Nside=4096 measurement that "
                         "follows the headline steps")
    ap.add_argument("--cpu-pixels", type=int, default=40000)
    ap.add_argument("--workload", default="config2",
                    choices=["config2", "config3", "config4", "events", "alm", "stack", "flat",
                             "counters", "hbm"],
                    help="config2: the headline Nside=2048 line (default); config3: the "
                         "batched uneven 256-box Nside=4096 sky; config4: forward + adjoint at "
                         "Nside=1024; events: light-cone event recording from slab-start "
                         "snapshots (25.6M segments); alm: spherical-harmonic analysis and "
                         "C_l of a rendered Nside=2048 map, lmax=4096; stack: healpix-cone "
                         "stacking of 1024 runs x 3 axes into the 3072 Nside_c=16 cones plus "
                         "12 Nside_c=1 cones (light-cone stage of 3084 placed boxes); flat: "
                         "flat-sky small-angle map of a 7.2 degree 1024^2 patch from 2M "
                         "segments; counters: one launch each of a known-FMA probe (FP32, "
                         "FP64), the bench step's k_fwd32 and k_fwd64, the config4 adjoint "
                         "and map2alm, for hardware counter runs; hbm: the streaming rate of "
                         "a plain device copy, the yardstick for the HBM-bound kernels")
    ap.add_argument("--stack-seg", type=int, default=200_000,
                    help="stack: segments per simulation run")
    ap.add_argument("--count-scale", type=float, default=1.0,
                    help="config3: scale of the per-box segment counts")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("TRACE_DIR", "PMC_A_DIR", "PMC_B_DIR",
                                                              "LAUNCHES_JSON"),
                    help="no GPU work: summarise the rocprofv3 kernel-trace and the two --pmc "
                         "runs of --workload counters (their output directories, and the JSON "
                         "line that run printed) into the per-kernel VALU record")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="before the timed region, run one plain device copy of this many "
                         "MiB (a known-size reference for hardware traffic counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        print(json.dumps(summarize_counters(*args.summarize_counters), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described, not run).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_5041_amd import binding as B
    assert torch.cuda.is_available(), "no GPU visible"
    if args.copy_calib_mib > 0:
        # One device copy of known size, before any workload, so that traffic
        # counters can be scaled by what they read for it.
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "config3":
        return bench_config3(args, B, torch)
    if args.workload == "config4":
        return bench_config4(args, B, torch)
    if args.workload == "events":
        return bench_events(args, B, torch)
    if args.workload == "alm":
        return bench_alm(args, B, torch)
    if args.workload == "stack":
        return bench_stack(args, B, torch)
    if args.workload == "flat":
        return bench_flat(args, B, torch)
    if args.workload == "counters":
        return bench_counters(args, B, torch)
    if args.workload == "hbm":
        return bench_hbm(args, torch)

    W, K = args.warmup, args.steps
    _log(f"bench: generating {W + K} boxes of {args.nseg:,} segments")
    skies = [make_sky(B, torch, b, B.CSMAP_FORM_FP32C, args.nseg, args.nside) for b in range(W + K)]
    npix = 12 * args.nside * args.nside
    maps = torch.empty(npix, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    for i in range(W):
        _log(f"bench: warm-up step {i}")
        skies[i][0].render(maps)
    torch.cuda.synchronize()

    fwd_ms, pairs = [], 0
    t0 = time.perf_counter()
    for k in range(K):
        sky = skies[W + k][0]
        sky.render(maps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # The last timed map, at the pixels the oracle will evaluate.
    import synth
    last = W + K - 1
    pix = synth.sample_pixels(npix, args.cpu_pixels, seed=98)
    pix_t = torch.from_numpy(pix).cuda()
    got32 = maps[pix_t].cpu().numpy()
    for k in range(K):
        st = skies[W + k][0].stats()
        fwd_ms.append(st["ms_forward"])
        pairs += st["pairs"]
        _log(f"bench: step {k} box {W + k}: pairs={st['pairs']} forward {st['ms_forward']:.1f} ms "
             f"precompute {st['ms_precompute']:.2f} ms fp64_steps={st['near_steps']} "
             f"mid_steps={st['mid_steps']} steps={st['steps']}")
    value = pairs / elapsed
    kern_s = float(np.mean(fwd_ms)) / 1e3
    pairs_per_step = pairs / K
    achieved = FLOP_PER_PAIR * pairs_per_step / kern_s / 1e12
    cfg = {k: v for k, v in skies[W][0].stats().items()
           if k in ("pix_per_lane", "waves", "schedule", "graph", "chunk", "near_w", "far_w",
                    "tiling")}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Nside={args.nside} full sky, one box of {args.nseg:,} FP32 "
                               f"segments per step (boxes of the 64-box 0.1-14 Gpc "
                               f"throughput set), FP32C form",
                   "nside": args.nside, "segments_per_step": args.nseg,
                   "pairs_per_step": pairs_per_step, "tile": cfg},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic("k_fwd32") if args.nseg == NSEG and args.nside == NSIDE
                     else None,
                     "kernel": "k_fwd32", "kernel_ms": kern_s * 1e3,
                     "flop_per_pair": FLOP_PER_PAIR},
    }
    if args.nseg == NSEG and args.nside == NSIDE:
        # Hardware-counted FLOP of this launch (rocprofv3 counters of the same
        # kernel on the same box size), over the launch time measured here.
        hw = measured_valu("k_fwd32", kern_s * 1e3)
        out["roofline"]["hw"] = hw
        out["roofline"]["hw_tflops"] = hw["fp32_tflops"] if hw else None
    del skies
    torch.cuda.synchronize()

    got64 = None
    if not args.no_fp64:
        _log(f"bench: FP64 form, box {last}")
        sky64, _ = make_sky(B, torch, last, B.CSMAP_FORM_FP64, args.nseg, args.nside)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sky64.render(maps)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t0
        st = sky64.stats()
        v64 = st["pairs"] / e64
        a64 = FLOP_PER_PAIR * st["pairs"] / (st["ms_forward"] / 1e3) / 1e12
        out["fp64"] = {"value": v64, "unit": "pairs/s", "ms_per_step": e64 * 1e3,
                       "kernel_ms": st["ms_forward"], "achieved_tflops": a64,
                       "frac_fp64_peak": a64 / FP64_PEAK_TFLOPS}
        if args.nseg == NSEG and args.nside == NSIDE:
            out["fp64"]["hw"] = measured_valu("k_fwd64", st["ms_forward"])
        got64 = maps[pix_t].cpu().numpy()
        out["speedup_fp32_over_fp64"] = value / v64
        sky64.close()

    if not args.no_cpu:
        _log("bench: CPU oracle baseline")
        box = synth.config2_box(last, args.nseg)
        out["cpu_baseline"], ref = cpu_baseline(box, last, args.nside, pix)
        acc = {"box": last, "pixels": int(len(pix)), "unit": "Theta/GU",
               "fp32c": err_metrics(got32, ref)}
        if got64 is not None:
            acc["fp64"] = err_metrics(got64, ref)
        out["accuracy_vs_oracle"] = acc

    if not args.no_batched:
        # The batched uneven workload (256 boxes, Nside 4096, cap visibility),
        # in the form the batched path is meant to run: autotuned, one
        # persistent launch captured in a graph and replayed once.
        bt = batched_config3(B, torch, steps=1, per_box=False, cpu=False)
        out["batched_config3"] = {k: bt[k] for k in (
            "value", "unit", "ms_per_step", "kernel_ms", "pairs", "segments", "achieved_tflops",
            "frac_fp32_peak", "tile", "autotune_s", "accuracy_vs_oracle")}
        out["batched_config3"]["workload"] = ("Nside=4096, 256 boxes, lognormal counts "
                                              "(22.1M FP32 segments), caps of 0.1%-5% of the sky")

    print(json.dumps(out), flush=True)


def _sky_from(B, torch, w, form):
    sky = B.Sky(w.nside, w.eta0, form)
    for bx in w.boxes:
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
             for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
        kw = {}
        if bx.cap_dir is not None:
            kw = {"cap_dir": tuple(float(v) for v in bx.cap_dir), "cap_cos": float(bx.cap_cos)}
        sky.add_box(*t, origin=tuple(float(v) for v in bx.origin), eta_lo=bx.eta_lo,
                    eta_hi=bx.eta_hi, vis=bx.vis, ext=tuple(float(v) for v in bx.ext), **kw)
    return sky


def batched_config3(B, torch, steps=1, count_scale=1.0, per_box=True, cpu=True):
    """256 boxes of lognormal size, each seen by a cap of 0.1%-5% of an
    Nside=4096 sky: autotuned launch shape, then one persistent launch over
    per-tile box lists captured in a graph (the first render captures it,
    `steps` replays are timed); accuracy against the oracle on 4,000 pixels
    drawn inside the caps; optionally compared with one launch per box."""
    import synth
    _log("bench config3: generating 256 boxes")
    w = synth.config3(count_scale=count_scale)
    _log(f"bench config3: {sum(b.n for b in w.boxes):,} segments; uploading")
    sky = _sky_from(B, torch, w, B.CSMAP_FORM_FP32C)
    out = torch.empty(w.npix, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    _log("bench config3: autotune")
    t0 = time.perf_counter()
    sky.autotune(None)
    tune_s = time.perf_counter() - t0
    _log(f"bench config3: autotune done in {tune_s:.1f} s: {sky.stats()}")
    sky.set_option(B.CSMAP_OPT_SCHEDULE, 1)
    sky.set_option(B.CSMAP_OPT_GRAPH, 1)
    sky.render(out)                               # capture + warm-up
    torch.cuda.synchronize()
    _log(f"bench config3: warm-up render done ({sky.stats()['ms_forward']:.0f} ms)")
    K = max(1, steps)
    t0 = time.perf_counter()
    for _ in range(K):
        sky.render(out)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / K
    st = sky.stats()
    res = {"metric": "config3 batched pairs/s", "value": st["pairs"] / el, "unit": "pairs/s",
           "ms_per_step": el * 1e3, "kernel_ms": st["ms_forward"], "pairs": st["pairs"],
           "kept": st["kept"], "segments": st["segments"],
           "tile": {k: st[k] for k in ("pix_per_lane", "waves", "schedule", "graph", "tiling",
                                       "near_w", "far_w")},
           "fp64_steps": st["near_steps"], "mid_steps": st["mid_steps"], "steps": st["steps"],
           "autotune_s": tune_s}
    res["achieved_tflops"] = FLOP_PER_PAIR * res["value"] / 1e12
    res["frac_fp32_peak"] = res["achieved_tflops"] / FP32_PEAK_TFLOPS
    pix = _cap_pixels(w, 4000, seed=396)
    res["accuracy_vs_oracle"], dt = _sampled_accuracy(torch, w, out, len(pix), seed=397, pix=pix)
    res["accuracy_vs_oracle"]["pixels_drawn"] = "inside the boxes' caps"
    if cpu:
        res["cpu_baseline"] = _sampled_cpu_baseline(w, st["pairs"], 4000, None)
    if per_box:
        _log(f"bench config3: batched render {el * 1e3:.0f} ms; per-box launches next")
        sky.set_option(B.CSMAP_OPT_GRAPH, 0)
        sky.set_option(B.CSMAP_OPT_SCHEDULE, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sky.render(out)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t0
        res["per_box_launches_pairs_per_s"] = sky.stats()["pairs"] / el2
        res["speedup_batched_over_per_box"] = el2 / el
    sky.close()
    return res


def _cap_pixels(w, count, seed):
    """Pixels drawn inside the boxes' caps (a box chosen with probability
    proportional to its cap's area, a direction uniform in that cap, its
    RING pixel by the oracle's ang2pix), so that each sees at least one box
    unless it sits on a cap's edge."""
    import oracle
    rng = np.random.default_rng(seed)
    area = np.array([1.0 - b.cap_cos for b in w.boxes])
    pick = rng.choice(len(w.boxes), size=count, p=area / area.sum())
    dirs = np.empty((count, 3))
    for i, b in enumerate(pick):
        bx = w.boxes[b]
        c = bx.cap_dir / np.linalg.norm(bx.cap_dir)
        a = np.cross(c, [1.0, 0.0, 0.0] if abs(c[0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        bb = np.cross(c, a)
        ct = rng.uniform(bx.cap_cos, 1.0)
        st = math.sqrt(max(0.0, 1.0 - ct * ct))
        ph = rng.uniform(0.0, 2.0 * math.pi)
        dirs[i] = ct * c + st * (math.cos(ph) * a + math.sin(ph) * bb)
    return np.unique(oracle.ang2pix(w.nside, dirs))


def bench_config3(args, B, torch):
    print(json.dumps(batched_config3(B, torch, args.steps, args.count_scale)), flush=True)


def _sampled_accuracy(torch, w, gpu_map, count, seed, pix=None):
    """Errors of a rendered map against the oracle on `count` random pixels
    (or on the given pixels)."""
    import oracle
    import synth
    if pix is None:
        pix = synth.sample_pixels(w.npix, count, seed=seed)
    got = gpu_map[torch.from_numpy(pix).cuda()].cpu().numpy()
    _log(f"bench: oracle on {count} sampled pixels")
    t0 = time.perf_counter()
    ref = oracle.theta_pixels(w.nside, pix, w.eta0, w.boxes)
    dt = time.perf_counter() - t0
    acc = {"pixels": int(count), "unit": "Theta/GU"}
    acc.update(err_metrics(got, ref))
    return acc, dt


def _sampled_cpu_baseline(w, pairs, count, dt):
    """The oracle's rate on the same map, from its time on `count` pixels
    drawn uniformly from the map (so that the time scales to the whole map in
    expectation, boxes seen by part of the sky included); timed here when dt
    is None."""
    import oracle
    import synth
    if dt is None:
        pix = synth.sample_pixels(w.npix, count, seed=397)
        t0 = time.perf_counter()
        oracle.theta_pixels(w.nside, pix, w.eta0, w.boxes)
        dt = time.perf_counter() - t0
    full_s = dt * w.npix / count
    return {"value": pairs / full_s, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{count} random pixels of the Nside={w.nside} map, all {len(w.boxes)} boxes "
                      f"({sum(b.n for b in w.boxes):,} segments): {dt:.1f} s, scaled to the "
                      f"{w.npix:,}-pixel map ({full_s:.3e} s)"}


HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
EVENT_BYTES = 24 + 33       # read x_rel, xdot (FP32); write position, D (FP64), keep (byte)


def bench_events(args, B, torch):
    """Light-cone event recording: 25.6M FP32 segments (the segment count of
    the 64-box Nside=2048 set) of a 1 Gpc box at ~5 Gpc, known at the start of
    the slab [11, 11.6) of eta0 = 16, each moved along its velocity to its
    crossing of the past light cone.  The kernel streams 57 bytes per
    segment, so its bound is HBM bandwidth."""
    import oracle
    import synth
    n = 25_600_000
    _log(f"bench events: generating {n:,} segments")
    x, xd, _, _ = synth.segments(n, 510, np.float32)
    rng = np.random.default_rng(511)
    v = rng.uniform(0.0, 0.95, n).astype(np.float32)
    xd = (xd / np.linalg.norm(xd, axis=1, keepdims=True) * v[:, None]).astype(np.float32)
    origin = (3.7, -2.1, 1.4)
    eta0, eta_lo, eta_hi = 16.0, 11.0, 11.6
    xt, vt = torch.from_numpy(x).cuda(), torch.from_numpy(xd).cuda()
    pos, d, keep = B.cone_events(xt, vt, origin, eta0, eta_lo, eta_hi)   # warm-up
    torch.cuda.synchronize()
    K = max(1, args.steps) * 10
    # The timed launches go straight to the C entry point with the outputs
    # allocated once, so the host issues them faster than the device runs
    # them and they run back to back; one pair of HIP events on the stream
    # they run on (torch's current stream) brackets all K.
    pos = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    keep8 = torch.empty(n, dtype=torch.uint8, device="cuda")
    box = B.csmap_box()
    box.n, box.dtype = n, B.CSMAP_F32
    box.x_rel, box.xdot = xt.data_ptr(), vt.data_ptr()
    box.origin = (B.ctypes.c_double * 3)(*origin)
    box.eta_lo, box.eta_hi = eta_lo, eta_hi
    sptr = torch.cuda.current_stream().cuda_stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(K):
        B.csmap_cone_events(box, eta0, pos.data_ptr(), d.data_ptr(), keep8.data_ptr(), sptr)
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / K
    kern = e0.elapsed_time(e1) / 1e3 / K
    keep = keep8.view(torch.bool)
    gbs = EVENT_BYTES * n / kern / 1e9
    res = {"metric": "light-cone events recorded per second (segments/s)", "value": n / kern,
           "unit": "segments/s", "segments": n, "kept": int(keep.sum().item()),
           "ms_per_launch": kern * 1e3, "wall_ms_per_launch": wall * 1e3,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "bytes_per_segment": EVENT_BYTES,
                        "traffic": measured_traffic("k_cone_events")}}
    # Agreement with the oracle: on all segments when the oracle is timed
    # (a few seconds on the host's cores), else on a sample of 200,000.
    if args.no_cpu:
        sel = synth.sample_pixels(n, 200_000, seed=512)
        xs, vs = x[sel], xd[sel]
    else:
        sel = slice(None)
        xs, vs = x, xd
    _log("bench events: oracle")
    t0 = time.perf_counter()
    rp, rd, rk = oracle.cone_events(xs, vs, np.array(origin), eta0, eta_lo, eta_hi)
    dt = time.perf_counter() - t0
    k = keep.cpu().numpy()[sel]
    dd = d.cpu().numpy()[sel]
    both = k & rk
    res["accuracy_vs_oracle"] = {"segments": int(len(rk)),
                                 "keep_mismatches": int(np.sum(k != rk)),
                                 "max_abs_delta_error": float(np.max(np.abs(dd[both] - rd[both])))}
    if not args.no_cpu:
        res["cpu_baseline"] = {"value": n / dt, "unit": "segments/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"the whole workload ({n:,} segments) in {dt:.2f} s"}
    print(json.dumps(res), flush=True)


STACK_RAW_BYTES = 40    # FP32 x_rel, Xdot, X', dsigma read once per placed segment
STACK_REC_BYTES = 100   # per kept segment: 64-byte record, FP64 direction + R, index


def bench_stack(args, B, torch):
    """Healpix-cone stacking: the 3072 cones of the Nside_c=16 grid between
    z=1089 and z=36 filled by 1024 runs used three times each (one per box
    axis), plus the 12 Nside_c=1 cones down to z=0.2, every run holding
    --stack-seg FP32 segments in its own box coordinates.  Each box is
    placed by csmap_cone_place and added with csmap_add_cone_box; one step
    is the light-cone stage of all 3084 boxes (csmap_precompute): rotation
    onto the sky in FP64, slab test, cone test (device ang2pix), compaction
    and record emission.  It streams 40 bytes per placed segment and writes
    100 bytes per kept one, so its bound is HBM bandwidth."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import synth
    plans = [synth.stack_highz(args.stack_seg), synth.stack_lowz(args.stack_seg)]
    sky = B.Sky(16, plans[0].eta0, B.CSMAP_FORM_FP32C)
    t0 = time.perf_counter()
    runs_host = {}
    nbox = 0
    for p in plans:
        _log(f"bench stack: generating {p.nruns} runs of {p.seg_per_run:,} segments ({p.name})")
        with ThreadPoolExecutor(16) as ex:
            data = list(ex.map(lambda r: p.run(r), range(p.nruns)))
        dev = [[torch.from_numpy(a).cuda() for a in d] for d in data]
        runs_host[p.name] = data[:48]
        del data
        for cone, r, axis in p.uses:
            c, origin, slack = B.cone_place(p.nside_c, cone, axis, p.r_in, p.r_out, p.side)
            assert slack >= 0, (p.name, cone)
            sky.add_box(*dev[r], origin=tuple(origin), eta_lo=p.eta_lo, eta_hi=p.eta_hi, cone=c)
            nbox += 1
        torch.cuda.synchronize()
        del dev
    t_add = time.perf_counter() - t0
    nseg = sum(len(p.uses) for p in plans) * args.stack_seg
    _log(f"bench stack: {nbox} boxes, {nseg:,} placed segments, set-up {t_add:.1f} s")
    for _ in range(max(1, args.warmup)):
        sky.precompute()
    torch.cuda.synchronize()
    K = max(1, args.steps)
    kern, walls = [], []
    for _ in range(K):
        w0 = time.perf_counter()
        sky.precompute()
        st = sky.stats()   # synchronises
        walls.append(time.perf_counter() - w0)
        kern.append(st["ms_precompute"] / 1e3)
    kept = st["kept"]
    k_avg = sum(kern) / K
    byts = STACK_RAW_BYTES * nseg + STACK_REC_BYTES * kept
    gbs = byts / k_avg / 1e9
    hz = plans[0]
    share = (4 * np.pi / (12 * hz.nside_c ** 2)) * (hz.r_out ** 3 - hz.r_in ** 3) / 3 / hz.side ** 3
    res = {"metric": "placed segments per second through healpix-cone stacking (segments/s)",
           "value": nseg / k_avg, "unit": "segments/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": k_avg * 1e3,
           "wall_ms_per_step": 1e3 * sum(walls) / K, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 geometry, fp32 records",
           "data": "synthetic", "setup_s": t_add,
           "config": {"workload": "healpix-cone stacking: 3072 Nside_c=16 cones (1024 runs x 3 "
                                  "axes) + 12 Nside_c=1 cones", "boxes": nbox,
                      "segments_per_run": args.stack_seg, "placed_segments": nseg,
                      "kept": kept, "kept_expected_high_z_share": share},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS,
                        "traffic": (measured_traffic("k_pre_count+k_pre_emit")
                                    if args.stack_seg == 200_000 else None),
                        "bytes": f"{STACK_RAW_BYTES} per placed + {STACK_REC_BYTES} per kept"}}
    if not args.no_cpu:
        # The oracle's placement and cone test on the first uses of the
        # high-z plan (runs 0..47, three axes each): its rate on this host.
        sample = [u for u in hz.uses if u[1] < 48]
        t0 = time.perf_counter()
        kept_cpu = 0
        for cone, r, axis in sample:
            x, xd, xp, ds = runs_host[hz.name][r]
            R, origin = oracle.cone_frame(hz.nside_c, cone, axis, hz.r_out, hz.side)
            P, V, T = oracle.place_segments(x, xd, xp, R, origin)
            rr = np.sqrt((P[:, 0] * P[:, 0] + P[:, 1] * P[:, 1]) + P[:, 2] * P[:, 2])
            eta = hz.eta0 - rr
            keep = (eta >= hz.eta_lo) & (eta < hz.eta_hi) & oracle.in_cone(hz.nside_c, cone, P)
            kept_cpu += int(keep.sum())
        dt = time.perf_counter() - t0
        n_cpu = len(sample) * args.stack_seg
        res["cpu_baseline"] = {"value": n_cpu / dt, "unit": "segments/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"{len(sample)} placed boxes (runs 0-47 x 3 axes), "
                                         f"{n_cpu:,} segments, {kept_cpu:,} kept, {dt:.1f} s"}
    sky.close()
    print(json.dumps(res), flush=True)


FLAT_FLOP_PER_PAIR = 10   # t - s (2), |t - s|^2 (3), u_perp.(t - s) (3), division, accumulation


def flat_vs_full(B, torch, fp):
    """A Fig. 3-style comparison on coherent strings: 40 long straight
    strings near the pole (synth.straight_strings), their flat map on the
    patch and their full-sky Eq. (1) at the same gnomonic pixel directions
    (csmap_render_dirs), both FP32C on the GPU; the relative rms difference
    per annulus around the patch centre."""
    import synth
    box = synth.straight_strings()
    sky = B.Sky(64, fp.eta0, B.CSMAP_FORM_FP32C)
    t = [torch.from_numpy(a).cuda() for a in (box.x_rel, box.xdot, box.xprime, box.dsigma)]
    sky.add_box(*t, origin=(0.0, 0.0, 0.0), eta_lo=box.eta_lo, eta_hi=box.eta_hi)
    tt = (np.arange(fp.nx) + 0.5 - fp.nx / 2) * fp.pix
    tx, ty = np.meshgrid(tt, tt)
    dirs = (fp.center[None, :] + tx.ravel()[:, None] * fp.e1[None, :] +
            ty.ravel()[:, None] * fp.e2[None, :])
    full = sky.render_dirs(torch.from_numpy(dirs).cuda()).cpu().numpy().reshape(fp.ny, fp.nx)
    ms_full = sky.stats()["ms_forward"]
    flat = sky.render_flat(fp.center, fp.e1, fp.e2, fp.nx, fp.ny, fp.pix,
                           math.cos(math.radians(20.0))).cpu().numpy()
    ms_flat = sky.stats()["ms_forward"]
    sky.close()
    rad = np.degrees(np.hypot(tx, ty))
    prof = {}
    for lo, hi in ((0.0, 1.2), (1.2, 2.4), (2.4, 3.6), (3.6, 5.2)):
        sel = (rad >= lo) & (rad < hi)
        prof[f"{lo}-{hi} deg"] = float(np.sqrt(np.mean((full - flat)[sel] ** 2) /
                                               np.mean(full[sel] ** 2)))
    return {"workload": "40 straight strings x 3,000 segments within 4 deg of the pole, "
                        "3-15 Gpc, 12 deg of arc each", "segments": int(box.n),
            "rel_rms_flat_minus_full_by_annulus": prof, "ms_full_sky_at_patch_dirs": ms_full,
            "ms_flat": ms_flat}


def bench_flat(args, B, torch):
    """Flat-sky small-angle map (Sec. II.A, Fig. 3): a 7.2 x 7.2 degree
    patch at the north pole, 1024 x 1024 pixels of 0.42', and 2,000,000 FP32
    segments in the 6 degree cap behind it between 1.4 and 15.5 Gpc.  One
    step is csmap_render_flat: the light-cone stage with the patch's
    acceptance cone, the record pass, and the FP32 pair kernel (timed with
    HIP events on the sky's stream)."""
    import oracle
    import synth
    fp = synth.flat_pencil()
    bx = fp.boxes[0]
    sky = B.Sky(64, fp.eta0, B.CSMAP_FORM_FP32C)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
         for a in (bx.x_rel, bx.xdot, bx.xprime, bx.dsigma)]
    sky.add_box(*t, origin=tuple(bx.origin), eta_lo=bx.eta_lo, eta_hi=bx.eta_hi)
    out = torch.empty((fp.ny, fp.nx), dtype=torch.float64, device="cuda")
    for _ in range(max(1, args.warmup)):
        sky.render_flat(fp.center, fp.e1, fp.e2, fp.nx, fp.ny, fp.pix, fp.accept_cos, out=out)
    torch.cuda.synchronize()
    K = max(1, args.steps)
    pair_ms, pre_ms, walls = [], [], []
    for _ in range(K):
        w0 = time.perf_counter()
        sky.render_flat(fp.center, fp.e1, fp.e2, fp.nx, fp.ny, fp.pix, fp.accept_cos, out=out)
        st = sky.stats()
        walls.append(time.perf_counter() - w0)
        pair_ms.append(st["ms_forward"])
        pre_ms.append(st["ms_precompute"])
    kept = st["kept"]
    pairs = float(fp.nx * fp.ny) * kept
    k_avg = sum(pair_ms) / K / 1e3
    step = (sum(pair_ms) + sum(pre_ms)) / K / 1e3
    tf = FLAT_FLOP_PER_PAIR * pairs / k_avg / 1e12
    res = {"metric": "flat-sky pixel-segment pairs/s (1024^2 patch, 2M segments)",
           "value": pairs / step, "unit": "pairs/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": step * 1e3,
           "wall_ms_per_step": 1e3 * sum(walls) / K, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "flat-sky 7.2 deg patch at the pole, 1024x1024 pixels, "
                                  "2,000,000 segments (1.4-15.5 Gpc, 6 deg cap)",
                      "kept": kept, "pairs_per_step": pairs,
                      "ms_light_cone_and_records": sum(pre_ms) / K,
                      "ms_pairs": sum(pair_ms) / K},
           "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": tf / FP32_PEAK_TFLOPS, "traffic": None,
                        "kernel": "k_flat32", "kernel_ms": k_avg * 1e3,
                        "flop_per_pair": FLAT_FLOP_PER_PAIR}}
    m = out.cpu().numpy()
    sky.close()
    res["fig3_style"] = flat_vs_full(B, torch, fp)
    if not args.no_cpu:
        rng = np.random.default_rng(851)
        ii = rng.integers(0, fp.nx, 60_000)
        jj = rng.integers(0, fp.ny, 60_000)
        tt = np.stack([(ii + 0.5 - fp.nx / 2) * fp.pix, (jj + 0.5 - fp.ny / 2) * fp.pix], 1)
        t0 = time.perf_counter()
        ref = oracle.flat_points(tt, fp.frame, fp.accept_cos, fp.eta0, fp.boxes)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(ii) * kept / dt, "unit": "pairs/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"{len(ii)} random pixels x {kept:,} segments, "
                                         f"{dt:.1f} s"}
        res["accuracy_vs_oracle"] = err_metrics(m[jj, ii], ref)
    print(json.dumps(res), flush=True)


def legendre_pairs_summed(nside: int, lmax: int, rings_per_block: int = 512) -> tuple:
    """(l, m, ring pair) triples the Legendre kernel sums at (nside, lmax),
    and all of them: a block of ring pairs is dropped for an m when the
    bound sqrt((2 lmax + 1)/4pi) sin^m sqrt((lmax+m)!/(lmax-m)!) / (2^m m!)
    on its most equatorial ring is below 2^-403 (the kernel's own test, on
    the ring's sin(theta) from the RING-scheme z)."""
    N, npair = nside, 2 * nside
    nblk = (npair + rings_per_block - 1) // rings_per_block
    s_edge = []
    for b in range(nblk):
        i = min((b + 1) * rings_per_block, npair)       # north ring index of the last pair
        z = 1.0 - i * i / (3.0 * N * N) if i < N else 4.0 / 3.0 - 2.0 * i / (3.0 * N)
        s_edge.append(math.sqrt(max(0.0, 1.0 - z * z)))
    L = lmax
    total = summed = 0
    for m in range(L + 1):
        nl = L - m + 1
        for b in range(nblk):
            pairs = min(rings_per_block, npair - b * rings_per_block)
            total += nl * pairs
            s = s_edge[b]
            lg = (0.5 * math.log2((2 * L + 1) / (4 * math.pi)) +
                  (m * math.log2(s) if s > 0 else -math.inf) +
                  (0.5 * (math.lgamma(L + m + 1) - math.lgamma(L - m + 1)) - math.lgamma(m + 1)) /
                  math.log(2) - m)
            if lg >= -403.0:
                summed += nl * pairs
    return summed, total


def bench_alm(args, B, torch):
    """Angular power spectrum of a string map: the FP32C map of one 400,000-
    segment box at Nside=2048 (rendered first, not timed), then a_lm up to
    lmax = 4096 = 2 Nside and C_l, timed over back-to-back whole calls (each
    takes its scratch from the library's stream-ordered pool and returns it),
    in FP64."""
    nside, lmax = NSIDE, 2 * NSIDE
    sky, _ = make_sky(B, torch, 0, B.CSMAP_FORM_FP32C, args.nseg, nside)
    hmap = sky.render()
    torch.cuda.synchronize()
    alm = B.map2alm(hmap, lmax)                      # warm-up
    torch.cuda.synchronize()
    K = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(K):
        alm = B.map2alm(hmap, lmax)
        cl = B.alm2cl(alm, lmax)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / K
    size = (lmax + 1) * (lmax + 2) // 2
    # Work of the path taken at this Nside (a power of two <= 2048): per
    # pair of cap rings of 4i pixels, nine power-of-two transforms of
    # P = 2^ceil(log2(2i - 1)) points (5 P log2 P each: the chirp filter and
    # two per quarter-length DFT), four pointwise products (6 P each) and
    # 20 per output m for the radix-4 step, the unpacking and the
    # half-pixel phase; one FFT per belt ring (5 H log2 H for the
    # half-length complex FFT, H = 2 Nside, and 10 per output m); and the
    # Legendre sums (8 FLOP per (l, m, ring pair) summed: the blocks whose
    # terms are all below 2^-403 are not evaluated and not counted).
    cap = 0.0
    for i in range(1, nside):
        P = 1 << max(0, (2 * i - 2).bit_length())
        cap += 9 * 5.0 * P * math.log2(P) + 24.0 * P + 20.0 * (lmax + 1)
    H = 2 * nside
    summed, all_triples = legendre_pairs_summed(nside, lmax)
    flop = (cap + (2 * nside + 1) * (5.0 * H * math.log2(H) + 10.0 * (lmax + 1)) +
            8.0 * summed)
    tf = flop / el / 1e12
    c = cl.cpu().numpy()
    res = {"metric": "map2alm + alm2cl at Nside=2048, lmax=4096 (s per call)", "value": el,
           "unit": "s", "higher_is_better": False, "alm_per_s": size / el,
           "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS, "flop": flop},
           "cl_sample": {str(l): float(c[l]) for l in (2, 10, 100, 1000, 4000)}}
    # The Legendre kernel alone: its time in one more call, from HIP events
    # on the stream it runs on, against the sums' 8 FLOP per (l, m, ring
    # pair) and against the counted hardware FLOP.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    B.map2alm(hmap, lmax)
    ev1.record()
    torch.cuda.synchronize()
    res["call_ms_events"] = ev0.elapsed_time(ev1)
    res["legendre"] = {"flop": 8.0 * summed, "triples_summed": summed,
                       "triples_all": all_triples, "summed_frac": summed / all_triples,
                       "flop_all_triples": 8.0 * all_triples,
                       "hw": measured_valu("k_legendre", None)}
    if not args.no_cpu:
        # The oracle's direct sum costs npix * lmax^2 / 2 terms, so at
        # lmax = 2 Nside its time grows as Nside^4: it is timed on the same
        # call at Nside = 128 and scaled.
        import oracle
        ns = 128
        small = np.random.default_rng(515).standard_normal(12 * ns * ns)
        _log(f"bench alm: oracle at Nside={ns}")
        t0 = time.perf_counter()
        oracle.alm2cl(2 * ns, oracle.map2alm(ns, 2 * ns, small))
        dt = time.perf_counter() - t0
        est = dt * (nside / ns) ** 4
        res["cpu_baseline"] = {"value": est, "unit": "s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"map2alm + alm2cl at Nside={ns}, lmax={2 * ns} in {dt:.1f} s, "
                                         f"scaled by (Nside ratio)^4 = {(nside / ns) ** 4:.0f} to "
                                         f"Nside={nside}"}
    print(json.dumps(res), flush=True)


def bench_config4(args, B, torch):
    """Nside=1024, 8 boxes x 50,000 segments: FP32C forward and the adjoint
    of L = sum_p w_p Theta_p^2."""
    import synth
    w = synth.config4()
    sky = _sky_from(B, torch, w, B.CSMAP_FORM_FP32C)
    wts = torch.from_numpy(synth.config4_weights(w.npix)).cuda()
    m = sky.render()
    g = 2.0 * wts * m
    sky.backward(g)                               # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = sky.render()
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    sky.backward(2.0 * wts * m)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    st = sky.stats()
    pairs = st["pairs"]
    res = {"metric": "config4 forward + adjoint pairs/s", "forward_pairs_per_s": pairs / tf,
           "adjoint_pairs_per_s": pairs / tb, "pairs": pairs, "forward_ms": tf * 1e3,
           "adjoint_ms": tb * 1e3, "adjoint_kernel_ms": st["ms_backward"]}
    adj_tf = ADJ_FLOP_PER_PAIR * pairs / (st["ms_backward"] / 1e3) / 1e12
    res["adjoint_roofline"] = {"bound": "alu", "kernel": "k_adj32", "flop_per_pair":
                               ADJ_FLOP_PER_PAIR, "achieved": adj_tf, "peak": FP32_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": adj_tf / FP32_PEAK_TFLOPS,
                               "hw": measured_valu("k_adj32", st["ms_backward"])}
    res["forward_accuracy_vs_oracle"], dt = _sampled_accuracy(torch, w, m, 4000, seed=213)
    res["cpu_baseline"] = _sampled_cpu_baseline(w, pairs, 4000, dt)
    # The adjoint's gradient on 64 sampled segments against the oracle's
    # (each over all pixels; the cotangent is 2 w Theta of the GPU map).
    import oracle
    grads = sky.backward(2.0 * wts * m)
    got = np.concatenate([np.concatenate([a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy(),
                                          d.cpu().numpy()[:, None]], 1)
                          for a, b, c, d in grads])
    sel = synth.sample_pixels(sum(bx.n for bx in w.boxes), 64, seed=210)
    _log("bench config4: oracle gradient on 64 segments")
    gref = oracle.grad(w.nside, np.arange(w.npix), (2.0 * wts * m).cpu().numpy(), w.eta0,
                       w.boxes, sel)
    acc = {"segments": 64}
    for name, sl in (("x_rel", slice(0, 3)), ("xdot", slice(3, 6)), ("xprime", slice(6, 9)),
                     ("dsigma", slice(9, 10))):
        d = got[sel][:, sl] - gref[:, sl]
        acc[name + "_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(gref[:, sl]))
    res["adjoint_accuracy_vs_oracle"] = acc
    print(json.dumps(res), flush=True)


def measured_valu(kernel, kernel_ms):
    """Hardware-counted vector FLOP of a kernel launch from the committed
    rocprofv3 counter runs (if taken on the kernel's current sources: the
    record holds their SHA-256), as FLOP per launch and the rate over a
    launch of kernel_ms."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("kernels", {}).get(kernel)
    if k is None or _sources_sha(k["sources"]) != k["sources_sha256"]:
        return None
    out = {"fp32_flop": k["fp32_flop"], "fp64_flop": k["fp64_flop"],
           "valu_insts": k["valu_insts"], "valu_insts_per_pair": k.get("valu_insts_per_pair"),
           "counted_launch_ms": k["trace_ns"] / 1e6, "summary": rec.get("summary")}
    ms = kernel_ms if kernel_ms else k["trace_ns"] / 1e6
    out["fp32_tflops"] = k["fp32_flop"] / (ms / 1e3) / 1e12
    out["fp64_tflops"] = k["fp64_flop"] / (ms / 1e3) / 1e12
    out["frac_fp32_peak"] = out["fp32_tflops"] / FP32_PEAK_TFLOPS
    out["frac_fp64_peak"] = out["fp64_tflops"] / FP64_PEAK_TFLOPS
    return out


# Sources each counted kernel is built from (its record holds their SHA-256).
VALU_SOURCES = {
    # The kernel sources, and the host code that chooses its launch (tiling,
    # tile plan), which changes what the counters see.
    "k_fwd32": ["paper_1204_5041_amd/csrc/kernels.hip", "paper_1204_5041_amd/csrc/segment_dev.h",
                "paper_1204_5041_amd/csrc/internal.h", "paper_1204_5041_amd/csrc/healpix_dev.h",
                "paper_1204_5041_amd/csrc/api.cpp", "paper_1204_5041_amd/csrc/sched.cpp"],
    "k_legendre": ["paper_1204_5041_amd/csrc/alm.hip", "paper_1204_5041_amd/csrc/healpix_dev.h"],
    "k_valu_probe": ["paper_1204_5041_amd/csrc/probe.hip"],
}
VALU_SOURCES["k_fwd64"] = VALU_SOURCES["k_adj32"] = VALU_SOURCES["k_fwd32"]


def _sources_sha(files):
    import hashlib
    h = hashlib.sha256()
    for src in files:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def summarize_counters(trace_dir, pmc_a, pmc_b, launches_json):
    """Per-kernel VALU record from the counter runs of --workload counters:
    instruction counts of each launch (SQ_INSTS_VALU and the FP32/FP64 FMA,
    ADD, MUL and TRANS counts, all per wavefront instruction), hardware FLOP
    (64 lanes x (2 FMA + ADD + MUL + TRANS)), the kernel-trace duration of
    the same launch, the rate against the published peaks, the issue rate
    per SIMD and clock, and the clock from SQ_BUSY_CYCLES (summed over the
    32 shader engines).  The FMA probe's counted instructions are compared
    with the number it issues by construction."""
    import csv
    runs = json.loads([l for l in open(launches_json) if l.startswith("{")][-1])

    def launches(d):
        out = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
            rec = out.setdefault(key, {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            rec[r["Counter_Name"]] = float(r["Counter_Value"])
        return out

    def trace_ns(name_part, nth=0):
        rows = [r for r in csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv")))
                if name_part in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        r = rows[nth]
        return int(r["End_Timestamp"]) - int(r["Start_Timestamp"])

    a, b = launches(pmc_a), launches(pmc_b)

    def counters(name_part, nth=0):
        ka = sorted(k for k in a if name_part in k[0])[nth]
        kb = sorted(k for k in b if name_part in k[0])[nth]
        c = dict(a[ka])
        c.update({k: v for k, v in b[kb].items() if k != "ns"})
        return ka[0], c

    rec = {"note": "rocprofv3 counters per launch of `bench.py --workload counters`; FLOP = "
                   "64 x (2 FMA + ADD + MUL + TRANS) per precision (counts are per wavefront "
                   "instruction); durations from the kernel-trace run of the same command",
           "peaks_tflops": {"fp32": FP32_PEAK_TFLOPS, "fp64": FP64_PEAK_TFLOPS},
           "summary": "profiles/valu_counters.md", "kernels": {}}
    plan = [("k_valu_probe<float, false>", "probe_fp32", None),
            ("k_valu_probe<double, false>", "probe_fp64", None),
            ("k_valu_probe<float, true>", "probe_fp32_scalar_operand", None),
            ("k_fwd32", "k_fwd32", ("k_fwd32", 0)),
            ("k_fwd64", "k_fwd64", ("k_fwd64", 0)),
            ("k_adj32", "k_adj32", ("k_adj32", 0)),
            ("k_legendre", "k_legendre", None)]
    for part, key, _ in plan:
        nth = -1 if key == "k_legendre" else 0   # the last of the map2alm calls
        name, c = counters(part, nth)
        ns = trace_ns(part, nth)
        s = ns / 1e9
        f32 = 64 * (2 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] +
                    c["SQ_INSTS_VALU_MUL_F32"] + c["SQ_INSTS_VALU_TRANS_F32"])
        f64 = 64 * (2 * c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_ADD_F64"] +
                    c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_TRANS_F64"])
        clock = c["SQ_BUSY_CYCLES"] / 32 / (c["ns"] / 1e9)
        k = {"kernel": name, "trace_ns": ns, "valu_insts": c["SQ_INSTS_VALU"],
             "salu_insts": c["SQ_INSTS_SALU"], "fp32_flop": f32, "fp64_flop": f64,
             "counts": {n: c[n] for n in sorted(c) if n.startswith("SQ_")},
             "hw_fp32_tflops": f32 / s / 1e12, "hw_fp64_tflops": f64 / s / 1e12,
             "frac_fp32_peak": f32 / s / 1e12 / FP32_PEAK_TFLOPS,
             "frac_fp64_peak": f64 / s / 1e12 / FP64_PEAK_TFLOPS,
             "clock_ghz_from_busy_cycles": clock / 1e9,
             "valu_issue_per_simd_clk_at_2p4ghz": c["SQ_INSTS_VALU"] / (s * 2.4e9 * 1024),
             "valu_issue_per_simd_clk_at_measured_clock": c["SQ_INSTS_VALU"] / (s * clock * 1024)}
        base = key if not key.startswith("probe") else "k_valu_probe"
        k["sources"] = VALU_SOURCES[base]
        k["sources_sha256"] = _sources_sha(VALU_SOURCES[base])
        if key.startswith("probe"):
            pr = runs[key]
            k["fma_insts_by_construction"] = pr["fma_insts"]
            fma = c["SQ_INSTS_VALU_FMA_F64" if "fp64" in key else "SQ_INSTS_VALU_FMA_F32"]
            k["counted_over_constructed"] = fma / pr["fma_insts"]
            k["fma_lanes_per_clk_per_cu_at_2p4ghz"] = fma * 64 / s / 256 / 2.4e9
            k["fma_lanes_per_clk_per_cu_at_measured_clock"] = fma * 64 / s / 256 / clock
        elif key in runs and "pairs" in runs[key]:
            p = runs[key]["pairs"]
            k["pairs"] = p
            k["valu_insts_per_pair"] = c["SQ_INSTS_VALU"] * 64 / p
            k["hw_flop_per_pair"] = (f32 + f64) / p
        rec["kernels"][key] = k
    return rec


def bench_hbm(args, torch):
    """The rate a plain device copy streams at (1 GiB read and 1 GiB written
    per copy, 20 back-to-back copies between HIP events): what an HBM-bound
    kernel can reach in practice, against the 8 TB/s of the specification."""
    n = 1 << 28
    x = torch.empty(n, dtype=torch.float32, device="cuda").normal_()
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 20 / 1e3
    gbs = 2 * 4 * n / s / 1e9
    print(json.dumps({"metric": "device copy rate (read + write)", "value": gbs, "unit": "GB/s",
                      "bytes_per_copy": 2 * 4 * n, "ms_per_copy": s * 1e3,
                      "frac_of_8000": gbs / 8000.0}), flush=True)


def bench_counters(args, B, torch):
    """One launch of each kernel that the hardware counter summaries cover,
    each preceded by a log line naming it: the FMA probe in FP32 and in
    FP64 (known instruction counts), map2alm at Nside 2048, lmax 4096 of a
    seeded random map six times (k_legendre; its work does not depend on the
    values; the summaries take the last call, once the clock has risen from
    its idle level), the default step's
    k_fwd32 (config2 box 0, FP32C), k_fwd64 (same box, FP64 form) and the
    config4 adjoint (k_adj32)."""
    import synth
    res = {"metric": "counter-run launches"}
    blocks = 2048
    for kind, name, iters in ((0, "fp32", 200_000), (1, "fp64", 100_000),
                              (2, "fp32_scalar_operand", 100_000)):
        _log(f"counters: probe {name}")
        ms, insts = B.valu_probe(kind, blocks, iters)
        lanes = insts * 64 / (ms / 1e3) / (256 * 2.4e9)
        res[f"probe_{name}"] = {"blocks": blocks, "iters": iters, "ms": ms, "fma_insts": insts,
                                "fma_lanes_per_clk_per_cu": lanes}
    _log("counters: map2alm (k_legendre), Nside 2048, lmax 4096")
    hm = torch.from_numpy(np.random.default_rng(2048).standard_normal(12 * NSIDE * NSIDE)).cuda()
    for _ in range(5):
        B.map2alm(hm, 4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.map2alm(hm, 4096)
    torch.cuda.synchronize()
    res["map2alm"] = {"nside": NSIDE, "lmax": 4096, "calls": 6,
                      "ms_last": (time.perf_counter() - t0) * 1e3}
    del hm
    _log("counters: k_fwd32 (config2 box 0)")
    sky, box = make_sky(B, torch, 0, B.CSMAP_FORM_FP32C, NSEG, NSIDE)
    sky.render()
    st = sky.stats()
    res["k_fwd32"] = {"pairs": st["pairs"], "ms": st["ms_forward"]}
    sky.close()
    _log("counters: k_fwd64 (config2 box 0)")
    sky, _ = make_sky(B, torch, 0, B.CSMAP_FORM_FP64, NSEG, NSIDE)
    sky.render()
    st = sky.stats()
    res["k_fwd64"] = {"pairs": st["pairs"], "ms": st["ms_forward"]}
    sky.close()
    _log("counters: k_adj32 (config4)")
    w = synth.config4()
    sky = _sky_from(B, torch, w, B.CSMAP_FORM_FP32C)
    wts = torch.from_numpy(synth.config4_weights(w.npix)).cuda()
    m4 = sky.render()
    sky.backward(2.0 * wts * m4)
    st = sky.stats()
    res["k_adj32"] = {"pairs": st["pairs"], "ms": st["ms_backward"]}
    sky.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
