"""GPU parity of the forward path against the FP64 oracle.

Every case runs the HIP library through its C ABI (ctypes binding) and the
oracle on the same seeded inputs.  Bars: pixel directions and pair counts
bit-exact; FP64 form within 1e-12 (relative rms and relative max over the
checked pixels); FP32C form within rel-rms 1e-5 and rel-max 1e-4."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import err_metrics, sky_from_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
FP32_RMS, FP32_MAX = 1e-5, 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    assert torch.cuda.is_available()
    return binding


# ----------------------------------------------------------------------------
# Pixel directions
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("nside", [1, 2, 3, 5, 16, 64, 512])
def test_pix2vec_bit_exact_all_pixels(B, nside):
    say(f"pix2vec all pixels nside={nside}")
    gpu = B.pix2vec_ring(nside).cpu().numpy()
    ref = oracle.pix2vec(nside, np.arange(12 * nside * nside))
    assert np.array_equal(gpu.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("nside", [2048, 4096, 8192])
def test_pix2vec_bit_exact_sampled(B, nside):
    say(f"pix2vec sampled nside={nside}")
    npx = 12 * nside * nside
    gpu = B.pix2vec_ring(nside)
    pick = synth.sample_pixels(npx, 200_000, seed=nside)
    # ring boundaries and the last pixels too
    extra = np.array([0, 1, 2, 3, 4, npx - 1, npx - 2, 2 * nside * (nside - 1),
                      2 * nside * (nside - 1) - 1, npx - 2 * nside * (nside - 1),
                      npx // 2, npx // 2 - 1], dtype=np.int64)
    pick = np.unique(np.concatenate([pick, extra]))
    ref = oracle.pix2vec(nside, pick)
    got = gpu[torch.from_numpy(pick).cuda()].cpu().numpy()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


# ----------------------------------------------------------------------------
# Small workloads covering every rule, with ragged tiles
# ----------------------------------------------------------------------------
def mixed_workload(nside=13, dtype=np.float64, n=(300, 0, 257, 120, 64)):
    eta0 = 3.0
    boxes = [
        synth.make_box(n[0], 31, origin=(-0.5, -0.5, -0.5), eta_lo=2.2, eta_hi=3.0, dtype=dtype),
        synth.make_box(n[1], 32, origin=(0.2, 0.1, 0.3), eta_lo=0.0, eta_hi=3.0, dtype=dtype),
        synth.make_box(n[2], 33, origin=(0.8, -0.4, 0.2), eta_lo=0.9, eta_hi=1.6, dtype=dtype,
                       vis=synth.VIS_BOX),
        synth.make_box(n[3], 34, origin=(-1.9, 0.4, -0.6), eta_lo=0.0, eta_hi=3.0, dtype=dtype,
                       vis=synth.VIS_CAP, cap_dir=np.array([-0.8, 0.6, 0.0]), cap_cos=0.7),
        synth.make_box(n[4], 35, origin=(0.3, 1.2, -1.5), eta_lo=-5.0, eta_hi=0.9, dtype=dtype,
                       vis=synth.VIS_BOX),
    ]
    return synth.Workload("mixed", nside, eta0, boxes)


def expected_pairs(w):
    pix = np.arange(w.npix)
    tot = 0
    for bx in w.boxes:
        if bx.n == 0:
            continue
        tot += int(oracle.visible(w.nside, pix, w.eta0, bx).sum()) * int(oracle.kept(w.eta0, bx).sum())
    return tot


@pytest.fixture(scope="module")
def mixed():
    w = mixed_workload()
    ref = oracle.theta_pixels(w.nside, np.arange(w.npix), w.eta0, w.boxes)
    return w, ref, expected_pairs(w)


@pytest.mark.parametrize("form", ["fp64", "fp32c", "fp32c-frac"])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
@pytest.mark.parametrize("schedule", [0, 1, 2])
@pytest.mark.parametrize("tiling", [1, 2])
def test_mixed_rules_all_shapes(B, mixed, form, K, schedule, tiling):
    w, ref, pairs = mixed
    say(f"mixed form={form} K={K} schedule={schedule} tiling={tiling}")
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    opts = {B.CSMAP_OPT_PIX_PER_LANE: K, B.CSMAP_OPT_SCHEDULE: schedule, B.CSMAP_OPT_WAVES: 2,
            B.CSMAP_OPT_TILING: tiling}
    if form != "fp64":
        opts[B.CSMAP_OPT_ACCUM] = 1 if form == "fp32c-frac" else 0
    sky = sky_from_workload(w, f, opts)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    assert st["tiling"] == tiling
    assert st["pairs"] == pairs
    assert st["kept"] == sum(int(oracle.kept(w.eta0, b).sum()) for b in w.boxes)
    if form == "fp64":
        assert e["rel_rms"] <= FP64_TOL and e["rel_max"] <= FP64_TOL, e
    else:
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


@pytest.mark.parametrize("accum", [0, 1])
@pytest.mark.parametrize("near_w", [1e-6, 1e-3, 5e-3, 0.2, 3.0])
def test_fp32c_near_threshold_any_value_within_gate(B, mixed, near_w, accum):
    """Small values send most pairs through the dot-product form, >= 2 sends
    every pair through the FP64 difference; both stay within the gate on
    this well-separated workload, and the literal form is the tighter one."""
    w, ref, _ = mixed
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C, {B.CSMAP_OPT_NEAR_W: near_w,
                                                    B.CSMAP_OPT_ACCUM: accum})
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    say(f"near_w={near_w} accum={accum} {e} near_steps={st['near_steps']}")
    assert np.all(np.isfinite(m))
    if near_w >= 2:
        # every step takes the FP64 difference (the literal form)
        assert st["mid_steps"] == 0 and st["near_steps"] > 0
        assert e["rel_rms"] <= 1e-7
    if near_w >= 1e-3:
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


@pytest.mark.parametrize("accum", [0, 1])
@pytest.mark.parametrize("near_w,far_w,path", [(1e-6, 1e-6, "far"), (1e-6, 3.0, "middle"),
                                               (3.0, 3.0, "fp64"), (5e-5, 5e-3, "default"),
                                               (1e-3, 0.2, "wide middle")])
def test_fp32c_three_pair_forms(B, mixed, near_w, far_w, path, accum):
    """The FP32C form takes one of three forms per (wavefront, segment) step:
    dot products when every pair is at least far_w from the segment (in
    1 - n.P/R), the FP32 difference n - P/R when some pair is closer but
    none below near_w, the FP64 difference otherwise.  Forcing each one in
    turn leaves the map within the gate (the all-dot-product case excepted,
    whose close pairs lose precision by design) and the counters say which
    form ran."""
    w, ref, pairs = mixed
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C, {B.CSMAP_OPT_NEAR_W: near_w,
                                                    B.CSMAP_OPT_FAR_W: far_w,
                                                    B.CSMAP_OPT_ACCUM: accum})
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    say(f"{path} accum={accum} {e} fp64_steps={st['near_steps']} mid_steps={st['mid_steps']}")
    assert st["pairs"] == pairs and np.all(np.isfinite(m))
    if path == "far":
        assert st["mid_steps"] == 0
    elif path == "middle":
        assert st["mid_steps"] > 0 and st["near_steps"] < st["mid_steps"] // 100
    elif path == "fp64":
        assert st["mid_steps"] == 0 and st["near_steps"] > 0
    if path != "far":
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def caps_workload(nside=96):
    """Cap-visibility boxes around a pole, across phi = 0, on the equator
    and at mid latitude, plus one box every pixel sees: ring blocks with
    full 64-pixel rows, polar blocks of unequal rings, and the belt."""
    eta0 = 3.0
    dirs = [(0.0, 0.0, 1.0), (1.0, 0.0, 0.05), (0.3, -0.95, 0.0), (-0.5, 0.4, -0.77)]
    boxes = []
    for b, d in enumerate(dirs):
        d = np.asarray(d) / np.linalg.norm(d)
        centre = 1.5 * d
        boxes.append(synth.make_box(150 + 37 * b, 60 + b, origin=centre - 0.5, eta_lo=0.0,
                                    eta_hi=3.0, dtype=np.float32, vis=synth.VIS_CAP, cap_dir=d,
                                    cap_cos=math.cos(0.35 + 0.1 * b)))
    boxes.append(synth.make_box(90, 65, origin=(-0.5, -0.5, -0.5), eta_lo=0.0, eta_hi=3.0,
                                dtype=np.float32))
    return synth.Workload("caps", nside, eta0, boxes)


@pytest.fixture(scope="module")
def caps():
    w = caps_workload()
    ref = oracle.theta_pixels(w.nside, np.arange(w.npix), w.eta0, w.boxes)
    return w, ref, expected_pairs(w)


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
@pytest.mark.parametrize("K", [2, 8])
@pytest.mark.parametrize("tiling,rings", [(1, 0), (2, 0), (2, 1), (2, 4), (2, 64)])
def test_cap_sky_both_tilings(B, caps, form, K, tiling, rings):
    """Strips and ring blocks of 1 to 64 rings per tile (64 rings: one lane
    per ring) give the oracle's map."""
    w, ref, pairs = caps
    say(f"caps form={form} K={K} tiling={tiling} rings={rings}")
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    sky = sky_from_workload(w, f, {B.CSMAP_OPT_PIX_PER_LANE: K, B.CSMAP_OPT_TILING: tiling,
                                   B.CSMAP_OPT_BLOCK_RINGS: rings})
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    assert st["tiling"] == tiling and st["pairs"] == pairs
    if form == "fp64":
        assert e["rel_rms"] <= FP64_TOL and e["rel_max"] <= FP64_TOL, e
    else:
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def test_graph_replay_matches_eager_and_is_deterministic(B, mixed):
    w, ref, _ = mixed
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C, {B.CSMAP_OPT_SCHEDULE: 1})
    eager = sky.render().cpu().numpy()
    eager2 = sky.render().cpu().numpy()
    assert np.array_equal(eager, eager2)
    sky.set_option(B.CSMAP_OPT_GRAPH, 1)
    out = torch.empty(w.npix, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        sky.render(out)
        got = out.cpu().numpy()
        assert np.array_equal(got, eager), rep
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
    sky.close()


def test_empty_sky_and_empty_box(B):
    w = synth.Workload("empty", 4, 1.0, [])
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    m = sky.render().cpu().numpy()
    assert np.all(m == 0.0) and sky.stats()["pairs"] == 0
    sky.close()
    w2 = mixed_workload(nside=2, n=(0, 0, 0, 0, 0))
    sky = sky_from_workload(w2, B.CSMAP_FORM_FP64)
    assert np.all(sky.render().cpu().numpy() == 0.0)
    sky.close()


def test_exact_coincidence_is_zero(B):
    # Nside=1 pixel 4 is exactly +x; a segment at (0.5, 0, 0) sits on it.
    x = np.array([[0.5, 0.0, 0.0], [0.1, 0.3, -0.2]])
    xd = np.array([[0.0, 0.5, 0.0], [0.3, 0.0, 0.1]])
    xp = np.array([[0.0, 0.0, math.sqrt(0.75)], [0.0, 0.6, 0.0]])
    ds = np.array([0.01, 0.01])
    bx = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=-10, eta_hi=10, x_rel=x, xdot=xd,
                   xprime=xp, dsigma=ds)
    w = synth.Workload("coincide", 1, 1.0, [bx])
    ref = oracle.theta_pixels(1, np.arange(12), 1.0, [bx])
    for form in (B.CSMAP_FORM_FP64, B.CSMAP_FORM_FP32C):
        sky = sky_from_workload(w, form)
        m = sky.render().cpu().numpy()
        assert np.all(np.isfinite(m))
        e = err_metrics(m, ref)
        assert e["rel_max"] <= (FP64_TOL if form == B.CSMAP_FORM_FP64 else FP32_MAX), e
        sky.close()


def test_sparse_keep_records_span_many_blocks(B):
    """2,000,000 segments of which every 1,700th lies in the slab: the first
    workgroup of the records pass finds its records spread over more source
    blocks than it stages in LDS, and searches the block prefixes in global
    memory.  The kept count and the map equal the oracle's."""
    n = 2_000_000
    _, xd, xp, ds = synth.segments(n, 61, np.float64)
    r = np.full(n, 5.0)
    r[::1700] = 2.0
    P = synth.uniform_directions(n, 62) * r[:, None]
    bx = synth.Box(origin=np.zeros(3), ext=np.ones(3), eta_lo=0.5, eta_hi=1.5, x_rel=P,
                   xdot=xd, xprime=xp, dsigma=ds)
    w = synth.Workload("sparse", 8, 3.0, [bx])
    kept = int(oracle.kept(3.0, bx).sum())
    assert kept == len(r[::1700])
    ref = oracle.theta_pixels(w.nside, np.arange(w.npix), w.eta0, w.boxes)
    for form, tol in ((B.CSMAP_FORM_FP64, (FP64_TOL, FP64_TOL)),
                      (B.CSMAP_FORM_FP32C, (FP32_RMS, FP32_MAX))):
        sky = sky_from_workload(w, form)
        m = sky.render().cpu().numpy()
        st = sky.stats()
        sky.close()
        e = err_metrics(m, ref)
        say(f"sparse keep form={form}: kept {st['kept']} of {n} {e}")
        assert st["kept"] == kept
        assert e["rel_rms"] <= tol[0] and e["rel_max"] <= tol[1], e


# ----------------------------------------------------------------------------
# The benchmark workloads
# ----------------------------------------------------------------------------
def test_config0_fp64_every_pixel(B):
    w = synth.config0()
    say("config0 oracle")
    ref = oracle.theta_pixels(w.nside, np.arange(w.npix), w.eta0, w.boxes)
    for form, tol in ((B.CSMAP_FORM_FP64, (FP64_TOL, FP64_TOL)),
                      (B.CSMAP_FORM_FP32C, (FP32_RMS, FP32_MAX))):
        say(f"config0 form={form}")
        sky = sky_from_workload(w, form)
        m = sky.render().cpu().numpy()
        e = err_metrics(m, ref)
        say(f"config0 form={form} {e}")
        assert sky.stats()["pairs"] == w.npix * 2000
        assert e["rel_rms"] <= tol[0] and e["rel_max"] <= tol[1], e
        sky.close()


@pytest.fixture(scope="module")
def config1():
    w = synth.config1()
    npx = w.npix
    pix = np.arange(npx)
    seen = np.zeros(npx, dtype=bool)
    vis_counts, kept_counts = [], []
    for bx in w.boxes:
        v = oracle.visible(w.nside, pix, w.eta0, bx)
        seen |= v
        vis_counts.append(int(v.sum()))
        kept_counts.append(int(oracle.kept(w.eta0, bx).sum()))
    rng = np.random.Generator(np.random.PCG64(25))
    check = np.sort(rng.choice(np.flatnonzero(seen), size=10_000, replace=False))
    ref = oracle.theta_pixels(w.nside, check, w.eta0, w.boxes)
    pairs = sum(a * b for a, b in zip(vis_counts, kept_counts))
    return w, check, ref, pairs


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_config1_shell_of_24_boxes(B, config1, form):
    w, check, ref, pairs = config1
    f = B.CSMAP_FORM_FP64 if form == "fp64" else B.CSMAP_FORM_FP32C
    say(f"config1 form={form}")
    sky = sky_from_workload(w, f)
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m[check], ref)
    say(f"config1 form={form} {e} pairs={st['pairs']} ms={st['ms_forward']:.1f}")
    assert st["pairs"] == pairs
    if form == "fp64":
        assert e["rel_rms"] <= FP64_TOL and e["rel_max"] <= FP64_TOL, e
    else:
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def test_config2_one_box_full_sky(B):
    """Nside=2048 and one 400,000-segment box (the benchmark step): the FP32C
    map on 2,000 sampled pixels against the oracle."""
    w = synth.config2(boxes=[0])
    check = synth.sample_pixels(w.npix, 2000, seed=98)
    say("config2 box0 oracle")
    ref = oracle.theta_pixels(w.nside, check, w.eta0, w.boxes)
    say("config2 box0 gpu")
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    m = sky.render()
    got = m[torch.from_numpy(check).cuda()].cpu().numpy()
    st = sky.stats()
    e = err_metrics(got, ref)
    say(f"config2 {e} pairs={st['pairs']} ms={st['ms_forward']:.1f} near={st['near_steps']}")
    assert st["pairs"] == w.npix * 400_000
    assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    sky.close()


def test_autotune_keeps_parity_and_caches(B, mixed, tmp_path):
    w, ref, pairs = mixed
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    cache = str(tmp_path / "tune.txt")
    sky.autotune(cache)
    st0 = sky.stats()
    m = sky.render().cpu().numpy()
    st = sky.stats()
    e = err_metrics(m, ref)
    assert st["pairs"] == pairs
    assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and "fp32c" in lines[0]
    # a second sky with the same shape takes the cached choice without timing
    sky2 = sky_from_workload(w, B.CSMAP_FORM_FP32C)
    sky2.autotune(cache)
    s2 = sky2.stats()
    for k in ("pix_per_lane", "waves", "schedule", "tiling", "chunk", "near_w", "far_w"):
        assert s2[k] == st0[k], k
    # tuning never picks a less accurate pair form than the defaults
    assert st0["far_w"] >= 5e-3 and st0["near_w"] >= 5e-5
    assert len(open(cache).read().strip().splitlines()) == 1
    sky.close()
    sky2.close()


def test_batched_uneven_caps_persistent_graph(B):
    """A reduced copy of the batched workload (Nside 256, 64 boxes with
    lognormal segment counts scaled by 1/20 and cap visibility): persistent
    schedule with per-tile box lists, captured in a graph, against the oracle
    on 3,000 pixels that see at least one box; the per-box schedule agrees."""
    w = synth.config3(nbox=64, nside=256, count_scale=0.05)
    pix = np.arange(w.npix)
    seen = np.zeros(w.npix, dtype=bool)
    pairs = 0
    for bx in w.boxes:
        v = oracle.visible(w.nside, pix, w.eta0, bx)
        seen |= v
        pairs += int(v.sum()) * int(oracle.kept(w.eta0, bx).sum())
    check = np.sort(np.random.default_rng(398).choice(np.flatnonzero(seen), 3000, replace=False))
    ref = oracle.theta_pixels(w.nside, check, w.eta0, w.boxes)
    sky = sky_from_workload(w, B.CSMAP_FORM_FP32C, {B.CSMAP_OPT_SCHEDULE: 1, B.CSMAP_OPT_GRAPH: 1})
    out = torch.empty(w.npix, dtype=torch.float64, device="cuda")
    for rep in range(3):
        sky.render(out)
        m = out.cpu().numpy()
        st = sky.stats()
        e = err_metrics(m[check], ref)
        say(f"batched rep={rep} {e} pairs={st['pairs']}")
        assert st["pairs"] == pairs
        assert e["rel_rms"] <= FP32_RMS and e["rel_max"] <= FP32_MAX, e
        assert np.all(m[~seen] == 0.0)
    sky.set_option(B.CSMAP_OPT_SCHEDULE, 2)
    sky.set_option(B.CSMAP_OPT_GRAPH, 0)
    m2 = sky.render().cpu().numpy()
    e2 = err_metrics(m2[check], ref)
    assert e2["rel_rms"] <= FP32_RMS and e2["rel_max"] <= FP32_MAX, e2
    sky.close()
