/*
 * csmap.h -- C ABI of libcsmap, the MI355X (gfx950) implementation of the
 * all-sky string integrated Sachs-Wolfe map maker of Ringeval & Bouchet.
 *
 * The problem (paper Sec. II.A, Eq. (1)-(2), and Sec. III opening
 * paragraph): simulations record, for every Nambu-Goto string segment on the
 * observer's past light cone, its position X, velocity Xdot, tangent X' and
 * length element dsigma.  The map value in direction n is
 *
 *   Theta(n) = -4 GU sum_s  u.(R n - X)/|R n - X|^2 * eps * dsigma,
 *   u = Xdot - (n.X') X' / (1 + n.Xdot),   eps^2 = X'^2 / (1 - Xdot^2),
 *
 * summed over every segment of every box (no cut, Sec. II.A), with R = |X|
 * the observer-relative distance of the event and n the centre of a HEALPix
 * RING pixel (Sec. II.D).  Maps of disjoint sets of boxes add (Sec. III.A:
 * the final map is the sum of full-sky maps from subsets of cones).  The
 * library returns Theta/GU; multiply by GU to obtain Theta = Delta T / T.
 *
 * Coordinates: the observer sits at the origin at conformal time eta0.  A
 * segment of a box at position x_rel (relative to the box's origin) has the
 * observer-relative position P = origin + x_rel (formed in FP64 on the
 * device), lies on the past light cone at eta = eta0 - |P| (gauge
 * X^0 = eta = tau, footnote of Sec. II.A), and enters the map only when
 * eta_lo <= eta < eta_hi (the conformal-time slab the box covers).
 *
 * Conventions of every entry point:
 *   - Array arguments are device pointers (memory from hipMalloc or a torch
 *     CUDA tensor) unless stated otherwise, row-major, naturally aligned.
 *   - Work is enqueued asynchronously on the HIP stream given at sky creation
 *     (NULL = the default stream); the caller synchronises that stream
 *     before reading results.  add_box copies the segment arrays on that
 *     stream, so the caller may free them once the stream has passed the copy.
 *   - Every call returns a csmap_status; on failure csmap_last_error() gives
 *     a message (thread-local, valid until the next call on that thread).
 *     Argument errors are detected on the host before any device work and
 *     leave the sky unchanged.  A HIP failure returns CSMAP_E_DEVICE and
 *     marks the sky failed: later calls on it return CSMAP_E_STATE.
 *   - A sky is not thread-safe: use one sky per thread.
 *   - Physical preconditions (|Xdot| < 1, |X'| > 0, no straight static string,
 *     Sec. II.A) are the caller's; they are documented, not checked.
 */
#ifndef CSMAP_H
#define CSMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csmap_sky csmap_sky;

typedef enum {
    CSMAP_OK = 0,
    CSMAP_E_INVALID = -1,      /* bad argument; nothing was changed */
    CSMAP_E_NOMEM = -2,        /* device or host allocation failed */
    CSMAP_E_DEVICE = -3,       /* a HIP call failed; the sky is now unusable */
    CSMAP_E_STATE = -4,        /* call not valid in the sky's current state */
    CSMAP_E_UNSUPPORTED = -5   /* valid request the library does not provide */
} csmap_status;

/* Arithmetic form of the pair evaluation.
 *   CSMAP_FORM_FP64  : every step in FP64, directions differenced in FP64.
 *   CSMAP_FORM_FP32C : light-cone geometry (P = origin + x_rel, |P|, the slab
 *                      test, unit vectors) in FP64; the pair arithmetic in
 *                      FP32, with the direction difference R(n - P/R) taken
 *                      in FP64 for pairs closer than a threshold angle (see
 *                      CSMAP_OPT_NEAR_W); per-pixel sums in FP32 with Kahan
 *                      compensation; the map written as FP64. */
typedef enum { CSMAP_FORM_FP64 = 0, CSMAP_FORM_FP32C = 1 } csmap_form;

/* Element type of segment arrays passed to csmap_add_box. */
typedef enum { CSMAP_F32 = 0, CSMAP_F64 = 1 } csmap_dtype;

/* Which pixels receive a box's segments.
 *   CSMAP_VIS_ALL : every pixel (the paper's rule: no cut, Sec. II.A).
 *   CSMAP_VIS_BOX : pixels whose ray t n (t >= 0) crosses the closed box
 *                   [origin, origin + ext] at a distance inside the slab's
 *                   radii (eta0 - eta_hi, eta0 - eta_lo].
 *   CSMAP_VIS_CAP : pixels with n . cap_dir >= cap_cos.
 * The last two restrict the sum to a subset of the sky; they exist to shape
 * workloads (they are not part of the paper's method). */
typedef enum { CSMAP_VIS_ALL = 0, CSMAP_VIS_BOX = 1, CSMAP_VIS_CAP = 2 } csmap_vis;

/* One simulation box of light-cone events. */
typedef struct {
    int64_t n;              /* number of segments, >= 0 */
    csmap_dtype dtype;      /* type of the four arrays below */
    const void *x_rel;      /* n x 3: position relative to origin */
    const void *xdot;       /* n x 3: Xdot, worldsheet velocity dX/dtau */
    const void *xprime;     /* n x 3: X', worldsheet tangent dX/dsigma */
    const void *dsigma;     /* n: worldsheet length parameter of the segment */
    double origin[3];       /* observer-relative position x_rel is measured from */
    double ext[3];          /* box extent (used by CSMAP_VIS_BOX), each > 0 */
    double eta_lo, eta_hi;  /* conformal-time slab [eta_lo, eta_hi), eta_lo < eta_hi */
    csmap_vis vis;          /* pixel visibility rule */
    double cap_dir[3];      /* CSMAP_VIS_CAP: cap centre, a unit vector, used as given */
    double cap_cos;         /* CSMAP_VIS_CAP: cosine of the cap radius, in [-1, 1] */
} csmap_box;

/* Caller-owned FP64 gradient outputs for one box (device pointers, same
 * shapes as the box's inputs).  Any pointer may be NULL to skip it. */
typedef struct {
    double *x_rel;          /* n x 3: dL/dx_rel (equal to dL/dP) */
    double *xdot;           /* n x 3: dL/dXdot */
    double *xprime;         /* n x 3: dL/dX' */
    double *dsigma;         /* n: dL/ddsigma */
} csmap_grad;

/* Tunables (csmap_set_option).  Values are doubles; integers are rounded. */
typedef enum {
    /* Launch schedule of render/backward:
     *   0 = one launch, one wavefront per pixel tile, tiles in RING order;
     *   1 = one persistent launch whose wavefronts pull tiles, most expensive
     *       first, from a device work counter;
     *   2 = one launch per box (each box accumulates into the map). */
    CSMAP_OPT_SCHEDULE = 0,
    /* 1 = capture render's launches in a hipGraph and replay it while the sky
     * and the output pointer are unchanged; 0 = plain launches. */
    CSMAP_OPT_GRAPH = 1,
    /* Pixels per lane of the forward kernels: 1, 2, 4 or 8 (default 8 for
     * the FP32C form, 4 for FP64).  A tile of 64 x this many pixels (see
     * CSMAP_OPT_TILING) is owned by one wavefront. */
    CSMAP_OPT_PIX_PER_LANE = 2,
    /* Wavefronts per workgroup: 1, 2 or 4. */
    CSMAP_OPT_WAVES = 3,
    /* FP32C form: a (wavefront, segment) step in which some pair has
     * 1 - n.P/R below this value (default 5e-5, an angle of about 0.01 rad)
     * takes the direction difference n - P/R in FP64.  A value >= 2 sends
     * every pair through the FP64 difference.  Minimum 1e-6. */
    CSMAP_OPT_NEAR_W = 4,
    /* Segments per FP32 partial sum before the Kahan-compensated update of a
     * pixel's running sum (FP32C form): a multiple of 4 in 8 .. 4096. */
    CSMAP_OPT_CHUNK = 5,
    /* Adjoint: number of pixel chunks each segment's sum is split into
     * (0 = chosen by the library). */
    CSMAP_OPT_ADJ_SPLIT = 6,
    /* FP32C forward: 0 = one reciprocal per pair; 1 = the terms of up to four
     * consecutive far segments are combined into one fraction per pixel
     * (p/q + m/d = (p d + m q)/(q d)) and divided once. */
    CSMAP_OPT_ACCUM = 7,
    /* How pixels are grouped into the tiles that wavefronts own:
     *   0 = automatic (ring blocks, 2);
     *   1 = strips of 64 x (pixels per lane) consecutive RING pixels;
     *   2 = ring blocks: G consecutive rings (CSMAP_OPT_BLOCK_RINGS) x up to
     *       64 x (pixels per lane) / G consecutive pixels per ring,
     *       azimuth-aligned across the rings (see csmap_ring_block_rows), so
     *       that a tile is a compact patch of sky; each ring of a tile has
     *       64 / G lanes, so the pixels of a lane share one ring.
     * Results agree up to rounding. */
    CSMAP_OPT_TILING = 8,
    /* FP32C form: a step in which every pair has 1 - n.P/R at or above this
     * value (default 5e-3, about 0.1 rad) and above CSMAP_OPT_NEAR_W uses
     * the algebraically equal form built from the dot products n.P/R, n.X',
     * n.Xdot; a step with some pair below it and none below
     * CSMAP_OPT_NEAR_W forms n - P/R in FP32.  Minimum 1e-6. */
    CSMAP_OPT_FAR_W = 9,
    /* Rings per tile G of the ring-block tiling: 0 (default: 2 x pixels per
     * lane, i.e. rows of 32 pixels) or a power of two in 1 .. 64. */
    CSMAP_OPT_BLOCK_RINGS = 10
} csmap_option;

/* Counters of the last render/backward (csmap_get_stats synchronises). */
typedef struct {
    int64_t nside, npix, nbox;
    int64_t segments;          /* segments added */
    int64_t kept;              /* segments inside their box's light-cone slab */
    int64_t pairs;             /* (visible pixel, kept segment) pairs evaluated */
    int64_t near_steps;        /* FP32C: (wavefront, segment) steps that took the FP64 path */
    double ms_precompute;      /* device time of the light-cone / record kernels */
    double ms_forward;         /* device time of the pair kernel of the last render */
    double ms_backward;        /* device time of the adjoint kernels of the last backward */
    int64_t pix_per_lane, waves, schedule, graph, chunk;
    double near_w;
    int64_t tiling;            /* tiling in use: 1 strips, 2 ring blocks */
    int64_t mid_steps;         /* FP32C: steps that formed n - P/R in FP32 */
    double far_w;
    int64_t steps;             /* FP32C: (wavefront, segment) steps of every form */
} csmap_stats;

/* Number of pixels of an Nside map, 12 Nside^2 (Sec. II.D); -1 if Nside is
 * outside [1, 8192]. */
int64_t csmap_npix(int64_t nside);

/* Create a sky of 12 Nside^2 RING pixels observed at conformal time eta0,
 * evaluated in the given form, enqueuing work on hip_stream (a hipStream_t,
 * NULL for the default stream).  Nside in [1, 8192].  *out receives a handle
 * owned by the caller until csmap_destroy_sky. */
csmap_status csmap_create_sky(int64_t nside, double eta0, csmap_form form, void *hip_stream,
                              csmap_sky **out);

/* Add one box of light-cone events (Sec. II.B-C: the events a simulation
 * recorded; Sec. III: events in, map out).  The arrays are copied into
 * library-owned device memory; box_id (may be NULL) receives the box's index
 * (0, 1, ... in call order). */
csmap_status csmap_add_box(csmap_sky *sky, const csmap_box *box, int64_t *box_id);

/* Add one box of segments known at the start eta_lo of its slab, rather than
 * on the light cone (Sec. II.B: as the strings evolve, photons are followed
 * and every segment crossing the past light cone is recorded).  Segment s is
 * taken to move on the straight worldline P0 + Xdot (eta - eta_lo),
 * P0 = origin + x_rel, during the slab; its event is where that worldline
 * meets the past light cone |P| = eta0 - eta, found in FP64 (see
 * csmap_cone_events), and the box contributes the events with
 * eta_lo <= eta < eta_hi, with the segment's Xdot, X' and dsigma.  Segments
 * with |Xdot| >= 1 record no event.  Arrays are copied as by csmap_add_box.
 * CSMAP_E_UNSUPPORTED for the CSMAP_VIS_BOX rule (events move out of the
 * box); csmap_backward is not provided for skies holding such boxes. */
csmap_status csmap_add_snapshot_box(csmap_sky *sky, const csmap_box *box, int64_t *box_id);

/* The light-cone events of a box of slab-start segments, on their own (the
 * crossing csmap_add_snapshot_box uses).  For segment i, with
 * P0 = origin + x_rel[i], D the smaller root of
 *     (Xdot.Xdot - 1) D^2 + 2 (P0.Xdot + R0) D + (P0.P0 - R0^2) = 0,
 * R0 = eta0 - eta_lo (the root where |P0 + Xdot D| = eta0 - eta_lo - D):
 * keep[i] = 1 iff |Xdot| < 1 and 0 <= D < eta_hi - eta_lo; then delta[i] = D
 * and pos[3i..3i+2] = P0 + Xdot D (observer-relative, FP64), else NaN.
 * Reads box->n, dtype, x_rel, xdot (device), origin, eta_lo, eta_hi; pos
 * (n x 3 doubles), delta (n doubles) and keep (n bytes) are device arrays
 * owned by the caller.  Enqueued on hip_stream; no synchronisation. */
csmap_status csmap_cone_events(const csmap_box *box, double eta0, double *pos, double *delta,
                               uint8_t *keep, void *hip_stream);

/* Placement of a simulation box in one healpix cone of a stacking grid
 * (Sec. II.C, Fig. 1: the comoving ball between two redshifts is cut into
 * cones subtending the pixels of a coarse HEALPix grid, each filled by a
 * rotated simulation box, and only the strings inside a box's cone count). */
typedef struct {
    int64_t nside;          /* Nside of the stacking grid, 1 .. 8192; 0: rotation only */
    int64_t pix;            /* RING pixel of the cone, 0 .. 12 nside^2 - 1 */
    double rot[9];          /* row-major rotation, box coordinates to sky:
                               P = origin + rot x_rel, Xdot -> rot Xdot, X' -> rot X';
                               orthonormal with determinant +1 (to 1e-9) */
} csmap_cone;

/* Add one box of a stacked simulation (Sec. II.C).  x_rel, xdot and xprime
 * are in the box's own coordinates; the box is turned onto the sky by
 * cone->rot (in FP64, per segment, by the light-cone stage of render) and
 * placed at box->origin, and only events whose position P lies in RING pixel
 * cone->pix of the Nside cone->nside grid are kept, besides the slab test.
 * snapshot = 0: the arrays hold events on the light cone, as csmap_add_box;
 * snapshot = 1: they hold slab-start segments, as csmap_add_snapshot_box
 * (the crossing is found after the rotation, and the cone test applies to
 * the event).  CSMAP_VIS_BOX is rejected (CSMAP_E_UNSUPPORTED; its box is
 * axis-aligned in the sky frame).  csmap_backward returns gradients with
 * respect to the box-frame arrays.  Arrays are copied as by csmap_add_box. */
csmap_status csmap_add_cone_box(csmap_sky *sky, const csmap_box *box, const csmap_cone *cone,
                                int snapshot, int64_t *box_id);

/* Run the light-cone stage of render on its own: every box's segments are
 * placed (rotation for cone boxes), tested against the slab and the cone,
 * and the kept ones written as the records the pair kernels read.  Enqueued
 * on the sky's stream; csmap_get_stats then reports `kept` and, as
 * ms_precompute, the device time of this stage (ms_forward 0).  Render
 * repeats the stage itself, so this call is only needed to inspect or time
 * it. */
csmap_status csmap_precompute(csmap_sky *sky);

/* RING pixel of each of n directions (Gorski et al. 2005; the inverse of
 * csmap_pix2vec_ring) at Nside in [1, 8192]: xyz is a device array of n x 3
 * doubles (vectors of any positive, finite length), pix a device array of n
 * int64 owned by the caller.  The same device routine makes the cone test of
 * csmap_add_cone_box.  Enqueued on hip_stream. */
csmap_status csmap_ang2pix_ring(int64_t nside, int64_t n, const double *xyz, int64_t *pix,
                                void *hip_stream);

/* Host-side helper, no device work: placement of a cubic box of side `side`
 * in cone `pix` of the Nside stacking grid for the shell
 * r_in <= |P| <= r_out (Sec. II.C: photons face the observer, the farthest
 * pixel fits in the farthest face).  Box axis `axis` (0, 1 or 2; one run is
 * used three times, once per axis) points out along the cone axis n (the
 * pixel centre), so photons travelling along -axis in the box travel
 * towards the observer; the other two axes follow (e_theta + e_phi)/sqrt(2)
 * and (e_phi - e_theta)/sqrt(2) at the pixel centre, in cyclic order (a
 * right-handed frame).  The far face (x_axis = side) is the plane
 * n.P = r_out, centred on the axis.  Writes cone->nside, cone->pix and
 * cone->rot, origin[3] (where box coordinate 0 lands), and *slack: the
 * smallest margin, in length units, of the conditions that put the whole
 * truncated cone inside the box (lateral half-width minus r_out times the
 * pixel's largest transverse extent, and r_in times its smallest cosine from
 * the axis minus the near face's distance), computed from 257 points on
 * each edge of the pixel's closed-form boundary; slack >= 0 means the cone
 * fits.  0 < r_in < r_out, side > 0. */
csmap_status csmap_cone_place(int64_t nside, int64_t pix, int axis, double r_in, double r_out,
                              double side, csmap_cone *cone, double origin[3], double *slack);

/* Host-side helper, no device work: the smallest Nside (a power of two, at
 * most 256) whose every cone fits a box of side `side` for the shell
 * r_in .. r_out by the test of csmap_cone_place (the largest healpix cone
 * fitting inside the box, Sec. II.C); *nside = 0 if none does. */
csmap_status csmap_cone_min_nside(double r_in, double r_out, double side, int64_t *nside);

/* Evaluate Theta/GU (Eq. (1)) at every RING pixel centre from all boxes
 * added so far and write it to map (device, 12 Nside^2 doubles, RING order).
 * Each pixel's value is its own sum; results are deterministic for a given
 * sky and options. */
csmap_status csmap_render(csmap_sky *sky, double *map);

/* Theta/GU (Eq. (1)) at n arbitrary directions: xyz is a device array of
 * n x 3 doubles (vectors of any positive, finite length; each is normalised
 * on the device), out a device array of n doubles, 0 <= n <= 2^31.  The same
 * light-cone stage and pair kernels as render, in the sky's form, with the
 * directions cut into strips in the caller's order; every box is walked for
 * every strip and its visibility rule applied per direction.  Used, e.g., to
 * evaluate the full-sky sum at the pixel directions of a gnomonic patch.
 * stats report the stages as for render.  Enqueued on the sky's stream. */
csmap_status csmap_render_dirs(csmap_sky *sky, int64_t n, const double *xyz, double *out);

/* A square-pixel patch of the sky in gnomonic projection (Sec. III.B,
 * Fig. 3). */
typedef struct {
    double center[3];       /* patch axis c, a unit vector */
    double e1[3], e2[3];    /* plane axes: unit vectors, orthogonal to c and each other */
    int64_t nx, ny;         /* pixels along e1 and e2, each >= 1, nx * ny <= 2^31 */
    double pix;             /* pixel size in radians (> 0) */
    double accept_cos;      /* a segment enters only if c.P > accept_cos |P|; in (0, 1]
                             * with tan(acos(accept_cos))/pix + max(nx, ny) <= 2^30 */
} csmap_patch;

/* Flat-sky, small-angle map of the sky's boxes on a patch (Sec. II.A: the
 * limit X n -> X with every photon path parallel to c; the paper compares
 * such maps with its full-sky map in Fig. 3).  A kept segment at P in front
 * of the observer (D = c.P > 0, D > accept_cos |P|) is seen at the plane
 * position s = (e1.P, e2.P)/D; pixel (i, j) is at
 * t = ((i + 1/2 - nx/2) pix, (j + 1/2 - ny/2) pix) and receives, from each
 * segment, -4 eps dsigma (u_perp . (t - s)) / (D |t - s|^2) with
 * u = Xdot - (c.X')/(1 + c.Xdot) X' and u_perp = (e1.u, e2.u); a pixel at
 * t = s receives 0.  Writes map (device, ny x nx doubles, index j nx + i).
 * Segment geometry (slab, cone boxes, snapshot crossings) is that of render,
 * in FP64; the pair sum is FP32 with compensated accumulation, whatever the
 * sky's form.  stats report the light-cone stage and the record pass as
 * ms_precompute and the pair kernel as ms_forward.  Enqueued on the sky's
 * stream.  CSMAP_E_INVALID for accept_cos outside (0, 1] or an acceptance
 * cone so wide that tan(acos(accept_cos))/pix + max(nx, ny) > 2^30 (the
 * bound on plane offsets in pixel units that keeps the FP32 pair arithmetic
 * in range). */
csmap_status csmap_render_flat(csmap_sky *sky, const csmap_patch *patch, double *map);

/* Adjoint of render: given dmap = dL/d(Theta_p/GU) (device, npix doubles),
 * write dL/d(x_rel, xdot, xprime, dsigma) of every segment of box b into
 * grads[b] for b = 0 .. nbox-1 (nbox must equal the number of boxes).
 * Segments outside their slab get zero gradient.  The paper does not
 * differentiate Eq. (1); this is its exact derivative. */
csmap_status csmap_backward(csmap_sky *sky, const double *dmap, const csmap_grad *grads,
                            int64_t nbox);

/* Drop all boxes (device memory is kept for reuse). */
csmap_status csmap_reset(csmap_sky *sky);

/* Free the sky and everything it owns.  NULL is accepted. */
csmap_status csmap_destroy_sky(csmap_sky *sky);

/* Message of the last failed call on this thread ("" if none). */
const char *csmap_last_error(void);

/* Write the unit vectors of RING pixels first .. first+count-1 of an Nside
 * map (Sec. II.D; HEALPix definition of Gorski et al. 2005, cited in the
 * paper) to xyz (device, count x 3 doubles), enqueued on hip_stream.  The
 * same device routine supplies the ray directions of render/backward. */
csmap_status csmap_pix2vec_ring(int64_t nside, int64_t first, int64_t count, double *xyz,
                                void *hip_stream);

/* Set a tunable (see csmap_option).  Invalidates any captured graph. */
csmap_status csmap_set_option(csmap_sky *sky, csmap_option opt, double value);

/* Counters and timings of the last render/backward; synchronises the stream. */
csmap_status csmap_get_stats(csmap_sky *sky, csmap_stats *out);

/* Time the forward kernel on this sky's boxes and keep the settings with the
 * most pairs per second, each candidate measured on a sample of its own
 * tiles spread evenly over the sky (about 25M pixels, each tile limited to
 * the first 2,048 segments of every box it sees).  First the launch shape
 * (pixels per lane, wavefronts per workgroup, accumulation mode; persistent
 * schedule), the shapes within 3% of the best measured again on 8,192
 * segments per box and tile; then, from the best shape, one setting at a
 * time: the tiling and rings per ring-block tile, the FP32
 * partial-sum length before each compensated update (16, 32 or 64; FP32C),
 * and the pair-form thresholds among those at least as accurate as the
 * defaults (CSMAP_OPT_FAR_W >= 5e-3, CSMAP_OPT_NEAR_W >= 5e-5), so tuning
 * never trades accuracy for speed.  If cache_path is not NULL the choice is
 * first looked up in, and afterwards appended to, that text file, keyed by
 * device architecture, form, Nside, box count, the number of boxes under
 * each visibility rule, the caps' summed sky fraction (two significant
 * digits) and the segment count (rounded to a power of two).  Allocates a
 * scratch map of 12 Nside^2 doubles for the duration of the call;
 * synchronises the stream; results of later renders agree with the untuned
 * ones to the form's accuracy (the sum order within a pixel may change). */
csmap_status csmap_autotune(csmap_sky *sky, const char *cache_path);

/* Spherical-harmonic analysis of a RING map (the angular power spectrum of
 * Sec. III, Fig. 4): for 0 <= m <= l <= lmax,
 *     a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(n_p)),
 * Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi} orthonormal with the
 * Condon-Shortley phase, n_p the pixel centres.  map: device, 12 Nside^2
 * doubles (RING order); alm: device, (lmax + 1)(lmax + 2) doubles, a_lm's
 * real and imaginary parts at positions 2 i and 2 i + 1 with
 * i = m (2 lmax + 1 - m) / 2 + l.  0 <= lmax <= 4 Nside.  Enqueued on
 * hip_stream, which must belong to the current device; does not
 * synchronise.  The work's device scratch (about 16 (4 Nside)(lmax + 1) +
 * 8 (ceil(Nside / 256) + 1)(lmax + 1)(lmax + 2) bytes: 1.7 GB at Nside
 * 2048, lmax 4096) is taken in stream order from a
 * memory pool that the library creates per device on first use and released
 * to it when the work ends; the pool keeps the memory for later calls until
 * the process ends.  CSMAP_E_NOMEM when the scratch cannot be had; errors of
 * the device work itself surface at the caller's next synchronisation. */
csmap_status csmap_map2alm(int64_t nside, int64_t lmax, const double *map, double *alm,
                           void *hip_stream);

/* csmap_map2alm for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, with the scratch taken from a fixed
 * 64 MiB device array of the library (one per GPU, held until the process
 * ends) instead of an allocation.  Calls no hipMalloc, hipFree or allocating
 * routine and does not synchronise: the work is enqueued on hip_stream, which
 * must belong to the current device.  Arguments, layout and errors as
 * csmap_map2alm, plus CSMAP_E_INVALID when (nside, lmax) needs more scratch
 * than 64 MiB (Nside 512 with lmax 1024 fits; Nside 1024 with lmax 1024
 * does not).  Every call on one GPU shares its array and nothing in it needs to
 * start at zero; calls that overlap on one GPU (different streams, or
 * threads) race on it and must be serialised by the caller. */
csmap_status csmap_map2alm_noalloc(int64_t nside, int64_t lmax, const double *map, double *alm,
                                   void *hip_stream);

/* C_l = (|a_l0|^2 + 2 sum_{m=1}^{l} |a_lm|^2) / (2l + 1) for l = 0 .. lmax of
 * a real map's a_lm (layout of csmap_map2alm); cl: device, lmax + 1
 * doubles.  Enqueued on hip_stream. */
csmap_status csmap_alm2cl(int64_t lmax, const double *alm, double *cl, void *hip_stream);

/* Host-side helper, no device work: the RING pixel tiles of `tile` pixels
 * that may contain pixels within angle rho (radians) of the unit vector
 * (cx, cy, cz) at Nside.  Writes up to max_ranges [first, last] tile index
 * pairs (inclusive, ascending, disjoint) to ranges and their number to
 * *n_ranges; returns CSMAP_E_INVALID if max_ranges is too small (with
 * *n_ranges set to the number needed).  The result is conservative: it may
 * include tiles with no such pixel, never omits one. */
csmap_status csmap_cap_tiles(int64_t nside, int64_t tile, double cx, double cy, double cz,
                             double rho, int64_t *ranges, int64_t max_ranges,
                             int64_t *n_ranges);

/* Host-side helper, no device work: the ring-block tiling of
 * CSMAP_OPT_TILING = 2 at Nside with `rings` rings per block (1 .. 64) and
 * rows of at most `width` pixels (1 .. 1023; the library uses
 * width = 64 x pixels per lane / rings).  Rings 1 .. 4 Nside - 1 are grouped
 * `rings` at a time; a block whose longest ring has L pixels is cut into
 * ceil(L / width) tiles, and tile c of the block holds, of each ring of n
 * pixels, the offsets floor(width c n / L) up to (not including)
 * min(n, floor(width (c + 1) n / L)).  Writes `rings` entries per tile,
 * (first RING pixel of the row << 10) | (pixels in the row), or 0 for an
 * empty row, for all tiles to rows (rings * max_tiles entries available;
 * rows may be NULL when max_tiles is 0) and the tile count to *n_tiles;
 * returns CSMAP_E_INVALID if max_tiles is too small (with *n_tiles set). */
csmap_status csmap_ring_block_rows(int64_t nside, int64_t rings, int64_t width, int64_t *rows,
                                   int64_t max_tiles, int64_t *n_tiles);

/* Host-side helper, no device work: as csmap_cap_tiles, for the tiles of
 * the ring-block tiling (csmap_ring_block_rows). */
csmap_status csmap_cap_block_tiles(int64_t nside, int64_t rings, int64_t width, double cx,
                                   double cy, double cz, double rho, int64_t *ranges,
                                   int64_t max_ranges, int64_t *n_ranges);

/* Measurement helper, outside the map path: a kernel of known vector-ALU
 * work against which hardware instruction counters and the achievable issue
 * rate are read.  kind 0 runs FP32 fused multiply-adds with vector-register
 * operands, kind 1 FP64 ones, kind 2 FP32 ones whose multiplier is read
 * from a scalar register: `blocks` workgroups of 256 threads, each lane
 * `iters` iterations of 16 independent FMAs, then one value per lane written
 * to out (device, blocks * 256 floats, or doubles for kind 1).  Synchronises
 * hip_stream; *ms (may be NULL) receives the kernel's time from HIP events
 * around it, *fma_insts (may be NULL) the FMA instructions issued, counted
 * per wavefront (blocks * 4 * iters * 16; each is 64 lanes x 2 FLOP).
 * CSMAP_E_INVALID for kind outside {0, 1, 2}, blocks outside [1, 2^24],
 * iters outside [1, 2^30] or a NULL out. */
csmap_status csmap_valu_probe(int kind, int64_t blocks, int64_t iters, void *out,
                              void *hip_stream, double *ms, double *fma_insts);

#ifdef __cplusplus
}
#endif

#endif /* CSMAP_H */
