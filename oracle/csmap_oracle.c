/*
 * csmap_oracle.c -- plain FP64 CPU oracle for the all-sky string ISW sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU baseline
 * of the benchmark do.  It shares no source, header or table with the HIP
 * implementation: the two are written independently from the same physics
 * (Ringeval & Bouchet, "All sky CMB map from cosmic strings integrated
 * Sachs-Wolfe effect") and the same published HEALPix definition (Gorski et
 * al. 2005, cited in the paper's Sec. I and Sec. II.D).
 *
 * What it computes (all in IEEE double precision, compiled without
 * floating-point contraction so every rounding is spelled out):
 *
 *   - HEALPix RING pixel centres (Sec. II.D: the map directions are the
 *     centres of an Nside HEALPix RING pixelisation).
 *   - The light-cone selection of a simulation box: an event recorded at
 *     observer-relative position P lies on the past light cone at conformal
 *     time eta = eta0 - |P| (Sec. II.A, gauge footnote X^0 = eta = tau); a box
 *     contributes the events with eta_lo <= eta < eta_hi.
 *   - Eq. (1) with Eq. (2), discretised over segments (Sec. II.A: every
 *     segment on the light cone enters every pixel, no cut):
 *         Theta(n)/GU = sum_s -4 u.(R n - P)/|R n - P|^2 * eps * dsigma,
 *         u = Xdot - (n.X')X'/(1 + n.Xdot),  eps^2 = X'^2/(1 - Xdot^2),
 *     with R = |P| (the non-bold X of Eq. (1)), each pixel sampled at its
 *     centre (Sec. III.B: each pixel represents the signal in its centroid
 *     direction).  A term whose |R n - P|^2 is exactly zero contributes 0.
 *     P is the FP64 sum origin + x_rel and R the FP64 square root of the
 *     FP64 sum of squares (these are the inputs of the sum); R n - P is
 *     formed with one rounding, so each term is accurate to a few units in
 *     the last place even for events a tiny angle off the line of sight.
 *   - The gradient of a linear functional sum_p g_p Theta_p with respect to
 *     every segment's (x_rel, Xdot, X', dsigma), by the chain rule applied to
 *     the same expression (the paper does not differentiate; this is the
 *     adjoint of its Eq. (1)).
 *
 * Sums over segments are Neumaier-compensated.  Pixels are distributed over
 * OpenMP threads; the order of terms inside one pixel is fixed (box order,
 * then segment order), so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Integer stage of the RING scheme.                                         */
/* Rings are numbered i = 1 .. 4N-1 from north to south.  North-cap ring     */
/* i < N holds 4i pixels, the 2N+1 rings N..3N of the equatorial belt hold  */
/* 4N pixels each, and the south cap mirrors the north.  Pixel indices run  */
/* ring by ring from the north pole, and by increasing azimuth in a ring.   */
/* ------------------------------------------------------------------------ */

/* floor(sqrt(x)) for 0 <= x < 2^62, exact. */
int64_t oracle_isqrt(int64_t x)
{
    if (x <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)x);
    while (r * r > x) --r;
    while ((r + 1) * (r + 1) <= x) ++r;
    return r;
}

/* Number of pixels in the north polar cap: sum_{i<N} 4i = 2N(N-1). */
static int64_t cap_pixels(int64_t n) { return 2 * n * (n - 1); }

/* Ring index (1-based, north to south) and 0-based position in the ring. */
void oracle_ring_of_pixel(int64_t nside, int64_t p, int64_t *ring, int64_t *pos)
{
    const int64_t ncap = cap_pixels(nside);
    const int64_t npix = 12 * nside * nside;
    if (p < ncap) {
        /* Largest i with 2i(i-1) <= p. */
        int64_t i = (1 + oracle_isqrt(1 + 2 * p)) / 2;
        *ring = i;
        *pos = p - 2 * i * (i - 1);
    } else if (p < npix - ncap) {
        int64_t q = p - ncap;
        *ring = nside + q / (4 * nside);
        *pos = q % (4 * nside);
    } else {
        /* Mirror image of a north-cap pixel; azimuth order is preserved. */
        int64_t m = npix - 1 - p;               /* index counted from the end */
        int64_t i = (1 + oracle_isqrt(1 + 2 * m)) / 2;
        int64_t back = m - 2 * i * (i - 1);     /* position counted from the ring's end */
        *ring = 4 * nside - i;
        *pos = 4 * i - 1 - back;
    }
}

/* ------------------------------------------------------------------------ */
/* Float stage.  Every quantity is a correctly rounded IEEE operation on     */
/* exact integers, or a fixed fma polynomial, so that any implementation     */
/* that follows the same steps reproduces the same bits.                     */
/* ------------------------------------------------------------------------ */

/* Taylor coefficients of sin(pi x / 2) = x * S(x^2): the double nearest to
 * (-1)^k (pi/2)^(2k+1) / (2k+1)!, k = 0..8. */
static const double SIN_C[9] = {
     0x1.921fb54442d18p+0, -0x1.4abbce625be53p-1,  0x1.466bc6775aae2p-4,
    -0x1.32d2cce62bd86p-8,  0x1.50783487ee782p-13, -0x1.e3074fde8871fp-19,
     0x1.e8f434d018d63p-25, -0x1.6fadb9f155744p-31, 0x1.aaec32af93359p-38,
};
/* Taylor coefficients of cos(pi x / 2) = C(x^2): the double nearest to
 * (-1)^k (pi/2)^(2k) / (2k)!, k = 0..8. */
static const double COS_C[9] = {
     0x1.0000000000000p+0, -0x1.3bd3cc9be45dep+0,  0x1.03c1f081b5ac4p-2,
    -0x1.55d3c7e3cbffap-6,  0x1.e1f506891babbp-11, -0x1.a6d1f2a204a8cp-16,
     0x1.f9d38a3763cc3p-22, -0x1.b6e24f44b128fp-28, 0x1.20c62c2f2d7f5p-34,
};

/* sin and cos of (pi/2) x for 0 <= x <= 1/2 (an angle of at most pi/4). */
static void sincos_quarter(double x, double *s, double *c)
{
    const double y = x * x;
    double ps = SIN_C[8], pc = COS_C[8];
    for (int k = 7; k >= 0; --k) {
        ps = fma(ps, y, SIN_C[k]);
        pc = fma(pc, y, COS_C[k]);
    }
    *s = x * ps;
    *c = pc;
}

/* Unit vector of an azimuth phi = (pi/2) * num/den, 0 <= num < 4 den.
 * The quadrant is split off with integers, the remainder is folded into
 * [0, pi/4] by the complement identity, and only then evaluated. */
static void azimuth(int64_t num, int64_t den, double *cphi, double *sphi)
{
    const int64_t quad = num / den;
    const int64_t rem = num - quad * den;
    double s, c, cq, sq;
    if (2 * rem <= den) {
        sincos_quarter((double)rem / (double)den, &s, &c);
        cq = c; sq = s;
    } else {
        sincos_quarter((double)(den - rem) / (double)den, &s, &c);
        cq = s; sq = c;
    }
    switch (quad & 3) {
    case 0: *cphi = cq;  *sphi = sq;  break;
    case 1: *cphi = -sq; *sphi = cq;  break;
    case 2: *cphi = -cq; *sphi = -sq; break;
    default: *cphi = sq; *sphi = -cq; break;
    }
}

/* Direction of the centre of RING pixel p (observer at the origin). */
void oracle_pix2vec(int64_t nside, int64_t p, double v[3])
{
    int64_t i, j;
    oracle_ring_of_pixel(nside, p, &i, &j);
    const int64_t n = nside;
    double z, st;
    int64_t num, den;
    if (i < n || i > 3 * n) {
        /* Polar caps.  k is the ring counted from the nearer pole:
         *   z = +-(3N^2 - k^2)/(3N^2),  sin(theta) = k sqrt(6N^2 - k^2)/(3N^2),
         *   phi = (pi/2)(2j + 1)/(2k). */
        const int64_t k = (i < n) ? i : 4 * n - i;
        const double d = (double)(3 * n * n);
        z = (double)(3 * n * n - k * k) / d;
        st = ((double)k * sqrt((double)(6 * n * n - k * k))) / d;
        if (i > 3 * n) z = -z;
        num = 2 * j + 1;
        den = 2 * k;
    } else {
        /* Equatorial belt: z = 2(2N - i)/(3N), sin(theta) = sqrt(9N^2 - 4(2N-i)^2)/(3N).
         * Ring N is shifted by half a pixel like the cap rings, and the shift
         * alternates ring by ring: phi = (pi/2)(2j + shift)/(2N). */
        const int64_t m = 2 * n - i;
        const double d = (double)(3 * n);
        z = (double)(2 * m) / d;
        st = sqrt((double)(9 * n * n - 4 * m * m)) / d;
        const int64_t shift = ((i - n) % 2 == 0) ? 1 : 0;
        num = 2 * j + shift;
        den = 2 * n;
    }
    double cphi, sphi;
    azimuth(num, den, &cphi, &sphi);
    v[0] = st * cphi;
    v[1] = st * sphi;
    v[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Box description.  One box is 16 doubles:                                   */
/*   [0..2] origin (observer-relative FP64 position of the box corner that   */
/*          x_rel is measured from), [3..5] box extent along x, y, z,        */
/*   [6] eta_lo, [7] eta_hi (conformal-time slab of its light-cone events),  */
/*   [8] visibility mode (0 all pixels, 1 pixels whose ray crosses the box   */
/*       within the slab's radii, 2 pixels inside a cap),                    */
/*   [9..11] cap centre (unit vector), [12] cosine of the cap radius.        */
/* ------------------------------------------------------------------------ */
enum { BOX_STRIDE = 16 };

/* Does the ray t n (t >= 0) cross the closed axis-aligned box at some
 * distance inside the slab's radii (r_lo, r_hi]? */
static int ray_sees_box(const double n[3], const double *box, double eta0)
{
    const double r_lo = eta0 - box[7];
    const double r_hi = eta0 - box[6];
    double t_in = 0.0, t_out = INFINITY;
    for (int k = 0; k < 3; ++k) {
        const double lo = box[k];
        const double hi = box[k] + box[3 + k];
        if (n[k] == 0.0) {
            if (lo > 0.0 || hi < 0.0) return 0;
            continue;
        }
        const double ta = lo / n[k];
        const double tb = hi / n[k];
        const double tmin = (ta < tb) ? ta : tb;
        const double tmax = (ta < tb) ? tb : ta;
        if (tmin > t_in) t_in = tmin;
        if (tmax < t_out) t_out = tmax;
    }
    return (t_in <= t_out) && (t_out > r_lo) && (t_in <= r_hi);
}

int oracle_pixel_sees_box(const double n[3], const double *box, double eta0)
{
    const int mode = (int)box[8];
    if (mode == 0) return 1;
    if (mode == 1) return ray_sees_box(n, box, eta0);
    const double dot = (n[0] * box[9] + n[1] * box[10]) + n[2] * box[11];
    return dot >= box[12];
}

/* Light-cone selection and per-segment constants of one segment.
 * Returns 1 if the event is on the part of the past light cone the box
 * covers (eta_lo <= eta0 - R < eta_hi with R > 0). */
typedef struct {
    double P[3];   /* observer-relative position */
    double R;      /* |P| = eta0 - eta */
    double V[3];   /* Xdot */
    double T[3];   /* X' */
    double eps;    /* sqrt(X'^2 / (1 - Xdot^2)) */
    double w;      /* dsigma */
} seg_t;

static int load_segment(const double *box, double eta0, const double *x,
                        const double *xd, const double *xp, double ds, seg_t *s)
{
    for (int k = 0; k < 3; ++k) {
        s->P[k] = box[k] + x[k];
        s->V[k] = xd[k];
        s->T[k] = xp[k];
    }
    s->R = sqrt((s->P[0] * s->P[0] + s->P[1] * s->P[1]) + s->P[2] * s->P[2]);
    const double eta = eta0 - s->R;
    if (!(s->R > 0.0) || !(eta >= box[6]) || !(eta < box[7])) return 0;
    const double tt = (s->T[0] * s->T[0] + s->T[1] * s->T[1]) + s->T[2] * s->T[2];
    const double vv = (s->V[0] * s->V[0] + s->V[1] * s->V[1]) + s->V[2] * s->V[2];
    s->eps = sqrt(tt / (1.0 - vv));
    s->w = ds;
    return 1;
}

int oracle_segment_kept(const double *box, double eta0, const double *x,
                        const double *xd, const double *xp, double ds)
{
    seg_t s;
    return load_segment(box, eta0, x, xd, xp, ds, &s);
}

static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* One term of the discrete Eq. (1) in units of GU. */
static double term(const double n[3], const seg_t *s)
{
    /* R n - P with a single rounding: for an event close to the line of
     * sight the two terms nearly cancel, and a separately rounded product
     * would leave an error of order eps R in a vector of length ~R theta. */
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = fma(s->R, n[k], -s->P[k]);
    const double q = dot3(d, d);
    if (q == 0.0) return 0.0;
    const double a = dot3(n, s->T);
    const double b = 1.0 + dot3(n, s->V);
    double u[3];
    for (int k = 0; k < 3; ++k) u[k] = s->V[k] - (a / b) * s->T[k];
    return -4.0 * (dot3(u, d) / q) * s->eps * s->w;
}

/* Neumaier compensated summation. */
typedef struct { double sum, comp; } csum_t;
static void cadd(csum_t *acc, double x)
{
    const double t = acc->sum + x;
    if (fabs(acc->sum) >= fabs(x)) acc->comp += (acc->sum - t) + x;
    else acc->comp += (x - t) + acc->sum;
    acc->sum = t;
}

/*
 * Theta/GU at ndir arbitrary unit directions dirs[ndir*3].
 * Segments of box b are x_rel/xdot/xprime[3*s..], dsigma[s] for
 * s in [seg_off[b], seg_off[b+1]).  When use_vis is non-zero each
 * direction only receives the boxes it sees.
 */
void oracle_theta_dirs(int64_t ndir, const double *dirs, double eta0,
                       int64_t nbox, const double *boxes, const int64_t *seg_off,
                       const double *x_rel, const double *xdot, const double *xprime,
                       const double *dsigma, int use_vis, double *out)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < ndir; ++p) {
        const double *n = dirs + 3 * p;
        csum_t acc = {0.0, 0.0};
        for (int64_t b = 0; b < nbox; ++b) {
            const double *box = boxes + BOX_STRIDE * b;
            if (use_vis && !oracle_pixel_sees_box(n, box, eta0)) continue;
            for (int64_t i = seg_off[b]; i < seg_off[b + 1]; ++i) {
                seg_t s;
                if (!load_segment(box, eta0, x_rel + 3 * i, xdot + 3 * i, xprime + 3 * i,
                                  dsigma[i], &s))
                    continue;
                cadd(&acc, term(n, &s));
            }
        }
        out[p] = acc.sum + acc.comp;
    }
}

/* Theta/GU at the RING pixels pix[npix_list] of an Nside map. */
void oracle_theta_pixels(int64_t nside, int64_t nlist, const int64_t *pix, double eta0,
                         int64_t nbox, const double *boxes, const int64_t *seg_off,
                         const double *x_rel, const double *xdot, const double *xprime,
                         const double *dsigma, double *out)
{
    double *dirs = (double *)malloc(sizeof(double) * 3 * (size_t)(nlist > 0 ? nlist : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nlist; ++p) oracle_pix2vec(nside, pix[p], dirs + 3 * p);
    oracle_theta_dirs(nlist, dirs, eta0, nbox, boxes, seg_off, x_rel, xdot, xprime, dsigma,
                      1, out);
    free(dirs);
}

void oracle_pix2vec_many(int64_t nside, int64_t nlist, const int64_t *pix, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nlist; ++p) oracle_pix2vec(nside, pix[p], out + 3 * p);
}

void oracle_ring_many(int64_t nside, int64_t nlist, const int64_t *pix, int64_t *ring,
                      int64_t *pos)
{
    for (int64_t p = 0; p < nlist; ++p) oracle_ring_of_pixel(nside, pix[p], ring + p, pos + p);
}

/* Visibility of box b for each listed pixel (1/0). */
void oracle_visible_many(int64_t nside, int64_t nlist, const int64_t *pix, double eta0,
                         const double *box, uint8_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nlist; ++p) {
        double n[3];
        oracle_pix2vec(nside, pix[p], n);
        out[p] = (uint8_t)oracle_pixel_sees_box(n, box, eta0);
    }
}

/* Light-cone selection flag of each segment of one box (1/0). */
void oracle_kept_many(int64_t nseg, const double *box, double eta0, const double *x_rel,
                      const double *xdot, const double *xprime, const double *dsigma,
                      uint8_t *out)
{
    for (int64_t i = 0; i < nseg; ++i)
        out[i] = (uint8_t)oracle_segment_kept(box, eta0, x_rel + 3 * i, xdot + 3 * i,
                                              xprime + 3 * i, dsigma[i]);
}

/*
 * Gradient of sum_p g_p Theta_p/GU over the pixels pix[nlist] of an Nside map
 * with respect to (x_rel[3], xdot[3], xprime[3], dsigma) of each listed
 * segment sel[nsel] (global segment indices; box_of_sel[j] is its box).
 * out[10*j + (0..9)].  Segments off the light-cone slab get zero gradient.
 *
 * With C = -4 eps w, d = R n - P, q = d.d, N = u.d, f = C N / q:
 *   df/dP  = C [ ((u.n) Phat - u)/q - N (2 (d.n) Phat - 2 d)/q^2 ]
 *            (d depends on P through R n - P, and dR/dP = Phat)
 *   df/dV  = (C/q) [ d + (a (T.d)/b^2) n ] + f V/(1 - V^2)
 *   df/dT  = -(C/(b q)) [ (T.d) n + a d ] + f T/T^2
 *   df/dw  = -4 eps N / q   (f is linear in w; finite at w = 0)
 * where the last terms come from eps = sqrt(T^2/(1 - V^2)).
 */
static void grad_sums(int64_t nside, int64_t nlist, const int64_t *pix, const double *g,
                      double eta0, int64_t nbox, const double *boxes, const int64_t *seg_off,
                      const double *x_rel, const double *xdot, const double *xprime,
                      const double *dsigma, int64_t nsel, const int64_t *sel, int absolute,
                      double *out);

void oracle_grad(int64_t nside, int64_t nlist, const int64_t *pix, const double *g,
                 double eta0, int64_t nbox, const double *boxes, const int64_t *seg_off,
                 const double *x_rel, const double *xdot, const double *xprime,
                 const double *dsigma, int64_t nsel, const int64_t *sel, double *out)
{
    grad_sums(nside, nlist, pix, g, eta0, nbox, boxes, seg_off, x_rel, xdot, xprime, dsigma,
              nsel, sel, 0, out);
}

/*
 * The same sums with every pixel's contribution taken in absolute value,
 * sum_p |g_p df_p/dtheta| per component: the scale of each gradient
 * component before its terms cancel (the bound on the error of a sum whose
 * terms each carry a relative error e is e times this).
 */
void oracle_grad_abs(int64_t nside, int64_t nlist, const int64_t *pix, const double *g,
                     double eta0, int64_t nbox, const double *boxes, const int64_t *seg_off,
                     const double *x_rel, const double *xdot, const double *xprime,
                     const double *dsigma, int64_t nsel, const int64_t *sel, double *out)
{
    grad_sums(nside, nlist, pix, g, eta0, nbox, boxes, seg_off, x_rel, xdot, xprime, dsigma,
              nsel, sel, 1, out);
}

static void grad_sums(int64_t nside, int64_t nlist, const int64_t *pix, const double *g,
                      double eta0, int64_t nbox, const double *boxes, const int64_t *seg_off,
                      const double *x_rel, const double *xdot, const double *xprime,
                      const double *dsigma, int64_t nsel, const int64_t *sel, int absolute,
                      double *out)
{
    double *dirs = (double *)malloc(sizeof(double) * 3 * (size_t)(nlist > 0 ? nlist : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nlist; ++p) oracle_pix2vec(nside, pix[p], dirs + 3 * p);

    /* Pixels are cut into a fixed number of chunks whose compensated partial
     * sums are combined in chunk order, so the result is independent of the
     * number of threads. */
    enum { NCHUNK = 256 };
    csum_t *part = (csum_t *)malloc(sizeof(csum_t) * 10 * NCHUNK);

    for (int64_t j = 0; j < nsel; ++j) {
        const int64_t i = sel[j];
        int64_t b = 0;
        while (b < nbox - 1 && seg_off[b + 1] <= i) ++b;
        const double *box = boxes + BOX_STRIDE * b;
        double *o = out + 10 * j;
        for (int c = 0; c < 10; ++c) o[c] = 0.0;
        seg_t s;
        if (!load_segment(box, eta0, x_rel + 3 * i, xdot + 3 * i, xprime + 3 * i, dsigma[i], &s))
            continue;
        double Ph[3];
        for (int k = 0; k < 3; ++k) Ph[k] = s.P[k] / s.R;
        const double vv = dot3(s.V, s.V);
        const double tt = dot3(s.T, s.T);
        const double C = -4.0 * s.eps * s.w;
        memset(part, 0, sizeof(csum_t) * 10 * NCHUNK);

        #pragma omp parallel for schedule(dynamic, 1)
        for (int ch = 0; ch < NCHUNK; ++ch) {
            csum_t *loc = part + 10 * ch;
            const int64_t p0 = nlist * ch / NCHUNK, p1 = nlist * (ch + 1) / NCHUNK;
            for (int64_t p = p0; p < p1; ++p) {
                const double *n = dirs + 3 * p;
                if (!oracle_pixel_sees_box(n, box, eta0)) continue;
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = fma(s.R, n[k], -s.P[k]);
                const double q = dot3(d, d);
                if (q == 0.0) continue;
                const double a = dot3(n, s.T);
                const double bb = 1.0 + dot3(n, s.V);
                double u[3];
                for (int k = 0; k < 3; ++k) u[k] = s.V[k] - (a / bb) * s.T[k];
                const double N = dot3(u, d);
                const double f = C * N / q;
                const double un = dot3(u, n), dn = dot3(d, n), td = dot3(s.T, d);
                const double gp = g[p];
                for (int k = 0; k < 3; ++k) {
                    const double dP = C * ((un * Ph[k] - u[k]) / q
                                           - N * (2.0 * dn * Ph[k] - 2.0 * d[k]) / (q * q));
                    const double dV = (C / q) * (d[k] + (a * td / (bb * bb)) * n[k])
                                      + f * s.V[k] / (1.0 - vv);
                    const double dT = -(C / (bb * q)) * (td * n[k] + a * d[k]) + f * s.T[k] / tt;
                    cadd(&loc[k], absolute ? fabs(gp * dP) : gp * dP);
                    cadd(&loc[3 + k], absolute ? fabs(gp * dV) : gp * dV);
                    cadd(&loc[6 + k], absolute ? fabs(gp * dT) : gp * dT);
                }
                /* Eq. (1) is linear in dsigma: its derivative is the summand
                 * without the dsigma factor, finite at dsigma = 0. */
                const double dw = gp * (-4.0 * s.eps * N / q);
                cadd(&loc[9], absolute ? fabs(dw) : dw);
            }
        }
        for (int c = 0; c < 10; ++c) {
            csum_t acc = {0.0, 0.0};
            for (int ch = 0; ch < NCHUNK; ++ch) {
                cadd(&acc, part[10 * ch + c].sum);
                cadd(&acc, part[10 * ch + c].comp);
            }
            o[c] = acc.sum + acc.comp;
        }
    }
    free(part);
    free(dirs);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Light-cone event recording from a snapshot (the step that precedes the   */
/* sum, Sec. II.B: as the strings evolve, photons are propagated and every   */
/* segment crossing the observer's past light cone is recorded).  A segment  */
/* known at the start eta_lo of a time slab, at observer-relative position   */
/* P0 = origin + x_rel with velocity Xdot, moves on the straight worldline   */
/* P(eta) = P0 + Xdot (eta - eta_lo) during the slab.  The past light cone   */
/* at conformal time eta is the sphere |P| = eta0 - eta.  With              */
/* D = eta - eta_lo and R0 = eta0 - eta_lo, the crossing solves              */
/*     h(D) = |P0 + Xdot D| + D - R0 = 0.                                    */
/* For |Xdot| < 1, h is strictly increasing (its slope is at least           */
/* 1 - |Xdot| > 0), so there is exactly one crossing; it is an event of this */
/* slab when 0 <= D < eta_hi - eta_lo.  Here it is found by bisection on h,  */
/* which needs nothing but the sign of h: plain, slow and obviously right.   */
/* Segments with |Xdot| >= 1 record no event.                               */
/* ------------------------------------------------------------------------ */
static double cone_gap(const double P0[3], const double V[3], double D, double R0)
{
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = P0[k] + V[k] * D;
    return sqrt(dot3(p, p)) + D - R0;
}

/* For every segment: keep[i] = 1 if its worldline crosses the past light
 * cone inside the slab, with delta[i] the crossing's D and pos[3i..3i+2]
 * the observer-relative event position P0 + Xdot D; otherwise keep[i] = 0
 * and delta[i], pos[3i..3i+2] are NaN. */
void oracle_cone_events(int64_t n, const double *x_rel, const double *xdot,
                        const double origin[3], double eta0, double eta_lo, double eta_hi,
                        double *pos, double *delta, uint8_t *keep)
{
    const double R0 = eta0 - eta_lo;
    const double width = eta_hi - eta_lo;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double P0[3], V[3];
        for (int k = 0; k < 3; ++k) {
            P0[k] = origin[k] + x_rel[3 * i + k];
            V[k] = xdot[3 * i + k];
        }
        keep[i] = 0;
        delta[i] = NAN;
        for (int k = 0; k < 3; ++k) pos[3 * i + k] = NAN;
        if (!(dot3(V, V) < 1.0) || !(width > 0.0)) continue;
        /* The crossing lies in [0, width) iff h(0) <= 0 < h(width). */
        if (cone_gap(P0, V, 0.0, R0) > 0.0) continue;
        if (!(cone_gap(P0, V, width, R0) > 0.0)) continue;
        double lo = 0.0, hi = width;            /* h(lo) <= 0 < h(hi) */
        for (;;) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;  /* no double strictly between */
            if (cone_gap(P0, V, mid, R0) > 0.0) hi = mid;
            else lo = mid;
        }
        /* Of the two neighbours, the one where |h| is smaller. */
        const double D = (fabs(cone_gap(P0, V, lo, R0)) <= fabs(cone_gap(P0, V, hi, R0))) ? lo : hi;
        keep[i] = 1;
        delta[i] = D;
        for (int k = 0; k < 3; ++k) pos[3 * i + k] = P0[k] + V[k] * D;
    }
}

/* ------------------------------------------------------------------------ */
/* Spherical-harmonic analysis of a RING map (the angular power spectrum of  */
/* Sec. III, Fig. 4).  With Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m   */
/* phi}, lambda_lm the associated Legendre function normalised so that the   */
/* Y_lm are orthonormal on the sphere and carrying the Condon-Shortley phase  */
/* (-1)^m:                                                                    */
/*     a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(n_p)),  0 <= m <= l <= lmax */
/*     C_l  = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1),                   */
/* i.e. each pixel weighted by its area at its centre.  lambda_lm comes from  */
/* the textbook recursions                                                    */
/*     lambda_00 = 1/sqrt(4 pi),                                              */
/*     lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},            */
/*     lambda_{m+1,m} = sqrt(2m+3) cos(theta) lambda_mm,                      */
/*     lambda_lm = A_lm (cos(theta) lambda_{l-1,m} - B_lm lambda_{l-2,m}),    */
/*     A_lm = sqrt((4l^2-1)/(l^2-m^2)), B_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),*/
/* carried as v * 2^(600 e) so that the factor sin^m(theta), far below the   */
/* double range for large m near the poles, is not lost before the l         */
/* recursion brings the value back up.                                        */
/* a_lm is stored at index m (2 lmax + 1 - m) / 2 + l (the order HEALPix      */
/* software uses), real and imaginary parts in separate arrays.              */
/* ------------------------------------------------------------------------ */
#define LEG_SCALE 600
#define ORACLE_PI 3.14159265358979323846   /* rounds to the double nearest pi */

/* lambda_lm(cos theta) for l = m .. lmax into out[l - m]. */
void oracle_lambda_lm(int64_t lmax, int64_t m, double z, double s, double *out)
{
    double v = 1.0 / sqrt(4.0 * ORACLE_PI);
    int e = 0;
    for (int64_t k = 1; k <= m; ++k) {
        v = -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * v;
        if (fabs(v) < ldexp(1.0, -LEG_SCALE)) {
            v = ldexp(v, LEG_SCALE);
            e -= 1;
        }
    }
    double prev = 0.0, cur = v;   /* lambda_{l-1,m}, lambda_{l,m}, scaled alike */
    for (int64_t l = m; l <= lmax; ++l) {
        if (l > m) {
            double next;
            if (l == m + 1) {
                next = sqrt(2.0 * m + 3.0) * z * cur;
            } else {
                const double ll = (double)l, mm = (double)m;
                const double A = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
                const double B = sqrt(((ll - 1.0) * (ll - 1.0) - mm * mm) /
                                      (4.0 * (ll - 1.0) * (ll - 1.0) - 1.0));
                next = A * (z * cur - B * prev);
            }
            prev = cur;
            cur = next;
            if (fabs(cur) > ldexp(1.0, LEG_SCALE) && e < 0) {
                cur = ldexp(cur, -LEG_SCALE);
                prev = ldexp(prev, -LEG_SCALE);
                e += 1;
            }
        }
        out[l - m] = (e == 0) ? cur : ldexp(cur, LEG_SCALE * e);
    }
}

int64_t oracle_alm_index(int64_t lmax, int64_t l, int64_t m)
{
    return m * (2 * lmax + 1 - m) / 2 + l;
}

/* a_lm for one m and l = m .. lmax into re[l - m], im[l - m]. */
void oracle_map2alm_m(int64_t nside, int64_t lmax, int64_t m, const double *map, double *re,
                      double *im)
{
    const int64_t npix = 12 * nside * nside;
    const double w = 4.0 * ORACLE_PI / (double)npix;
    double *lam = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    csum_t *sre = (csum_t *)malloc(sizeof(csum_t) * (size_t)(lmax + 1));
    csum_t *sim = (csum_t *)malloc(sizeof(csum_t) * (size_t)(lmax + 1));
    for (int64_t l = m; l <= lmax; ++l) {
        sre[l] = (csum_t){0.0, 0.0};
        sim[l] = (csum_t){0.0, 0.0};
    }
    for (int64_t p = 0; p < npix; ++p) {
        double n[3];
        oracle_pix2vec(nside, p, n);
        const double s = sqrt(n[0] * n[0] + n[1] * n[1]);
        const double phi = atan2(n[1], n[0]);
        oracle_lambda_lm(lmax, m, n[2], s, lam);
        /* conj(e^{i m phi}) = cos(m phi) - i sin(m phi) */
        const double c = cos((double)m * phi), sn = sin((double)m * phi);
        for (int64_t l = m; l <= lmax; ++l) {
            const double t = map[p] * lam[l - m];
            cadd(&sre[l], t * c);
            cadd(&sim[l], -t * sn);
        }
    }
    for (int64_t l = m; l <= lmax; ++l) {
        re[l - m] = w * (sre[l].sum + sre[l].comp);
        im[l - m] = w * (sim[l].sum + sim[l].comp);
    }
    free(lam);
    free(sre);
    free(sim);
}

void oracle_map2alm(int64_t nside, int64_t lmax, const double *map, double *alm_re,
                    double *alm_im)
{
#pragma omp parallel
    {
        double *re = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        double *im = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m <= lmax; ++m) {
            oracle_map2alm_m(nside, lmax, m, map, re, im);
            for (int64_t l = m; l <= lmax; ++l) {
                const int64_t i = oracle_alm_index(lmax, l, m);
                alm_re[i] = re[l - m];
                alm_im[i] = im[l - m];
            }
        }
        free(re);
        free(im);
    }
}

void oracle_alm2cl(int64_t lmax, const double *alm_re, const double *alm_im, double *cl)
{
    for (int64_t l = 0; l <= lmax; ++l) {
        csum_t acc = {0.0, 0.0};
        for (int64_t m = 0; m <= l; ++m) {
            const int64_t i = oracle_alm_index(lmax, l, m);
            const double p = alm_re[i] * alm_re[i] + alm_im[i] * alm_im[i];
            cadd(&acc, m == 0 ? p : 2.0 * p);
        }
        cl[l] = (acc.sum + acc.comp) / (2.0 * (double)l + 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* HEALPix RING pixel of a direction (the inverse of pix2vec), used to keep  */
/* the strings that live inside a healpix cone when simulations are stacked  */
/* (Sec. II.C: the comoving ball is cut into cones subtending the pixels of  */
/* a coarse healpix grid, and every box keeps only the strings of its cone).  */
/* The published construction (Gorski et al. 2005): with z = cos(theta) and  */
/* t = phi / (pi/2) in [0, 4),                                              */
/*   |z| <= 2/3: the pixel edges are the lines N (1/2 + t) -+ (3N/4) z =    */
/*               integer; with a, b the integer parts of those two values,   */
/*               the ring (counted from z = 2/3) is N + 1 + a - b and the    */
/*               position in it (a + b - N + shift + 1) / 2 mod 4N;         */
/*   |z| >  2/3: with s = N sqrt(3 (1 - |z|)) and f the fraction of t, the   */
/*               ring counted from the pole is floor(f s) + floor((1-f) s)   */
/*               + 1 and the position floor(t ring) mod 4 ring.             */
/* 1 - |z| is taken as (x^2 + y^2) / (r (r + |z_v|)) for a vector (x, y, z_v) */
/* of length r, which keeps its accuracy near the poles.                     */
/* The azimuth t comes from the fixed arctangent recipe below (IEEE          */
/* operations only), so that two implementations of it agree bit for bit.   */
/* ------------------------------------------------------------------------ */

/* atan(u) / (pi/2) for |u| <= tan(pi/8): the Maclaurin series of atan,
 *   atan(u) = u - u^3/3 + u^5/5 - ... ,
 * cut after u^45 (|u|^46/47 < 2e-19 |u| there), summed in u^2 by
 * fma-Horner from the highest term, with coefficients (-1)^k/(2k+1) as the
 * doubles nearest them, then scaled by 2/pi (the double nearest). */
static double atan_quarter(double u)
{
    static const double c[22] = {
        -1.0 / 3.0,  1.0 / 5.0,  -1.0 / 7.0,  1.0 / 9.0,  -1.0 / 11.0, 1.0 / 13.0,
        -1.0 / 15.0, 1.0 / 17.0, -1.0 / 19.0, 1.0 / 21.0, -1.0 / 23.0, 1.0 / 25.0,
        -1.0 / 27.0, 1.0 / 29.0, -1.0 / 31.0, 1.0 / 33.0, -1.0 / 35.0, 1.0 / 37.0,
        -1.0 / 39.0, 1.0 / 41.0, -1.0 / 43.0, 1.0 / 45.0};
    const double v = u * u;
    double p = c[21];
    for (int k = 20; k >= 0; --k) p = fma(p, v, c[k]);
    const double a = fma(u * v, p, u);
    return a * 0.63661977236758134308;
}

/* phi / (pi/2) in [0, 4) for the direction (x, y) of azimuth phi in
 * [0, 2 pi), (x, y) != (0, 0):
 *   1. the quadrant q from the signs, and (a, b) the direction turned by
 *      -q pi/2 into a >= 0, b >= 0 (exact swaps and negations);
 *   2. r = min(a, b) / max(a, b) in [0, 1] (one division);
 *   3. atan(r) / (pi/2): if r > tan(pi/8) (the double nearest), as
 *      1/2 + atan_quarter((r - 1) / (r + 1)), else atan_quarter(r);
 *   4. the angle from the a axis is that value when b <= a, else one minus
 *      it; t = q + angle, and t = 4 wraps to 0. */
double oracle_quarter_turns(double x, double y)
{
    int q;
    double a, b;
    if (y >= 0.0) {
        if (x > 0.0) { q = 0; a = x; b = y; }
        else { q = 1; a = y; b = -x; }
    } else {
        if (x < 0.0) { q = 2; a = -x; b = -y; }
        else { q = 3; a = -y; b = x; }
    }
    const int swap = b > a;
    const double r = swap ? a / b : b / a;
    double f;
    if (r > 0.41421356237309503) f = 0.5 + atan_quarter((r - 1.0) / (r + 1.0));
    else f = atan_quarter(r);
    const double ang = swap ? 1.0 - f : f;
    double t = (double)q + ang;
    if (t >= 4.0) t -= 4.0;
    return t;
}

void oracle_quarter_turns_many(int64_t n, const double *xy, double *t)
{
    for (int64_t i = 0; i < n; ++i) t[i] = oracle_quarter_turns(xy[2 * i], xy[2 * i + 1]);
}

int64_t oracle_ang2pix(int64_t nside, const double v[3])
{
    const int64_t N = nside;
    const double rho2 = v[0] * v[0] + v[1] * v[1];
    const double r = sqrt(rho2 + v[2] * v[2]);
    const double z = v[2] / r;
    const double t = oracle_quarter_turns(v[0], v[1]);
    const double az = fabs(z);
    if (az <= 2.0 / 3.0) {
        const double t1 = (double)N * (0.5 + t);
        const double t2 = (double)N * z * 0.75;
        const int64_t a = (int64_t)(t1 - t2);
        const int64_t b = (int64_t)(t1 + t2);
        const int64_t ring = N + 1 + a - b;                 /* 1 .. 2N+1 */
        const int64_t shift = 1 - (ring & 1);
        int64_t pos = (a + b - N + shift + 1) / 2;
        pos = ((pos % (4 * N)) + 4 * N) % (4 * N);
        return 2 * N * (N - 1) + (ring - 1) * 4 * N + pos;
    }
    const double f = t - floor(t);
    const double one_minus = rho2 / (r * (r + fabs(v[2])));
    const double s = (double)N * sqrt(3.0 * one_minus);
    const int64_t a = (int64_t)(f * s);
    const int64_t b = (int64_t)((1.0 - f) * s);
    int64_t ring = a + b + 1;                               /* from the pole */
    if (ring > N) ring = N;                                 /* |z| just above 2/3 */
    int64_t pos = (int64_t)(t * (double)ring);
    pos = ((pos % (4 * ring)) + 4 * ring) % (4 * ring);
    if (z > 0.0) return 2 * ring * (ring - 1) + pos;
    return 12 * N * N - 2 * ring * (ring + 1) + pos;
}

void oracle_ang2pix_many(int64_t nside, int64_t n, const double *v, int64_t *pix)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) pix[i] = oracle_ang2pix(nside, v + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Flat-sky, small-angle form of Eq. (1) (Sec. II.A: the limit X n -> X,    */
/* with every photon path parallel to a fixed axis c; Sec. III.B, Fig. 3:   */
/* the flat-sky maps the paper compares with a gnomonic projection of its   */
/* full-sky map).  For a patch around c with orthonormal axes e1, e2:       */
/*   a segment at P (depth D = c.P) is seen at the plane position            */
/*   s = (e1.P, e2.P) / D (gnomonic), and in u the line of sight n is        */
/*   replaced by c: u = Xdot - (c.X')/(1 + c.Xdot) X' ;                     */
/*   pixel (i, j) (index j nx + i) is at t = ((i + 1/2 - nx/2) h,            */
/*   (j + 1/2 - ny/2) h), and the term of the segment is                     */
/*   -4 eps dsigma (u_perp . (t - s)) / (D |t - s|^2),                        */
/*   u_perp = (e1.u, e2.u), the transverse separation D (t - s) standing for */
/*   X n - X.                                                               */
/* A segment enters when it is in its box's slab (as for Eq. (1)), in front */
/* of the observer (D > 0, where the gnomonic position exists) and          */
/* c.P > accept_cos |P|; a pixel at t = s exactly receives 0.               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double s[2];    /* plane position */
    double a[2];    /* -4 eps dsigma u_perp / D */
} flat_seg_t;

/* The segments that enter a flat patch, with their plane positions and
 * weights; returns their number (*out is malloc'ed, caller frees). */
static int64_t flat_segments(const double *frame, double accept_cos, double eta0, int64_t nbox,
                             const double *boxes, const int64_t *seg_off, const double *x_rel,
                             const double *xdot, const double *xprime, const double *dsigma,
                             flat_seg_t **out)
{
    const double *c = frame, *e1 = frame + 3, *e2 = frame + 6;
    const int64_t nseg = seg_off[nbox];
    flat_seg_t *fs = (flat_seg_t *)malloc(sizeof(flat_seg_t) * (size_t)(nseg > 0 ? nseg : 1));
    int64_t nf = 0;
    for (int64_t b = 0; b < nbox; ++b) {
        const double *box = boxes + BOX_STRIDE * b;
        for (int64_t i = seg_off[b]; i < seg_off[b + 1]; ++i) {
            seg_t sg;
            if (!load_segment(box, eta0, x_rel + 3 * i, xdot + 3 * i, xprime + 3 * i,
                              dsigma[i], &sg))
                continue;
            const double D = dot3(c, sg.P);
            if (!(D > 0.0) || !(D > accept_cos * sg.R)) continue;
            const double a = dot3(c, sg.T);
            const double bb = 1.0 + dot3(c, sg.V);
            double u[3];
            for (int k = 0; k < 3; ++k) u[k] = sg.V[k] - (a / bb) * sg.T[k];
            const double kap = -4.0 * sg.eps * sg.w / D;
            fs[nf].s[0] = dot3(e1, sg.P) / D;
            fs[nf].s[1] = dot3(e2, sg.P) / D;
            fs[nf].a[0] = kap * dot3(e1, u);
            fs[nf].a[1] = kap * dot3(e2, u);
            ++nf;
        }
    }
    *out = fs;
    return nf;
}

static double flat_sum(double tx, double ty, const flat_seg_t *fs, int64_t nf)
{
    csum_t acc = {0.0, 0.0};
    for (int64_t k = 0; k < nf; ++k) {
        const double dx = tx - fs[k].s[0];
        const double dy = ty - fs[k].s[1];
        const double q = dx * dx + dy * dy;
        if (q == 0.0) continue;
        cadd(&acc, (fs[k].a[0] * dx + fs[k].a[1] * dy) / q);
    }
    return acc.sum + acc.comp;
}

/* The flat map at npts plane positions t[2 k], t[2 k + 1] (radians). */
void oracle_flat_points(int64_t npts, const double *t, const double *frame, double accept_cos,
                        double eta0, int64_t nbox, const double *boxes, const int64_t *seg_off,
                        const double *x_rel, const double *xdot, const double *xprime,
                        const double *dsigma, double *out)
{
    flat_seg_t *fs;
    const int64_t nf = flat_segments(frame, accept_cos, eta0, nbox, boxes, seg_off, x_rel, xdot,
                                     xprime, dsigma, &fs);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npts; ++k) out[k] = flat_sum(t[2 * k], t[2 * k + 1], fs, nf);
    free(fs);
}

/* The flat map on the nx x ny grid of pixel size h. */
void oracle_flat_theta(int64_t nx, int64_t ny, double h, const double *frame,
                       double accept_cos, double eta0, int64_t nbox, const double *boxes,
                       const int64_t *seg_off, const double *x_rel, const double *xdot,
                       const double *xprime, const double *dsigma, double *out)
{
    flat_seg_t *fs;
    const int64_t nf = flat_segments(frame, accept_cos, eta0, nbox, boxes, seg_off, x_rel, xdot,
                                     xprime, dsigma, &fs);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < ny; ++j) {
        const double ty = ((double)j + 0.5 - 0.5 * (double)ny) * h;
        for (int64_t i = 0; i < nx; ++i) {
            const double tx = ((double)i + 0.5 - 0.5 * (double)nx) * h;
            out[j * nx + i] = flat_sum(tx, ty, fs, nf);
        }
    }
    free(fs);
}
