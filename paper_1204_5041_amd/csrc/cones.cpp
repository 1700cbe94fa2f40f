// cones.cpp -- placement of simulation boxes in healpix cones (Sec. II.C).
//
// The boundary of a HEALPix pixel in closed form.  In the belt the pixel
// edges are the lines U = N (1/2 + t) - (3N/4) z = integer and
// V = N (1/2 + t) + (3N/4) z = integer (t = phi / (pi/2)); a belt pixel is
// the cell a <= U <= a + 1, b <= V <= b + 1.  In a polar cap (z > 2/3),
// with s = N sqrt(3 (1 - z)) and f the fraction of t inside its quarter q,
// the edges are p = f s = integer and m = (1 - f) s = integer, and a cap
// pixel is the cell a <= p <= a + 1, b <= m <= b + 1.  At z = 2/3 the two
// descriptions join as U = q N + p and V = (q + 2) N - m, which lets the
// pixels of ring N (centred on z = 2/3) run from one into the other.  The
// south cap is the mirror image of the north.
#include "cones.h"

#include <math.h>

#include <algorithm>

namespace csmap {
namespace {

constexpr double kPi = 3.141592653589793;

int64_t isqrt_host(int64_t v) {
  int64_t r = (int64_t)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Ring (1 .. 4N-1 from the north) and position of RING pixel p.
void ring_pos(int64_t N, int64_t p, int64_t& ring, int64_t& pos) {
  const int64_t npix = 12 * N * N, ncap = 2 * N * (N - 1);
  if (p < ncap) {
    const int64_t k = (1 + isqrt_host(2 * p + 1)) >> 1;
    ring = k;
    pos = p - 2 * k * (k - 1);
  } else if (p >= npix - ncap) {
    const int64_t m = npix - 1 - p;
    const int64_t k = (1 + isqrt_host(2 * m + 1)) >> 1;
    ring = 4 * N - k;
    pos = 4 * k - 1 - (m - 2 * k * (k - 1));
  } else {
    ring = N + (p - ncap) / (4 * N);
    pos = (p - ncap) % (4 * N);
  }
}

// A pixel in the cell coordinates of its description.
struct Cell {
  int64_t N;
  bool cap;     // polar-cap pixel (coordinates p, m)
  bool south;   // mirrored from the north
  int64_t q;    // quarter of the pixel centre
  double a, b;  // lower corner of the cell
};

Cell cell_of(int64_t N, int64_t pix) {
  int64_t ring, pos;
  ring_pos(N, pix, ring, pos);
  Cell c;
  c.N = N;
  c.south = ring > 2 * N;
  const int64_t i = c.south ? 4 * N - ring : ring;  // mirrored ring has the same position
  if (i < N) {
    c.cap = true;
    c.q = pos / i;
    const int64_t jj = pos - c.q * i;
    c.a = (double)jj;
    c.b = (double)(i - 1 - jj);
  } else {
    c.cap = false;
    const int64_t h = (i - N + 1) & 1;
    c.a = (double)(pos + (i - N + h - 1) / 2);
    c.b = (double)(pos + (3 * N + h - i - 1) / 2);
    const double tc = (c.a + c.b + 1.0) / (2.0 * (double)N) - 0.5;
    c.q = (int64_t)floor(tc);
  }
  return c;
}

// Unit vector at cap coordinates (p, m) of quarter q (north).
void cap_dir(double N, int64_t q, double p, double m, double d[3]) {
  const double s = p + m;
  if (s <= 0.0) {
    d[0] = 0.0;
    d[1] = 0.0;
    d[2] = 1.0;
    return;
  }
  const double w = s * s / (3.0 * N * N);  // 1 - z
  const double z = 1.0 - w;
  const double st = sqrt(w * (2.0 - w));
  const double phi = 0.5 * kPi * ((double)q + p / s);
  d[0] = st * cos(phi);
  d[1] = st * sin(phi);
  d[2] = z;
}

// Unit vector at cell coordinates (x, y) of cell c (x along a, y along b).
void cell_dir(const Cell& c, double x, double y, double d[3]) {
  const double N = (double)c.N;
  if (c.cap) {
    cap_dir(N, c.q, x, y, d);
  } else {
    const double z = 2.0 * (y - x) / (3.0 * N);
    if (z <= 2.0 / 3.0) {
      const double phi = 0.5 * kPi * ((x + y) / (2.0 * N) - 0.5);
      const double st = sqrt((1.0 - z) * (1.0 + z));
      d[0] = st * cos(phi);
      d[1] = st * sin(phi);
      d[2] = z;
    } else {
      cap_dir(N, c.q, x - (double)c.q * N, (double)(c.q + 2) * N - y, d);
    }
  }
  if (c.south) d[2] = -d[2];
}

double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

constexpr int kEdgeSamples = 256;  // intervals per edge

// Point k (0 .. kEdgeSamples) of edge e (0 .. 3) of cell c.
void edge_point(const Cell& c, int e, int k, double d[3]) {
  const double tau = (double)k / kEdgeSamples;
  double x, y;
  switch (e) {
    case 0: x = c.a; y = c.b + tau; break;
    case 1: x = c.a + 1.0; y = c.b + tau; break;
    case 2: x = c.a + tau; y = c.b; break;
    default: x = c.a + tau; y = c.b + 1.0; break;
  }
  cell_dir(c, x, y, d);
}

}  // namespace

void cone_place(int64_t nside, int64_t pix, int axis, double r_in, double r_out, double side,
                ConePlacement& out) {
  const Cell c = cell_of(nside, pix);
  double n[3];
  cell_dir(c, c.a + 0.5, c.b + 0.5, n);
  const double st = hypot(n[0], n[1]);
  const double cp = n[0] / st, sp = n[1] / st;
  const double eth[3] = {n[2] * cp, n[2] * sp, -st};
  const double eph[3] = {-sp, cp, 0.0};
  const double h = sqrt(0.5);
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = h * (eth[k] + eph[k]);
    e2[k] = h * (eph[k] - eth[k]);
  }
  const double* col[3];
  col[axis] = n;
  col[(axis + 1) % 3] = e1;
  col[(axis + 2) % 3] = e2;
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) out.rot[3 * r + k] = col[k][r];
  for (int k = 0; k < 3; ++k)
    out.origin[k] = (r_out - side) * n[k] - 0.5 * side * (e1[k] + e2[k]);
  // Extremes of e1.d, e2.d and n.d over the pixel lie on its boundary (the
  // only stationary points of a linear function on the sphere are +-its
  // axis, which the pixel does not contain).
  double lat = 0.0, ncos = 1.0;
  for (int edge = 0; edge < 4; ++edge)
    for (int k = 0; k <= kEdgeSamples; ++k) {
      double d[3];
      edge_point(c, edge, k, d);
      lat = std::max(lat, std::max(fabs(dot3(e1, d)), fabs(dot3(e2, d))));
      ncos = std::min(ncos, dot3(n, d));
    }
  out.slack = std::min(0.5 * side - r_out * lat, r_in * ncos - (r_out - side));
}

void cone_caps(int64_t nside, int64_t pix, double dir[3], double& cos_out, double& cos_in) {
  const Cell c = cell_of(nside, pix);
  double n[3];
  cell_dir(c, c.a + 0.5, c.b + 0.5, n);
  double lo = 1.0, hi = -1.0;
  for (int edge = 0; edge < 4; ++edge)
    for (int k = 0; k <= kEdgeSamples; ++k) {
      double d[3];
      edge_point(c, edge, k, d);
      const double cd = dot3(n, d);
      lo = std::min(lo, cd);
      hi = std::max(hi, cd);
    }
  const double a_out = acos(std::max(-1.0, std::min(1.0, lo)));
  const double a_in = acos(std::max(-1.0, std::min(1.0, hi)));
  for (int k = 0; k < 3; ++k) dir[k] = n[k];
  cos_out = cos(std::min(kPi, 1.02 * a_out + 1e-7));
  const double inner = 0.98 * a_in - 1e-7;
  cos_in = inner > 0.0 ? cos(inner) : 2.0;
}

void cone_edges(int64_t nside, int64_t pix, ConeEdges& out) {
  const Cell c = cell_of(nside, pix);
  double ctr[3];
  cell_dir(c, c.a + 0.5, c.b + 0.5, ctr);
  double pts[4][kEdgeSamples + 1][3];
  double lo_cap = 1.0;
  for (int e = 0; e < 4; ++e)
    for (int k = 0; k <= kEdgeSamples; ++k) {
      edge_point(c, e, k, pts[e][k]);
      lo_cap = std::min(lo_cap, dot3(ctr, pts[e][k]));
    }
  const double a_out = 1.02 * acos(std::max(-1.0, std::min(1.0, lo_cap))) + 1e-7;
  const double margin = 1e-7 + (4.0 * a_out / kEdgeSamples) * (4.0 * a_out / kEdgeSamples);
  bool ok = a_out < 0.5 * kPi;
  for (int e = 0; e < 4; ++e) {
    const double* p0 = pts[e][0];
    const double* p1 = pts[e][kEdgeSamples];
    double n[3] = {p0[1] * p1[2] - p0[2] * p1[1], p0[2] * p1[0] - p0[0] * p1[2],
                   p0[0] * p1[1] - p0[1] * p1[0]};
    const double len = sqrt(dot3(n, n));
    if (!(len > 0.0)) {
      ok = false;
      n[0] = 1.0;
      n[1] = n[2] = 0.0;
    } else {
      const double sgn = dot3(n, ctr) < 0.0 ? -1.0 : 1.0;
      for (int k = 0; k < 3; ++k) n[k] *= sgn / len;
    }
    double hi = -INFINITY, lo = INFINITY;
    for (int k = 0; k <= kEdgeSamples; ++k) hi = std::max(hi, dot3(n, pts[e][k]));
    for (int f = 0; f < 4; ++f)
      for (int k = 0; k <= kEdgeSamples; ++k) lo = std::min(lo, dot3(n, pts[f][k]));
    for (int k = 0; k < 3; ++k) out.n[e][k] = n[k];
    out.hi[e] = hi + margin;
    out.lo[e] = lo - margin;
    ok = ok && dot3(n, ctr) > out.hi[e];
  }
  if (!ok)
    for (int e = 0; e < 4; ++e) {
      out.hi[e] = INFINITY;
      out.lo[e] = -INFINITY;
    }
}

double cone_grid_slack(int64_t nside, double r_in, double r_out, double side) {
  // Cones congruent under quarter turns, the north-south mirror and (in the
  // belt) turns by one pixel share their slack: visit one of each.
  const int64_t N = nside;
  double worst = INFINITY;
  ConePlacement pl;
  for (int64_t i = 1; i <= 2 * N; ++i) {
    const int64_t first = i < N ? 2 * i * (i - 1) : 2 * N * (N - 1) + (i - N) * 4 * N;
    const int64_t count = i < N ? i : (i == N ? N : 1);
    for (int64_t j = 0; j < count; ++j) {
      cone_place(N, first + j, 2, r_in, r_out, side, pl);
      worst = std::min(worst, pl.slack);
    }
  }
  return worst;
}

}  // namespace csmap
