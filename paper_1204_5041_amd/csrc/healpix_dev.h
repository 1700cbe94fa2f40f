// healpix_dev.h -- HEALPix RING pixel centres on the device.
//
// The map directions of the paper (Sec. II.D) are the centres of an Nside
// HEALPix RING pixelisation (Gorski et al. 2005, cited in Sec. I).  This
// routine follows the published definition:
//   * rings i = 1 .. 4N-1 from north to south; north-cap ring i < N holds 4i
//     pixels, each of the 2N+1 belt rings N .. 3N holds 4N, the south cap
//     mirrors the north, pixels run by increasing azimuth inside a ring;
//   * cap ring k (counted from its pole): z = +-(1 - k^2/(3N^2)),
//     azimuth (pi/2)(j + 1/2)/k;
//   * belt ring i: z = (4N - 2i)/(3N), azimuth (pi/2)(j + h)/N with a half
//     pixel offset h = 1/2 on ring N and on every second ring after it.
//
// Only correctly rounded IEEE double operations on exact integers and a
// fixed fma polynomial are used, in a fixed order, and the file is compiled
// without floating-point contraction, so the result is reproducible bit for
// bit by any implementation of the same steps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csmap {

// floor(sqrt(v)) for 0 <= v < 2^62.
__device__ __forceinline__ int64_t dev_isqrt(int64_t v) {
  int64_t r = (int64_t)sqrt((double)v);
  r -= (r * r > v) ? 1 : 0;
  r += ((r + 1) * (r + 1) <= v) ? 1 : 0;
  return r;
}

// Maclaurin coefficients of sin(pi t/2)/t and cos(pi t/2) in powers of t^2:
// element k is the double nearest (-1)^k (pi/2)^(2k+1)/(2k+1)! and
// (-1)^k (pi/2)^(2k)/(2k)! respectively.
__device__ __forceinline__ void quarter_sincos(double t, double* s, double* c) {
  const double t2 = t * t;
  double ps = 6.0669357311061955e-12;
  ps = fma(ps, t2, -6.688035109811468e-10);
  ps = fma(ps, t2, 5.692172921967927e-08);
  ps = fma(ps, t2, -3.598843235212085e-06);
  ps = fma(ps, t2, 0.00016044118478735983);
  ps = fma(ps, t2, -0.004681754135318688);
  ps = fma(ps, t2, 0.07969262624616705);
  ps = fma(ps, t2, -0.6459640975062463);
  ps = fma(ps, t2, 1.5707963267948966);
  double pc = 6.565963114979473e-11;
  pc = fma(pc, t2, -6.386603083791852e-09);
  pc = fma(pc, t2, 4.710874778818172e-07);
  pc = fma(pc, t2, -2.5202042373060607e-05);
  pc = fma(pc, t2, 0.0009192602748394266);
  pc = fma(pc, t2, -0.02086348076335296);
  pc = fma(pc, t2, 0.25366950790104803);
  pc = fma(pc, t2, -1.2337005501361697);
  pc = fma(pc, t2, 1.0);
  *s = t * ps;
  *c = pc;
}

// Unit vector of RING pixel p of an Nside map.
__device__ __forceinline__ void pix2vec_ring(int64_t nside, int64_t p, double* vx, double* vy,
                                             double* vz) {
  const int64_t N = nside;
  const int64_t npix = 12 * N * N;
  const int64_t ncap = 2 * N * (N - 1);
  // Integer stage: ring number from the nearer pole (k), 0-based azimuth
  // index (j), and which zone the pixel is in.
  int64_t k, j;
  int zone;  // 0 north cap, 1 belt, 2 south cap
  if (p < ncap) {
    k = (1 + dev_isqrt(2 * p + 1)) >> 1;
    j = p - 2 * k * (k - 1);
    zone = 0;
  } else if (p >= npix - ncap) {
    const int64_t m = npix - 1 - p;
    k = (1 + dev_isqrt(2 * m + 1)) >> 1;
    j = 4 * k - 1 - (m - 2 * k * (k - 1));
    zone = 2;
  } else {
    const int64_t q = p - ncap;
    k = N + q / (4 * N);  // ring number counted from the north
    j = q - (k - N) * (4 * N);
    zone = 1;
  }
  double z, st;
  int64_t num, den;
  if (zone != 1) {
    const double d = (double)(3 * N * N);
    const int64_t kk = k * k;
    z = (double)(3 * N * N - kk) / d;
    st = ((double)k * sqrt((double)(6 * N * N - kk))) / d;
    if (zone == 2) z = -z;
    num = 2 * j + 1;
    den = 2 * k;
  } else {
    const int64_t m = 2 * N - k;
    const double d = (double)(3 * N);
    z = (double)(2 * m) / d;
    st = sqrt((double)(9 * N * N - 4 * m * m)) / d;
    num = 2 * j + (((k - N) & 1) == 0 ? 1 : 0);
    den = 2 * N;
  }
  // Azimuth (pi/2) num/den: integer quadrant, then fold into [0, pi/4].
  const int64_t quad = num / den;
  const int64_t r = num - quad * den;
  double s, c, cq, sq;
  if (2 * r <= den) {
    quarter_sincos((double)r / (double)den, &s, &c);
    cq = c;
    sq = s;
  } else {
    quarter_sincos((double)(den - r) / (double)den, &s, &c);
    cq = s;
    sq = c;
  }
  double cp, sp;
  switch (quad & 3) {
    case 0: cp = cq; sp = sq; break;
    case 1: cp = -sq; sp = cq; break;
    case 2: cp = -cq; sp = -sq; break;
    default: cp = sq; sp = -cq; break;
  }
  *vx = st * cp;
  *vy = st * sp;
  *vz = z;
}

// Azimuth of (x, y) in quarter turns, phi / (pi/2) in [0, 4), from IEEE
// operations only (so that any implementation of the same steps agrees bit
// for bit; the device atan2 is not correctly rounded):
//   * the quadrant q from the signs of x and y, and (a, b) the direction
//     turned back by q quarter turns, a >= 0, b >= 0 (swaps and negations);
//   * r = min(a, b) / max(a, b);
//   * atan(r) in quarter turns: 1/2 + A((r - 1)/(r + 1)) above tan(pi/8)
//     (the double nearest), else A(r), where A(u) is the Maclaurin series
//     of atan through u^45 (|u| <= tan(pi/8), so the first omitted term is
//     below 2e-19 |u|), fma-Horner in u^2 from the top, coefficients the
//     doubles nearest (-1)^k/(2k+1), times the double nearest 2/pi;
//   * the angle from the a axis is that value if b <= a, else 1 minus it;
//     t = q + angle, wrapped from 4 to 0.
// Within 2 ulp of the exact azimuth.
__device__ __forceinline__ double atan_quarter_turns(double u) {
  constexpr double kC[22] = {
      -1.0 / 3.0,  1.0 / 5.0,  -1.0 / 7.0,  1.0 / 9.0,  -1.0 / 11.0, 1.0 / 13.0,
      -1.0 / 15.0, 1.0 / 17.0, -1.0 / 19.0, 1.0 / 21.0, -1.0 / 23.0, 1.0 / 25.0,
      -1.0 / 27.0, 1.0 / 29.0, -1.0 / 31.0, 1.0 / 33.0, -1.0 / 35.0, 1.0 / 37.0,
      -1.0 / 39.0, 1.0 / 41.0, -1.0 / 43.0, 1.0 / 45.0};
  const double v = u * u;
  double p = kC[21];
#pragma unroll
  for (int k = 20; k >= 0; --k) p = fma(p, v, kC[k]);
  return fma(u * v, p, u) * 0.63661977236758134308;
}

__device__ __forceinline__ double quarter_turns(double x, double y) {
  int q;
  double a, b;
  if (y >= 0.0) {
    if (x > 0.0) {
      q = 0; a = x; b = y;
    } else {
      q = 1; a = y; b = -x;
    }
  } else {
    if (x < 0.0) {
      q = 2; a = -x; b = -y;
    } else {
      q = 3; a = -y; b = x;
    }
  }
  const bool swap = b > a;
  const double r = swap ? a / b : b / a;
  const double f = (r > 0.41421356237309503) ? 0.5 + atan_quarter_turns((r - 1.0) / (r + 1.0))
                                             : atan_quarter_turns(r);
  double t = (double)q + (swap ? 1.0 - f : f);
  if (t >= 4.0) t -= 4.0;
  return t;
}

// RING pixel of the direction of (x, y, z), a vector of any positive length:
// the inverse of pix2vec_ring (Gorski et al. 2005).  With c = cos(theta) and
// t = phi / (pi/2) in [0, 4) (quarter_turns):
//   * |c| <= 2/3: the pixel edges are the lines N (1/2 + t) - (3N/4) c = k and
//     N (1/2 + t) + (3N/4) c = k' for integers k, k'; the cell (k, k') is
//     belt ring N + 1 + k - k' (of the 2N + 1 belt rings, from the north),
//     position (k + k' - N + h + 1) / 2 mod 4N, with h = 1 on the belt rings
//     of even index;
//   * |c| > 2/3: with s = N sqrt(3 (1 - |c|)) and u the fractional part of t,
//     the edges are u s = k and (1 - u) s = k'; the cell is cap ring
//     k + k' + 1 from the nearer pole, position floor(t (k + k' + 1)).
// 1 - |c| is formed as (x^2 + y^2) / (r (r + |z|)), free of cancellation
// near the poles.  Used to decide which strings lie inside a healpix cone.
__device__ __forceinline__ int64_t ang2pix_ring(int64_t nside, double x, double y, double z) {
  const int64_t N = nside;
  const double rho2 = x * x + y * y;
  const double r = sqrt(rho2 + z * z);
  const double c = z / r;
  const double t = quarter_turns(x, y);
  const double ac = fabs(c);
  if (ac <= 2.0 / 3.0) {
    const double base = (double)N * (0.5 + t);
    const double tilt = (double)N * c * 0.75;
    const int64_t k1 = (int64_t)(base - tilt);  // ascending edge index
    const int64_t k2 = (int64_t)(base + tilt);  // descending edge index
    const int64_t bring = N + 1 + k1 - k2;      // 1 .. 2N + 1 among belt rings
    const int64_t h = 1 - (bring & 1);
    const int64_t L = 4 * N;
    int64_t pos = (k1 + k2 - N + h + 1) / 2;
    pos %= L;
    if (pos < 0) pos += L;
    return 2 * N * (N - 1) + (bring - 1) * L + pos;
  }
  const double u = t - floor(t);
  const double one_minus = rho2 / (r * (r + fabs(z)));
  const double sc = (double)N * sqrt(3.0 * one_minus);
  const int64_t k1 = (int64_t)(u * sc);
  const int64_t k2 = (int64_t)((1.0 - u) * sc);
  int64_t ring = k1 + k2 + 1;  // counted from the nearer pole
  if (ring > N) ring = N;      // rounding just above |c| = 2/3
  const int64_t L = 4 * ring;
  int64_t pos = (int64_t)(t * (double)ring);
  pos %= L;
  if (pos < 0) pos += L;
  return (z > 0.0) ? 2 * ring * (ring - 1) + pos : 12 * N * N - 2 * ring * (ring + 1) + pos;
}

}  // namespace csmap
