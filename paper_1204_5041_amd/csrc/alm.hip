// alm.hip -- spherical-harmonic analysis of a RING map on the device.
//
// a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(n_p)) for 0 <= m <= l <= lmax,
// Y_lm = lambda_lm(cos theta) e^{i m phi} (orthonormal, Condon-Shortley
// phase), and C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1): the angular
// power spectrum of a map (Sec. III, Fig. 4).  The pixels of a HEALPix ring
// share z and are evenly spaced in azimuth, so the sum splits into
//   1. a Fourier sum along every ring, F_m(r) = sum_j map_{r,j} e^{-i m phi_j};
//   2. a Legendre sum over rings, a_lm = (4 pi/Npix) sum_r lambda_lm(z_r) F_m(r),
// where rings r and 4N - r (z and -z) enter together through
// lambda_lm(-z) = (-1)^(l+m) lambda_lm(z).
//
// lambda_lm follows the recursions
//   lambda_00 = 1/sqrt(4 pi),  lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},
//   lambda_{m+1,m} = sqrt(2m+3) z lambda_mm,
//   lambda_lm = A_lm (z lambda_{l-1,m} - B_lm lambda_{l-2,m}),
//   A_lm = sqrt((4l^2-1)/(l^2-m^2)),  B_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
// with values carried as v * 2^(600 e): sin^m(theta) leaves the double range
// for large m near the poles long before the l recursion brings it back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "healpix_dev.h"

namespace csmap {

namespace {

constexpr int kLegScale = 600;   // values are v * 2^(600 e)
// Ring pairs summed by one lane of the Legendre kernel.  The wavefront
// reduction of each group of eight degrees is spread over more pairs as this
// grows, at the cost of registers.  With the Fourier-factor reload kept out
// of the loop's live registers, 8 pairs take 162 VGPRs (three wavefronts per
// SIMD); at Nside 2048, lmax 4096 the kernel took 7.7 ms with 6 pairs and
// 6.4-6.7 ms with 8 (7 pairs: 140 VGPRs, slower than 8).
constexpr int kRingsPerLane = 8;
constexpr int kAnchor = 32;      // Fourier twiddles are recomputed exactly every 32 pixels

typedef const double __attribute__((address_space(4)))* cdp;

struct Ring {
  int64_t first;   // RING index of the ring's first pixel
  int64_t len;     // pixels in the ring
  int32_t half;    // 1 if the azimuths carry the half-pixel offset
};

// Ring i (1 .. 4N-1) of the RING scheme.
__device__ __forceinline__ Ring ring_of(int64_t N, int64_t i) {
  Ring r;
  if (i < N) {
    r.len = 4 * i;
    r.first = 2 * i * (i - 1);
    r.half = 1;
  } else if (i <= 3 * N) {
    r.len = 4 * N;
    r.first = 2 * N * (N - 1) + (i - N) * 4 * N;
    r.half = ((i - N) % 2 == 0) ? 1 : 0;
  } else {
    const int64_t k = 4 * N - i;
    r.len = 4 * k;
    r.first = 12 * N * N - 2 * k * (k + 1);
    r.half = 1;
  }
  return r;
}

__device__ __forceinline__ int64_t alm_idx(int64_t lmax, int64_t l, int64_t m) {
  return m * (2 * lmax + 1 - m) / 2 + l;
}

// e^{-i pi t / L} for an integer t in [0, 2L).
__device__ __forceinline__ void twiddle(int64_t t, int64_t L, double& c, double& s) {
  double sp, cp;
  sincospi((double)t / (double)L, &sp, &cp);
  c = cp;
  s = -sp;
}

// Step 1: F[(i-1) M + m] = sum_j map_{i,j} e^{-i m phi_j}, M = mmax + 1.
// One wavefront per (ring, 64 consecutive m); the ring's pixel values are
// uniform across the wavefront and stream through scalar registers.  Ring
// lengths are multiples of 4, and pixels j, j + L/4, j + L/2, j + 3L/4 see
// the twiddle of pixel j times (-i)^m, (-1)^m, i^m: the four values are
// folded first (x0 + x2, x1 + x3, x0 - x2, x3 - x1 combine into the real and
// imaginary parts for m mod 4), so one complex twiddle serves four pixels.
// Each lane advances e^{-i m 2 pi j / L} by one complex multiplication per
// step and recomputes it exactly every kAnchor steps.
// Only rings ring_lo .. ring_hi; the others are left to the FFT kernels.
__global__ void __launch_bounds__(256) k_ring_dft(int64_t nside, int64_t mmax, const double* map,
                                                 double* F, int64_t ring_lo, int64_t ring_hi) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t mblocks = (mmax + 64) / 64;
  if (wave >= (ring_hi - ring_lo + 1) * mblocks) return;
  const int64_t i = ring_lo + wave / mblocks;
  const int64_t m = (wave % mblocks) * 64 + lane;
  const Ring r = ring_of(nside, i);
  const int64_t L = r.len;
  const int64_t Q = L / 4;
  const int64_t mm = m % L;                 // e^{-i m 2pi j/L} depends on m mod L only
  double oc, os;                            // e^{-i 2 pi m / L}
  twiddle((2 * mm) % (2 * L), L, oc, os);
  // The folded value of a quadruple for this lane's m mod 4:
  //   re = ca (x0 + x2) + cb (x1 + x3) + cc (x0 - x2),  im = cd (x3 - x1).
  const int q4 = (int)(m & 3);
  const double ca = (q4 & 1) ? 0.0 : 1.0;
  const double cb = (q4 == 0) ? 1.0 : (q4 == 2 ? -1.0 : 0.0);
  const double cc = (q4 & 1) ? 1.0 : 0.0;
  const double cd = (q4 == 1) ? 1.0 : (q4 == 3 ? -1.0 : 0.0);
  double acc_re = 0.0, acc_im = 0.0;
  cdp px = (cdp)(map + r.first);
  for (int64_t j0 = 0; j0 < Q; j0 += kAnchor) {
    double wc, ws;
    twiddle((2 * mm * j0) % (2 * L), L, wc, ws);
    const int64_t je = (j0 + kAnchor < Q) ? j0 + kAnchor : Q;
    for (int64_t j = j0; j < je; ++j) {
      const double x0 = px[j], x1 = px[j + Q], x2 = px[j + 2 * Q], x3 = px[j + 3 * Q];
      const double s02 = x0 + x2, s13 = x1 + x3, d02 = x0 - x2, d31 = x3 - x1;
      const double fr = fma(ca, s02, fma(cb, s13, cc * d02));
      const double fi = cd * d31;
      acc_re = fma(fr, wc, fma(-fi, ws, acc_re));
      acc_im = fma(fr, ws, fma(fi, wc, acc_im));
      const double nc = fma(wc, oc, -(ws * os));
      const double ns = fma(wc, os, ws * oc);
      wc = nc;
      ws = ns;
    }
  }
  // The half-pixel azimuth offset: phi_j = 2 pi (j + 1/2) / L, a factor
  // e^{-i pi m / L} (period 2L in m).
  if (r.half) {
    double hc, hs;
    twiddle(m % (2 * L), L, hc, hs);
    const double re = fma(acc_re, hc, -(acc_im * hs));
    const double im = fma(acc_re, hs, acc_im * hc);
    acc_re = re;
    acc_im = im;
  }
  if (m <= mmax) {
    double* o = F + 2 * ((i - 1) * (mmax + 1) + m);
    o[0] = acc_re;
    o[1] = acc_im;
  }
}

struct cplx {
  double r, i;
};

// The ring transforms of step 1 share one FFT over P = 2^e <= kFftMaxP
// complex points in LDS, taken by a workgroup of kFftThreads threads in
// radix-8 passes (one radix-2 or radix-4 pass when e is not a multiple of
// 3), each thread taking one butterfly in registers per pass: forward by
// decimation in frequency (natural order in, digit-reversed order out),
// inverse by decimation in time with the passes reversed (digit-reversed
// order in, natural order out), so no reordering pass is needed.  With
// kSwz, point j lives at complex slot j ^ ((j >> 3) & 15): bits 3-6 of the
// index are folded into bits 0-3, so that in every radix-8 pass the lanes
// of an aligned group of 8 or 16 read and write 16-byte slots in distinct
// LDS banks (stored in order, the lanes of the passes whose butterflies
// take points 1, 2, 4 or 8 apart meet in the same banks: lane b reads
// point 8b + q in the last forward pass, 128 bytes from its neighbours).
// Only a final radix-2 or radix-4 pass keeps a two-way conflict within 16
// lanes.  The fold leaves bits 4 and above alone, so a slot stays below P.
// It costs an address computation per access, which pays where LDS bounds
// the kernel (the belt rings) and not where latency does (the cap rings,
// whose nine transforms per workgroup run at the same speed either way).
// ftab[k] = e^{-2 pi i k/kFftMaxP}, k < kFftMaxP/4, a quarter of the
// period: a workgroup copies it into LDS and forms every twiddle from it,
// e^{-2 pi i (q kFftMaxP/4 + r)/kFftMaxP} = (-i)^q e^{-2 pi i r/kFftMaxP}
// (a swap and sign changes, exact).  Read from global memory, the seven
// twiddles of each butterfly waited on the L2 in every pass: the two ring
// kernels took 30% and 20% longer than with constant twiddles.
constexpr int kFftThreads = 512;
constexpr int64_t kFftMaxP = 4096;   // 64 KB of LDS, and 16 KB for the twiddles
constexpr int kTwQ = (int)(kFftMaxP / 4);

// LDS bytes of a workgroup transforming P points: the quarter twiddle
// table, then the points (gfx950 gives a workgroup up to 160 KB, so two of
// the largest share a CU).
constexpr size_t fft_lds_bytes(int64_t P) { return 16 * (size_t)(kTwQ + P); }

// Slot of quarter-table entry r (< 1024) in LDS: bits 4-9 folded into bits
// 0-3.  A pass of span S reads entries pos q (4096/S) apart across its
// lanes; stored in order, those of spans 512 and 64 meet in one or two
// banks (8- to 16-way conflicts), folded they spread over most of them
// (1.5-way on average over all passes in a CPU model of the accesses).
__device__ __forceinline__ int tw_slot(int r) { return r ^ ((r >> 4) & 15) ^ (r >> 8); }

// Copies the quarter table into LDS (tl); the caller synchronises.
__device__ __forceinline__ void fft_load_twiddles(double* tl, const double* ftab) {
  for (int k = threadIdx.x; k < kTwQ; k += kFftThreads)
    reinterpret_cast<double2*>(tl)[tw_slot(k)] = reinterpret_cast<const double2*>(ftab)[k];
}

// e^{-2 pi i k/kFftMaxP}, 0 <= k < kFftMaxP, from the quarter table.
__device__ __forceinline__ cplx fft_twiddle(const double* tl, int k) {
  const int q = k >> 10, r = k & (kTwQ - 1);
  static_assert(kTwQ == 1024, "quarter index");
  const double2 u = reinterpret_cast<const double2*>(tl)[tw_slot(r)];
  // (-i)^q (x + i y): q = 1 gives (y, -x), q = 2 (-x, -y), q = 3 (-y, x).
  double x = (q & 1) ? u.y : u.x, y = (q & 1) ? u.x : u.y;
  if (q & 2) x = -x;
  if ((q ^ (q >> 1)) & 1) y = -y;
  return {x, y};
}

template <bool kSwz>
__device__ __forceinline__ int fft_slot(int j) { return kSwz ? j ^ ((j >> 3) & 15) : j; }

// Point j of the transform in LDS, read and written as one 16-byte access.
template <bool kSwz>
__device__ __forceinline__ cplx fft_get(const double* x, int j) {
  const double2 u = reinterpret_cast<const double2*>(x)[fft_slot<kSwz>(j)];
  return {u.x, u.y};
}
template <bool kSwz>
__device__ __forceinline__ void fft_put(double* x, int j, cplx v) {
  reinterpret_cast<double2*>(x)[fft_slot<kSwz>(j)] = make_double2(v.r, v.i);
}

__device__ void fft_twiddles_block(double* ftab, int64_t blk) {
  const int64_t k = blk * 256 + threadIdx.x;
  if (k >= kTwQ) return;
  double sp, cp;
  sincospi((double)(2 * k) / (double)kFftMaxP, &sp, &cp);
  ftab[2 * k] = cp;
  ftab[2 * k + 1] = -sp;
}

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx w) {
  return {fma(a.r, w.r, -(a.i * w.i)), fma(a.r, w.i, a.i * w.r)};
}
// a * (-i) for the forward direction (kInv false), a * i for the inverse.
template <bool kInv>
__device__ __forceinline__ cplx rot90(cplx a) {
  return kInv ? cplx{-a.i, a.r} : cplx{a.i, -a.r};
}

// In-register DFT of R = 2, 4 or 8 points, natural order in and out:
// y_q' = sum_q x_q e^{-+2 pi i q q'/R} (minus sign forward, plus inverse).
template <int R, bool kInv>
__device__ __forceinline__ void dft_small(cplx* x) {
  if constexpr (R == 2) {
    const cplx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cplx s0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
    const cplx s1 = cadd(x[1], x[3]), d1 = rot90<kInv>(csub(x[1], x[3]));
    x[0] = cadd(s0, s1);
    x[2] = csub(s0, s1);
    x[1] = cadd(d0, d1);
    x[3] = csub(d0, d1);
  } else {
    // Split by halves: a_k = x_k + x_{k+4} feeds the even outputs,
    // b_k = (x_k - x_{k+4}) e^{-+2 pi i k/8} the odd ones.
    constexpr double h = 0.70710678118654752440;   // 1/sqrt(2), rounded
    cplx a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = cadd(x[k], x[k + 4]);
      b[k] = csub(x[k], x[k + 4]);
    }
    // e^{-+i pi/4} = (1 -+ i)/sqrt(2), e^{-+i pi/2} = -+i, e^{-+3 i pi/4} = (-1 -+ i)/sqrt(2).
    b[1] = kInv ? cplx{(b[1].r - b[1].i) * h, (b[1].r + b[1].i) * h}
                : cplx{(b[1].r + b[1].i) * h, (b[1].i - b[1].r) * h};
    b[2] = rot90<kInv>(b[2]);
    b[3] = kInv ? cplx{-(b[3].r + b[3].i) * h, (b[3].r - b[3].i) * h}
                : cplx{(b[3].i - b[3].r) * h, -(b[3].r + b[3].i) * h};
    dft_small<4, kInv>(a);
    dft_small<4, kInv>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[2 * k] = a[k];
      x[2 * k + 1] = b[k];
    }
  }
}

// One decimation-in-frequency pass of radix R over spans of S points (in
// place in LDS, P points): for every span and position p < h = S/R,
// y_q' = e^{-2 pi i p q'/S} sum_q x_{p + q h} e^{-2 pi i q q'/R}, written at
// p + q' h.  The inverse pass undoes it up to a factor R: twiddles
// conjugated and applied first, then the inverse R-point DFT.
template <int R, bool kInv, bool kSwz>
__device__ __forceinline__ void fft_pass(double* x, int P, int S, const double* tl) {
  const int h = S / R;
  const int tw = (int)kFftMaxP / S;   // table step of e^{-2 pi i/S}
  for (int b = threadIdx.x; b < P / R; b += kFftThreads) {
    const int pos = b & (h - 1);
    const int base = (b - pos) * R + pos;
    cplx v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = fft_get<kSwz>(x, base + q * h);
    if constexpr (!kInv) dft_small<R, false>(v);
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const cplx t = fft_twiddle(tl, (pos * q * tw) & ((int)kFftMaxP - 1));
      const cplx w = {t.r, kInv ? -t.i : t.i};
      v[q] = cmul(v[q], w);
    }
    if constexpr (kInv) dft_small<R, true>(v);
#pragma unroll
    for (int q = 0; q < R; ++q) fft_put<kSwz>(x, base + q * h, v[q]);
  }
  __syncthreads();
}

// Forward transform of P (a power of two <= kFftMaxP) values in LDS,
// natural order in, digit-reversed order out: radix-8 passes from the
// widest span down, then one radix-4 or radix-2 pass if log2 P mod 3 is 2
// or 1.
template <bool kSwz>
__device__ void fft_dif(double* x, int P, const double* tl) {
  int S = P;
  while (S >= 8) {
    fft_pass<8, false, kSwz>(x, P, S, tl);
    S >>= 3;
  }
  if (S == 4) fft_pass<4, false, kSwz>(x, P, 4, tl);
  if (S == 2) fft_pass<2, false, kSwz>(x, P, 2, tl);
}

// Inverse of fft_dif times P: digit-reversed order in, natural order out,
// the passes in reverse order.
template <bool kSwz>
__device__ void fft_dit_inv(double* x, int P, const double* tl) {
  int e = 0;
  while ((1 << e) < P) ++e;
  int S = 1 << (e % 3);
  if (S == 4) fft_pass<4, true, kSwz>(x, P, 4, tl);
  if (S == 2) fft_pass<2, true, kSwz>(x, P, 2, tl);
  while (S < P) {
    S <<= 3;
    fft_pass<8, true, kSwz>(x, P, S, tl);
  }
}

// Position of frequency k in fft_dif's output over 2^e points.  The pass of
// span S and radix R sends the points whose frequencies are q' mod R to the
// block at q' S/R, so the base-8 digits of k, least significant first,
// become the digits of the position from the most significant down, and
// the digit of a final radix-2 or radix-4 pass (k's top e mod 3 bits) ends
// up lowest.
__device__ __forceinline__ int dif_pos(int k, int e) {
  int p = 0;
  for (; e >= 3; e -= 3, k >>= 3) p |= (k & 7) << (e - 3);
  return p | k;
}

// Step 1 for the 2N + 1 belt rings when Nside is a power of two: every belt
// ring has L = 4N pixels, so its Fourier sums are one length-L DFT of real
// data.  It is taken as a complex FFT of half length H = L/2 on
// z_n = x_{2n} + i x_{2n+1} (natural order in, digit-reversed out), then
// unpacked: with E_k = (Z_k + conj Z_{H-k})/2 and O_k = (Z_k - conj
// Z_{H-k})/(2i), X_k = E_k + e^{-2 pi i k/L} O_k for 0 <= k <= H and
// X_k = conj X_{L-k} above.  F_m = X_{m mod L}, times e^{-i pi m/L} on
// rings with the half-pixel offset.  tab[k] = e^{-i pi k/L}, k = 0 .. L.
// One workgroup per ring.
constexpr int64_t kBeltMaxH = kFftMaxP;   // H <= 4096: Nside <= 2048

__device__ void fft_table_block(int64_t L, double* tab, int64_t blk) {
  const int64_t k = blk * 256 + threadIdx.x;
  if (k > L) return;
  double sp, cp;
  sincospi((double)k / (double)L, &sp, &cp);
  tab[2 * k] = cp;
  tab[2 * k + 1] = -sp;
}

__global__ void __launch_bounds__(kFftThreads) k_ring_fft(int64_t nside, int64_t mmax,
                                                          const double* map, const double* tab,
                                                          const double* ftab, double* F) {
  extern __shared__ double sm[];   // quarter twiddle table, then H points
  double* tl = sm;
  double* zs = sm + 2 * kTwQ;      // H complex values at fft_slot<true> positions
  fft_load_twiddles(tl, ftab);
  const int64_t i = nside + blockIdx.x;
  const Ring r = ring_of(nside, i);
  const int L = (int)r.len, H = L / 2;
  const int e = __builtin_ctz((unsigned)H);
  const double* x = map + r.first;
  for (int n = threadIdx.x; n < H; n += kFftThreads) fft_put<true>(zs, n, {x[2 * n], x[2 * n + 1]});
  __syncthreads();
  fft_dif<true>(zs, H, tl);
  double* out = F + 2 * (i - 1) * (mmax + 1);
  for (int m = threadIdx.x; m <= (int)mmax; m += kFftThreads) {
    int k = (int)((unsigned)m % (unsigned)L);
    const bool upper = k > H;
    if (upper) k = L - k;
    const int ka = (k == H) ? 0 : k, kb = (k == 0) ? 0 : H - k;
    const cplx za = fft_get<true>(zs, dif_pos(ka, e)), zb = fft_get<true>(zs, dif_pos(kb, e));
    const double zr = za.r, zi = za.i;
    const double cr = zb.r, ci = -zb.i;                         // conj Z_{H-k}
    const double er = 0.5 * (zr + cr), ei = 0.5 * (zi + ci);
    const double orr = 0.5 * (zi - ci), oi = -0.5 * (zr - cr);  // (Z - conj)/(2i)
    const double wc = tab[4 * k], ws = tab[4 * k + 1];          // e^{-2 pi i k/L}
    double xr = er + fma(wc, orr, -(ws * oi));
    double xi = ei + fma(wc, oi, ws * orr);
    if (upper) xi = -xi;
    if (r.half) {
      const double hc = tab[2 * m], hs = tab[2 * m + 1];        // e^{-i pi m/L}
      const double yr = fma(xr, hc, -(xi * hs)), yi = fma(xr, hs, xi * hc);
      xr = yr;
      xi = yi;
    }
    out[2 * m] = xr;
    out[2 * m + 1] = xi;
  }
}

// Step 1 for the polar-cap rings (Nside <= 2048).  North ring i and south
// ring 4N - i both have L = 4i pixels at azimuths 2 pi (j + 1/2)/L; they are
// taken together as z_j = x^N_j + i x^S_j, whose DFT Z gives both:
// X^N_k = (Z_k + conj Z_{L-k})/2, X^S_k = (Z_k - conj Z_{L-k})/(2i), and
// F_m = e^{-i pi m/L} X_{m mod L}.  L = 4i is split by four (j = 4n + r):
// Z_{kappa + s i} = sum_r (-i)^{rs} e^{-2 pi i r kappa/L} D_r(kappa), D_r the
// length-i DFT of z_{4n+r}.  i is arbitrary, so each D_r is taken by
// Bluestein's chirp transform: with w_n = e^{-i pi n^2/i} (from n^2 mod 2i,
// exact), D(kappa) = w_kappa sum_n (y_n w_n) conj(w_{kappa-n}), a linear
// convolution computed as a cyclic one of power-of-two length P >= 2i - 1
// by the shared FFT: the product with the chirp filter's transform is taken
// in the forward transform's digit-reversed order, which the inverse reads.
// The filter's transform stays in registers over the four D_r, and D_r
// stays in registers until the radix-4 step; Z goes through a global slot
// of 4i values before the unpacking, which pairs k with L - k.  One
// workgroup per ring pair.
constexpr int kCapPer = (int)(kFftMaxP / kFftThreads);  // transform positions per thread
constexpr int kCapKappa = kCapPer / 2;                  // D_r values per thread (i <= kFftMaxP / 2)

__device__ __forceinline__ int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// w_n = e^{-i pi n^2 / len}.
__device__ __forceinline__ void chirp(int64_t n, int64_t len, double& c, double& s) {
  double sp, cp;
  sincospi((double)((n * n) % (2 * len)) / (double)len, &sp, &cp);
  c = cp;
  s = -sp;
}

__global__ void __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_cap_bluestein(int64_t nside, int64_t mmax, const double* map, const double* ftab,
                double* zslot, double* F) {
  extern __shared__ double sm[];   // quarter twiddle table, then P points
  double* tl = sm;
  double* xs = sm + 2 * kTwQ;      // P complex values, in order
  fft_load_twiddles(tl, ftab);
  const int t = threadIdx.x;
  const int64_t N = nside, i = 1 + blockIdx.x, L = 4 * i;
  const int P = (int)pow2_at_least(2 * i - 1);
  const double inv_p = 1.0 / (double)P;   // exact: P is a power of two
  const double* xn = map + 2 * i * (i - 1);
  const double* xsth = map + 12 * N * N - 2 * i * (i + 1);
  // Chirp filter b_m = conj(w_m) at m mod P for |m| < i, then its transform.
  for (int p = t; p < P; p += kFftThreads) {
    const int64_t n = p < i ? p : (p > P - i ? P - p : -1);
    double br = 0.0, bi = 0.0;
    if (n >= 0) {
      double c, s;
      chirp(n, i, c, s);
      br = c;
      bi = -s;
    }
    fft_put<false>(xs, p, {br, bi});
  }
  __syncthreads();
  fft_dif<false>(xs, P, tl);
  double Br[kCapPer], Bi[kCapPer];
#pragma unroll
  for (int j = 0; j < kCapPer; ++j) {
    const int p = t + j * kFftThreads;
    const cplx b = p < P ? fft_get<false>(xs, p) : cplx{0.0, 0.0};
    Br[j] = b.r;
    Bi[j] = b.i;
  }
  __syncthreads();
  // The chirp w_n and the twist e^{-2 pi i n/L} at this thread's positions
  // n = t + j * kFftThreads < i, shared by the four quarter-length DFTs:
  // the inputs y_n w_n, the outputs w_kappa (...) and the twist powers
  // e^{-2 pi i r kappa/L} = (e^{-2 pi i kappa/L})^r.
  double wc[kCapKappa], ws[kCapKappa], tc[kCapKappa], ts[kCapKappa];
#pragma unroll
  for (int j = 0; j < kCapKappa; ++j) {
    const int64_t n = t + (int64_t)j * kFftThreads;
    wc[j] = ws[j] = tc[j] = ts[j] = 0.0;
    if (n < i) {
      chirp(n, i, wc[j], ws[j]);
      double sp, cp;
      sincospi((double)(2 * n) / (double)L, &sp, &cp);
      tc[j] = cp;
      ts[j] = -sp;
    }
  }
  // E_r(kappa) = e^{-2 pi i r kappa / L} D_r(kappa), staged in the ring's Z
  // slot at r i + kappa: the radix-4 step below reads back, from the same
  // thread, exactly the four positions kappa + s i that it then writes.
  double* Z = zslot + 2 * (2 * i * (i - 1));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int j = 0; j < kCapPer; ++j) {
      const int p = t + j * kFftThreads;
      if (p < P) {
        double ar = 0.0, ai = 0.0;
        if (j < kCapKappa && p < i) {
          const double yr = xn[4 * p + r], yi = xsth[4 * p + r];
          ar = fma(yr, wc[j], -(yi * ws[j]));
          ai = fma(yr, ws[j], yi * wc[j]);
        }
        fft_put<false>(xs, p, {ar, ai});
      }
    }
    __syncthreads();
    fft_dif<false>(xs, P, tl);
#pragma unroll
    for (int j = 0; j < kCapPer; ++j) {
      const int p = t + j * kFftThreads;
      if (p < P) {
        const cplx a = fft_get<false>(xs, p);
        fft_put<false>(xs, p, {fma(a.r, Br[j], -(a.i * Bi[j])), fma(a.r, Bi[j], a.i * Br[j])});
      }
    }
    __syncthreads();
    fft_dit_inv<false>(xs, P, tl);
#pragma unroll
    for (int j = 0; j < kCapKappa; ++j) {
      const int64_t kap = t + (int64_t)j * kFftThreads;
      if (kap < i) {
        const cplx c = fft_get<false>(xs, (int)kap);
        const double cr = c.r * inv_p, ci = c.i * inv_p;
        double dr = fma(cr, wc[j], -(ci * ws[j])), di = fma(cr, ws[j], ci * wc[j]);
        // times e^{-2 pi i r kappa / L}, r multiplications by the twist
#pragma unroll
        for (int q = 0; q < r; ++q) {
          const double er = fma(dr, tc[j], -(di * ts[j]));
          di = fma(dr, ts[j], di * tc[j]);
          dr = er;
        }
        Z[2 * (r * i + kap)] = dr;
        Z[2 * (r * i + kap) + 1] = di;
      }
    }
    __syncthreads();
  }
  // Radix-4 step: Z_{kappa + s i} = sum_r (-i)^{rs} E_r(kappa).
#pragma unroll
  for (int j = 0; j < kCapKappa; ++j) {
    const int64_t kap = t + (int64_t)j * kFftThreads;
    if (kap < i) {
      double Er[4], Ei[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Er[r] = Z[2 * (r * i + kap)];
        Ei[r] = Z[2 * (r * i + kap) + 1];
      }
      const double s0r = Er[0] + Er[2], s0i = Ei[0] + Ei[2];
      const double d0r = Er[0] - Er[2], d0i = Ei[0] - Ei[2];
      const double s1r = Er[1] + Er[3], s1i = Ei[1] + Ei[3];
      const double d1r = Er[1] - Er[3], d1i = Ei[1] - Ei[3];
      Z[2 * kap] = s0r + s1r;                 // s = 0
      Z[2 * kap + 1] = s0i + s1i;
      Z[2 * (kap + i)] = d0r + d1i;           // s = 1: E0 - i E1 - E2 + i E3
      Z[2 * (kap + i) + 1] = d0i - d1r;
      Z[2 * (kap + 2 * i)] = s0r - s1r;       // s = 2
      Z[2 * (kap + 2 * i) + 1] = s0i - s1i;
      Z[2 * (kap + 3 * i)] = d0r - d1i;       // s = 3: E0 + i E1 - E2 - i E3
      Z[2 * (kap + 3 * i) + 1] = d0i + d1r;
    }
  }
  __syncthreads();
  double* fn = F + 2 * (i - 1) * (mmax + 1);
  double* fs = F + 2 * (4 * N - i - 1) * (mmax + 1);
  const int Li = (int)L;
  for (int m = t; m <= (int)mmax; m += kFftThreads) {
    const int k = (int)((unsigned)m % (unsigned)Li), k2 = k == 0 ? 0 : Li - k;
    const double zr = Z[2 * k], zi = Z[2 * k + 1], yr = Z[2 * k2], yi = Z[2 * k2 + 1];
    const double nr = 0.5 * (zr + yr), ni = 0.5 * (zi - yi);    // (Z_k + conj Z_{L-k}) / 2
    const double sr = 0.5 * (zi + yi), si = -0.5 * (zr - yr);   // (Z_k - conj Z_{L-k}) / (2i)
    double sp, cp;
    sincospi((double)((unsigned)m % (unsigned)(2 * Li)) / (double)L, &sp, &cp);   // e^{-i pi m/L}
    fn[2 * m] = fma(nr, cp, ni * sp);
    fn[2 * m + 1] = fma(ni, cp, -(nr * sp));
    fs[2 * m] = fma(sr, cp, si * sp);
    fs[2 * m + 1] = fma(si, cp, -(sr * sp));
  }
}

// Step 2a: the pieces of lambda_mm(z) = g[m] sin^m(theta) for the north
// ring of every ring pair (its z >= 0): the factor g[m] and each ring's
// cos and sin of the colatitude.  The Legendre kernel forms sin^m itself.
// g[m] = (-1)^m sqrt(prod_{k=1}^m (2k+1)/(2k)) / sqrt(4 pi), the
// ring-independent factor of lambda_mm = g[m] sin^m(theta), for
// m = 0 .. mmax: one workgroup of 256 threads, each taking a run of
// consecutive m, then a scan of the runs' products in LDS.  Its magnitude
// grows like m^(1/4), so plain doubles hold it.
__device__ void mm_gain_block(int64_t mmax, double* g, double* part) {
  const int t = threadIdx.x;
  const int M = (int)mmax + 1;
  const int run = (M + 255) / 256;
  const int lo = t * run, hi = min(lo + run, M);
  double p = 1.0;
  for (int m = max(lo, 1); m < hi; ++m) p *= -sqrt((2.0 * m + 1.0) / (2.0 * m));
  part[t] = p;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {   // inclusive product scan
    const double o = t >= d ? part[t - d] : 1.0;
    __syncthreads();
    part[t] *= o;
    __syncthreads();
  }
  double v = (t > 0 ? part[t - 1] : 1.0) * (1.0 / sqrt(4.0 * 3.14159265358979323846));
  for (int m = lo; m < hi; ++m) {
    if (m > 0) v *= -sqrt((2.0 * m + 1.0) / (2.0 * m));
    g[m] = v;
  }
}

// cos and sin of the colatitude of ring pair q (north ring q + 1), from the
// ring's first pixel direction (sin from x and y, exact near the poles).
__device__ void ring_zs_block(int64_t nside, double* ring_z, double* ring_s, int64_t blk) {
  const int64_t q = blk * 256 + threadIdx.x;
  if (q >= 2 * nside) return;
  const Ring r = ring_of(nside, q + 1);
  double x, y, z;
  pix2vec_ring(nside, r.first, &x, &y, &z);
  ring_z[q] = z;
  ring_s[q] = sqrt(x * x + y * y);
}

// s^m as mant * 2^ex (s > 0), by binary powering with the operands
// renormalised after every product, so that no intermediate leaves the
// double range: at most 2 log2(m) roundings.
__device__ __forceinline__ void pow_scaled(double s, int m, double& mant, int& ex) {
  int eb;
  double b = frexp(s, &eb);
  double r = 1.0;
  int er = 0;
  for (int k = m; k > 0; k >>= 1) {
    int t;
    if (k & 1) {
      r = frexp(r * b, &t);
      er += t + eb;
    }
    if (k > 1) {
      b = frexp(b * b, &t);
      eb = 2 * eb + t;
    }
  }
  mant = r;
  ex = er;
}

// Step 2a': the coefficients of the rescaled recursion.  With
// lambda_lm = c_l mu_l, where c_m = c_{m+1} = 1 and c_l = -A_l B_l c_{l-2},
// the three-term recursion lambda_l = A_l (z lambda_{l-1} - B_l lambda_{l-2})
// becomes
//   mu_l = (a_l z) mu_{l-1} + mu_{l-2},   a_l = A_l c_{l-1} / c_l,
// two operations per step instead of three, and c_l multiplies the ring sum
// once per (l, m).  At l = m + 1 (B = 0) the step is mu_{m+1} =
// sqrt(2m+3) z mu_m; at l = m, a_m = 0 takes (mu_{m-1}, mu_{m-2}) =
// (0, lambda_mm) to mu_m = lambda_mm.
// One wavefront per m: A_l and g_l = -A_l B_l for 64 consecutive degrees at
// a time, one per lane (A = 0, g = 1 at l = m; A = sqrt(2m+3), g = 1 at
// l = m + 1, so that c_m = c_{m+1} = 1), then c_l as the product of g over
// l, l - 2, ... by a product scan over the lanes of equal parity (strides
// 2 .. 32), times the last c of that parity from the previous 64, and
// a_l = A_l c_{l-1} / c_l.  coef[2 i] = a_l, coef[2 i + 1] = c_l at a_lm's
// position i.
__device__ void leg_scan_block(int64_t lmax, double* coef, int64_t blk) {
  const int lane = threadIdx.x & 63;
  const int64_t m = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (m > lmax) return;
  const int64_t row = alm_idx(lmax, m, m) - m;   // idx(l, m) = row + l
  const double mm = (double)m;
  double carry0 = 1.0, carry1 = 1.0;             // c_{base-2}, c_{base-1}
  for (int64_t base = m; base <= lmax; base += 64) {
    const int64_t l = base + lane;
    const bool in = l <= lmax;
    const double ll = (double)l;
    double A, p;
    if (l == m) {
      A = 0.0;
      p = 1.0;
    } else if (l == m + 1) {
      A = sqrt(2.0 * mm + 3.0);
      p = 1.0;
    } else {
      A = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
      const double B =
          sqrt(((ll - 1.0) * (ll - 1.0) - mm * mm) / (4.0 * (ll - 1.0) * (ll - 1.0) - 1.0));
      p = -(A * B);
    }
    if (!in) p = 1.0;
#pragma unroll
    for (int s = 2; s < 64; s <<= 1) {
      const double o = __shfl_up(p, s);
      if (lane >= s) p *= o;
    }
    const double c = p * ((lane & 1) ? carry1 : carry0);
    double cm1 = __shfl_up(c, 1);
    if (lane == 0) cm1 = carry1;
    if (in) {
      coef[2 * (row + l)] = A * cm1 / c;
      coef[2 * (row + l) + 1] = c;
    }
    carry0 = __shfl(c, 62);
    carry1 = __shfl(c, 63);
  }
}

// The set-up of one call in a single launch of 256-thread workgroups, each
// taking one role by its index: the recursion coefficients (four m per
// workgroup), the lambda_mm gains (one workgroup), the ring geometry, the
// half-pixel phase table and the twiddle quarter.  The roles share nothing;
// every later kernel reads their tables.
struct SetupArgs {
  int64_t nside, lmax, L;
  double *coef, *gain, *ring_z, *ring_s, *tab, *ftab;
  int64_t n_scan, n_zs, n_tab, n_tw;   // workgroups per role, in this order after the gain's
};

__global__ void __launch_bounds__(256) k_setup(SetupArgs a) {
  __shared__ double part[256];
  int64_t b = blockIdx.x;
  if (b < a.n_scan) return leg_scan_block(a.lmax, a.coef, b);
  b -= a.n_scan;
  if (b == 0) return mm_gain_block(a.lmax, a.gain, part);
  b -= 1;
  if (b < a.n_zs) return ring_zs_block(a.nside, a.ring_z, a.ring_s, b);
  b -= a.n_zs;
  if (b < a.n_tab) return fft_table_block(a.L, a.tab, b);
  b -= a.n_tab;
  if (b < a.n_tw) fft_twiddles_block(a.ftab, b);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// x moved across lanes by a DPP pattern, as two 32-bit moves; lanes outside
// the row mask receive 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, kCtrl, kRowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), kCtrl, kRowMask, 0xf,
                                             false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

// The sum over the wavefront of x (lanes with bit b of the lane index clear)
// and of y (bit b set) as one register: the halves are exchanged across
// lanes x <-> x + 2^b and added.  b = 5 and 4 use the gfx950 half and row
// swaps; b = 3 and 2 use a row mirror and a half-row mirror written into
// the lanes that keep x (banks kLoBanks) and those that keep y (kHiBanks).
__device__ __forceinline__ double sum_swap32(double x, double y) {
  const unsigned long long ux = (unsigned long long)__double_as_longlong(x);
  const unsigned long long uy = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ux, (unsigned)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32),
                                                   false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a + b;
}

__device__ __forceinline__ double sum_swap16(double x, double y) {
  const unsigned long long ux = (unsigned long long)__double_as_longlong(x);
  const unsigned long long uy = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ux, (unsigned)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32),
                                                   false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a + b;
}

// old, with the lanes of kBanks replaced by src moved by DPP pattern kCtrl.
template <int kCtrl, int kBanks>
__device__ __forceinline__ double dpp_into(double old, double src) {
  const unsigned long long uo = (unsigned long long)__double_as_longlong(old);
  const unsigned long long us = (unsigned long long)__double_as_longlong(src);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)uo, (int)(unsigned)us, kCtrl, 0xf,
                                             kBanks, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(uo >> 32), (int)(unsigned)(us >> 32),
                                             kCtrl, 0xf, kBanks, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

template <int kCtrl, int kLoBanks, int kHiBanks>
__device__ __forceinline__ double sum_mirror(double x, double y) {
  return dpp_into<kCtrl, kLoBanks>(y, x) + dpp_into<kCtrl, kHiBanks>(x, y);
}

// Sixteen values per lane summed over the wavefront: afterwards every lane
// of quad (lane >> 2) holds the total of value (lane >> 2).  Each of the
// four halving steps pairs each lane with one whose partial sums cover a
// disjoint set of lanes, so a lane's total covers all 64 at the end.
__device__ __forceinline__ double wave_sum16(const double v[16]) {
  double r8[8], r4[4], r2[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) r8[k] = sum_swap32(v[k], v[k + 8]);
#pragma unroll
  for (int k = 0; k < 4; ++k) r4[k] = sum_swap16(r8[k], r8[k + 4]);
#pragma unroll
  for (int k = 0; k < 2; ++k) r2[k] = sum_mirror<0x140, 0x3, 0xc>(r4[k], r4[k + 2]);  // row_mirror
  double r = sum_mirror<0x141, 0x5, 0xa>(r2[0], r2[1]);                               // row_half_mirror
  r += dpp_f64<0x4E, 0xf>(r);   // quad_perm [2,3,0,1]
  r += dpp_f64<0xB1, 0xf>(r);   // quad_perm [1,0,3,2]
  return r;
}

// Step 2b: partial a_lm of one block of 64 * kRingsPerLane ring pairs, for
// one m: part[blk * S + idx(l, m)] = sum over the block's pairs of
// lambda_lm(z) (F_north +- F_south), the sign (-1)^(l+m).  Degrees are taken
// eight at a time: each lane keeps the eight partial sums (real and
// imaginary) and the wavefront sums all sixteen at once.  The 2^(600 e)
// scale of a ring's lambda is carried by its two Fourier factors instead
// (exact while they stay normal; a ring whose lambda is below 2^-177 gives
// products far below any a_lm and may lose them), so that a step is the
// recursion and two multiply-adds.
__global__ void __launch_bounds__(256) k_legendre(int64_t nside, int64_t lmax, int64_t mmax,
                                                 const double* __restrict__ F,
                                                 const double* __restrict__ gain,
                                                 const double* __restrict__ ring_z,
                                                 const double* __restrict__ ring_s,
                                                 const double* __restrict__ coef, int64_t nblk,
                                                 double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave >= (mmax + 1) * nblk) return;
  const int64_t m = wave / nblk;
  // Blocks rotate with m: workgroups go to the XCDs in turn, and with a
  // fixed block per wave slot every XCD would always get the same blocks
  // (polar or equatorial), whose work differs once negligible terms are
  // skipped.
  const int64_t blk = (wave % nblk + m) % nblk;
  const int64_t npair = 2 * nside;
  const int64_t nring = 4 * nside - 1;
  const int64_t M = mmax + 1;
  double* out = part + 2 * blk * ((lmax + 1) * (lmax + 2) / 2);
  // Degree and table indices in 32 bits (2 (lmax + 1)(lmax + 2) / 2 < 2^31
  // for lmax <= 32768), so that the loop's bounds and clamps stay on the
  // scalar unit, which has no 64-bit ordered compare.
  const int row = (int)(alm_idx(lmax, m, m) - m);   // idx(l, m) = row + l
  const int L = (int)lmax;
  const int v = lane >> 2;   // value a lane holds after the group reduction
  // A block whose every term stays below 2^-403 up to lmax writes zeros.
  // |lambda_lm(cos theta)| <= sqrt((2l+1)/(4 pi)) sin^m(theta)
  //     sqrt((l+m)!/(l-m)!) / (2^m m!),
  // from |P_l^(m)(x)| <= P_l^(m)(1) = (l+m)! / (2^m m! (l-m)!) on [-1, 1]
  // (the m-th derivative of P_l is a Gegenbauer polynomial of positive
  // index, largest at 1).  The bound grows with l and with sin(theta), so
  // its value at lmax on the block's most equatorial ring bounds the block.
  {
    const int64_t qe = min((blk + 1) * 64 * kRingsPerLane, npair) - 1;
    const double md = (double)m, Ld = (double)lmax;
    const double lg = 0.5 * log2((2.0 * Ld + 1.0) / (4.0 * 3.14159265358979323846)) +
                      md * log2(ring_s[qe]) +
                      (0.5 * (lgamma(Ld + md + 1.0) - lgamma(Ld - md + 1.0)) - lgamma(md + 1.0)) *
                          1.44269504088896340736 - md;
    if (__builtin_amdgcn_readfirstlane((int)(lg < -403.0))) {
      for (int l0 = (int)m; l0 <= L; l0 += 8)
        if ((lane & 3) == 0 && l0 + (v >> 1) <= L) out[2 * (row + l0) + v] = 0.0;
      return;
    }
  }
  double z[kRingsPerLane], cur[kRingsPerLane], prev[kRingsPerLane];
  double er[kRingsPerLane], ei[kRingsPerLane], orr[kRingsPerLane], oi[kRingsPerLane];
  int32_t sc[kRingsPerLane];
  // Fourier factors of pair k scaled by 2^(600 sc[k]).  The lane index is
  // re-read here through an opaque instruction so that the compiler cannot
  // hoist the reload's addresses out of the degree loop, where they would
  // hold 2 * kRingsPerLane 64-bit registers for a path taken a few times per
  // wavefront.
  auto factors = [&](int k) {
    int ln;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
    const int64_t q = (blk * kRingsPerLane + k) * 64 + ln;
    er[k] = ei[k] = orr[k] = oi[k] = 0.0;
    if (q < npair) {
      const int64_t north = q + 1;
      const int64_t south = nring + 1 - north;   // equal to north for the equator ring
      const double* fn = F + 2 * ((north - 1) * M + m);
      double sr = 0.0, si = 0.0;
      if (south != north) {
        const double* fs = F + 2 * ((south - 1) * M + m);
        sr = fs[0];
        si = fs[1];
      }
      const int e = kLegScale * sc[k];
      er[k] = ldexp(fn[0] + sr, e);
      ei[k] = ldexp(fn[1] + si, e);
      orr[k] = ldexp(fn[0] - sr, e);
      oi[k] = ldexp(fn[1] - si, e);
    }
  };
  // lambda_mm = g[m] sin^m(theta) as v * 2^(600 sc), 2^-602 < |v| < 8:
  // sin^m by binary powering, its binary exponent split into sc and the
  // rest.  The step at l = m moves it from prev to cur.
  const double gm = gain[m];
#pragma unroll
  for (int k = 0; k < kRingsPerLane; ++k) {
    const int64_t q = (blk * kRingsPerLane + k) * 64 + lane;   // pair index, 0-based
    z[k] = 0.0;
    cur[k] = 0.0;
    prev[k] = 0.0;
    sc[k] = 0;
    if (q < npair) {
      z[k] = ring_z[q];
      double mant;
      int ex;
      pow_scaled(ring_s[q], (int)m, mant, ex);
      if (ex < -599) sc[k] = -((-ex) / kLegScale);   // -ceil((-599 - ex) / 600)
      prev[k] = ldexp(gm * mant, ex - kLegScale * sc[k]);
    }
    factors(k);
  }
  const double big = ldexp(1.0, kLegScale);
  cdp cf = (cdp)coef;
  // Recursion coefficients a_l of degrees l0 .. l0 + 7, the next group's
  // requested one group ahead.  Degrees past lmax take lmax's: their steps
  // run (every group is eight steps) but their sums are not written.
  double cA[8];
#pragma unroll
  for (int g = 0; g < 8; ++g) cA[g] = cf[2 * (row + min((int)m + g, L))];
  // The ring data loaded above has arrived: without this wait the loop's
  // first use of it waits on every vector memory operation in flight, the
  // previous group's store included, in every iteration.
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  // Bring scaled values back once they have grown, every 32 degrees: with
  // |z| <= 1, max(|mu_l|, |mu_{l-1}|) grows by at most |a_l| + 1 per step,
  // which over any 32 consecutive degrees is below 2^200 for every
  // m <= l <= 32768, far inside the 2^424 between the 2^600 threshold and
  // the double range.  One wavefront-wide test skips the whole block when
  // no lane needs it.
  auto rescale = [&]() {
    bool need[kRingsPerLane];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kRingsPerLane; ++k) {
      need[k] = sc[k] < 0 && fmax(fabs(cur[k]), fabs(prev[k])) > big;
      any |= need[k];
    }
    if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
      for (int k = 0; k < kRingsPerLane; ++k) {
        if (need[k]) {
          cur[k] = ldexp(cur[k], -kLegScale);
          prev[k] = ldexp(prev[k], -kLegScale);
          sc[k] += 1;
          factors(k);
        }
      }
    }
  };
  for (int l0 = (int)m; l0 <= L; l0 += 8) {
    double nA[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) nA[g] = cf[2 * (row + min(l0 + 8 + g, L))];
    __builtin_amdgcn_sched_barrier(0);    // issue the requests before the arithmetic
    if (((l0 - (int)m) & 31) == 0) rescale();
    double acc[16];
#pragma unroll
    for (int g = 0; g < 16; ++g) acc[g] = 0.0;
    // Degree l0 + g: l + m has the parity of g, so even g takes
    // F_north + F_south and odd g F_north - F_south.
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      // mu_l = (a_l z) mu_{l-1} + mu_{l-2}: the product a_l z does not wait
      // on the recursion, so the dependent chain is one FMA per degree; the
      // operations run over the lane's ring pairs one after the other.
      double t[kRingsPerLane];
#pragma unroll
      for (int k = 0; k < kRingsPerLane; ++k) t[k] = cA[g] * z[k];
#pragma unroll
      for (int k = 0; k < kRingsPerLane; ++k) {
        const double nu = fma(t[k], cur[k], prev[k]);
        prev[k] = cur[k];
        cur[k] = nu;
      }
#pragma unroll
      for (int k = 0; k < kRingsPerLane; ++k) {
        acc[2 * g] = fma(cur[k], (g & 1) ? orr[k] : er[k], acc[2 * g]);
        acc[2 * g + 1] = fma(cur[k], (g & 1) ? oi[k] : ei[k], acc[2 * g + 1]);
      }
    }
    const double tot = wave_sum16(acc);
    // v: the real (even) or imaginary (odd) part of degree l0 + v/2
    if ((lane & 3) == 0 && l0 + (v >> 1) <= L) out[2 * (row + l0) + v] = tot;
#pragma unroll
    for (int g = 0; g < 8; ++g) cA[g] = nA[g];
  }
}

// Step 3: a_lm = (4 pi / Npix) c_l sum over blocks, in block order (the
// block sums are of the rescaled mu_l).
__global__ void k_alm_sum(int64_t size, int64_t nblk, double w, const double* part,
                          const double* coef, double* alm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= size) return;
  double re = 0.0, im = 0.0;
  for (int64_t b = 0; b < nblk; ++b) {
    re += part[2 * (b * size + i)];
    im += part[2 * (b * size + i) + 1];
  }
  const double f = w * coef[2 * i + 1];
  alm[2 * i] = f * re;
  alm[2 * i + 1] = f * im;
}

// C_l: one wavefront per l, lanes stride over m, then a fixed-order
// wavefront sum.
__global__ void __launch_bounds__(256) k_alm2cl(int64_t lmax, const double* alm, double* cl) {
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (l > lmax) return;
  double acc = 0.0;
  for (int64_t m = lane; m <= l; m += 64) {
    const int64_t i = alm_idx(lmax, l, m);
    const double p = alm[2 * i] * alm[2 * i] + alm[2 * i + 1] * alm[2 * i + 1];
    acc += (m == 0) ? p : 2.0 * p;
  }
  acc = wave_sum(acc);
  if (lane == 0) cl[l] = acc / (2.0 * (double)l + 1.0);
}

}  // namespace

// Doubles of the region that holds the Legendre partial sums; the cap
// rings' Z slots (2 N (N - 1) complex values) use it first.
static int64_t part_doubles(int64_t nside, int64_t lmax) {
  const int64_t npair = 2 * nside;
  const int64_t nblk = (npair + 64 * kRingsPerLane - 1) / (64 * kRingsPerLane);
  const int64_t size = (lmax + 1) * (lmax + 2) / 2;
  const int64_t zs = 4 * nside * (nside - 1);
  return 2 * nblk * size > zs ? 2 * nblk * size : zs;
}

// Scratch needs of map2alm at (nside, lmax): bytes of the Fourier table,
// the ring geometry, the recursion coefficients, the block partials and the
// small tables.
size_t map2alm_scratch_bytes(int64_t nside, int64_t lmax) {
  const int64_t M = lmax + 1;
  const int64_t nring = 4 * nside - 1, npair = 2 * nside;
  const int64_t size = (lmax + 1) * (lmax + 2) / 2;
  return sizeof(double) * (size_t)(2 * nring * M) + sizeof(double) * (size_t)(2 * npair) +
         sizeof(double) * (size_t)(2 * size) + sizeof(double) * (size_t)part_doubles(nside, lmax) +
         sizeof(double) * (size_t)(2 * (4 * nside + 1)) + sizeof(double) * (size_t)(2 * kFftMaxP) +
         sizeof(double) * (size_t)M + 8 * 256;
}

// All of map2alm on `st`; `scratch` holds map2alm_scratch_bytes(nside, lmax).
hipError_t launch_map2alm(int64_t nside, int64_t lmax, const double* map, double* alm,
                          void* scratch, hipStream_t st) {
  const int64_t M = lmax + 1;
  const int64_t nring = 4 * nside - 1, npair = 2 * nside;
  const int64_t nblk = (npair + 64 * kRingsPerLane - 1) / (64 * kRingsPerLane);
  const int64_t size = (lmax + 1) * (lmax + 2) / 2;
  auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* p = (char*)scratch;
  double* F = (double*)p;
  p += align(sizeof(double) * (size_t)(2 * nring * M));
  double* ring_z = (double*)p;
  double* ring_s = ring_z + npair;
  p += align(sizeof(double) * (size_t)(2 * npair));
  double* coef = (double*)p;
  p += align(sizeof(double) * (size_t)(2 * size));
  double* part = (double*)p;
  p += align(sizeof(double) * (size_t)part_doubles(nside, lmax));
  double* tab = (double*)p;
  p += align(sizeof(double) * (size_t)(2 * (4 * nside + 1)));
  double* ftab = (double*)p;
  p += align(sizeof(double) * (size_t)(2 * kFftMaxP));
  double* gain = (double*)p;
  const int64_t mblocks = (lmax + 64) / 64;
  // Belt rings by FFT when their length 4N is a power of two whose half
  // fits the LDS buffer; cap rings by the chirp transform when their
  // convolutions fit it; every other ring by direct sums.
  const bool fft = (nside & (nside - 1)) == 0 && 2 * nside <= kBeltMaxH;
  const bool caps = nside >= 2 && nside - 1 <= kFftMaxP / 2;
  {
    SetupArgs a;
    a.nside = nside;
    a.lmax = lmax;
    a.L = 4 * nside;
    a.coef = coef;
    a.gain = gain;
    a.ring_z = ring_z;
    a.ring_s = ring_s;
    a.tab = tab;
    a.ftab = ftab;
    a.n_scan = (M + 3) / 4;
    a.n_zs = (npair + 255) / 256;
    a.n_tab = fft ? (a.L + 256) / 256 : 0;
    a.n_tw = (fft || caps) ? (kTwQ + 255) / 256 : 0;
    const int64_t nb = a.n_scan + 1 + a.n_zs + a.n_tab + a.n_tw;
    k_setup<<<dim3((unsigned)nb), dim3(256), 0, st>>>(a);
  }
  if (fft) {
    k_ring_fft<<<dim3((unsigned)(2 * nside + 1)), dim3(kFftThreads),
                 fft_lds_bytes(2 * nside), st>>>(nside, lmax, map, tab, ftab, F);
  }
  if (caps) {
    int64_t P = 1;
    while (P < 2 * (nside - 1) - 1) P <<= 1;
    k_cap_bluestein<<<dim3((unsigned)(nside - 1)), dim3(kFftThreads),
                      fft_lds_bytes(P), st>>>(nside, lmax, map, ftab, part, F);
  }
  // Rings left for the direct sums: none, the belt, or all (Nside 1 has no
  // cap rings; a belt done by FFT implies Nside <= 2048, where the caps
  // take the chirp transform).
  const bool caps_done = caps || nside == 1;
  if (!(fft && caps_done)) {
    const int64_t lo = caps_done ? nside : 1, hi = caps_done ? 3 * nside : 4 * nside - 1;
    const int64_t dft_waves = (hi - lo + 1) * mblocks;
    k_ring_dft<<<dim3((unsigned)((dft_waves + 3) / 4)), dim3(256), 0, st>>>(nside, lmax, map, F,
                                                                           lo, hi);
  }
  const int64_t leg_waves = M * nblk;
  k_legendre<<<dim3((unsigned)((leg_waves + 3) / 4)), dim3(256), 0, st>>>(
      nside, lmax, lmax, F, gain, ring_z, ring_s, coef, nblk, part);
  const double w = 4.0 * 3.14159265358979323846 / (double)(12 * nside * nside);
  k_alm_sum<<<dim3((unsigned)((size + 255) / 256)), dim3(256), 0, st>>>(size, nblk, w, part,
                                                                        coef, alm);
  return hipGetLastError();
}

// Scratch of the allocation-free map2alm: a fixed device array, one copy per
// GPU, held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there), looked up once per device and kept.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

size_t map2alm_noalloc_max_bytes() { return kNoAllocScratchBytes; }

hipError_t map2alm_noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_alm2cl(int64_t lmax, const double* alm, double* cl, hipStream_t st) {
  k_alm2cl<<<dim3((unsigned)((lmax + 4) / 4)), dim3(256), 0, st>>>(lmax, alm, cl);
  return hipGetLastError();
}

}  // namespace csmap
