// segment_dev.h -- device-side segment geometry shared by the kernels.
//
// Box descriptors read with scalar loads, the FP64 light-cone geometry of
// one segment (event position P, distance R, slab test, eps; the rotation of
// a stacked box; the light-cone crossing of a slab-start segment), and the
// cone test of a stacked box.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace csmap {

// Plain clang vector types, loadable through constant-address-space pointers:
// loads whose address is the same in every lane become scalar loads.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef const v4f __attribute__((address_space(4)))* cf4p;
typedef const v2d __attribute__((address_space(4)))* cd2p;
typedef const int32_t __attribute__((address_space(4)))* ci32p;

typedef const DevBox __attribute__((address_space(4)))* cbox_p;
typedef const DevBoxCount __attribute__((address_space(4)))* ccnt_p;

// Box descriptor read through the constant address space, field by field, so
// that a wave-uniform box index gives scalar loads.
__device__ __forceinline__ DevBox load_box(const DevBox* boxes, int64_t b) {
  const cbox_p q = (cbox_p)boxes + b;
  DevBox r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.origin[k] = q->origin[k];
    r.ext[k] = q->ext[k];
    r.cap_dir[k] = q->cap_dir[k];
  }
  r.eta_lo = q->eta_lo;
  r.eta_hi = q->eta_hi;
  r.cap_cos = q->cap_cos;
  r.vis = q->vis;
  r.dtype = q->dtype;
  r.snapshot = q->snapshot;
  r.rotated = q->rotated;
  r.n = q->n;
  r.raw_off = q->raw_off;
  r.rec_off = q->rec_off;
  r.blk_off = q->blk_off;
  r.cone_pix = q->cone_pix;
  r.cone_nside = q->cone_nside;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.rot[k] = q->rot[k];
  return r;
}

__device__ __forceinline__ int64_t load_kept(const DevBoxCount* c, int64_t b) {
  return ((ccnt_p)c)[b].kept;
}

// ---------------------------------------------------------------------------
// Light-cone geometry of one segment (FP64).
// ---------------------------------------------------------------------------
struct SegGeom {
  double P[3], V[3], T[3];
  double R, eps, ds;
  bool keep;
};

__device__ __forceinline__ double raw_at(const char* base, int dtype, int64_t idx) {
  return dtype == 0 ? (double)((const float*)base)[idx] : ((const double*)base)[idx];
}

// Row k of a row-major 3x3 matrix times v, summed left to right (FP64).
__device__ __forceinline__ double rot_row(const double* m, int k, const double v[3]) {
  return (m[3 * k] * v[0] + m[3 * k + 1] * v[1]) + m[3 * k + 2] * v[2];
}

// Column k of a row-major 3x3 matrix times v (the transpose's row k).
__device__ __forceinline__ double rot_col(const double* m, int k, const double v[3]) {
  return (m[k] * v[0] + m[3 + k] * v[1]) + m[6 + k] * v[2];
}

// Light-cone crossing of a straight worldline.  A segment at P0 when the
// slab starts (eta_lo), moving with velocity V (|V| < 1), is at P0 + V D at
// eta = eta_lo + D; it meets the past light cone |P| = eta0 - eta where
//   (V.V - 1) D^2 + 2 (P0.V + R0) D + (P0.P0 - R0^2) = 0,  R0 = eta0 - eta_lo.
// The crossing is the smaller root (the other lies beyond D = R0, on the
// future branch).  Both roots come from q = -(b + sign(b) sqrt(b^2 - a c)) as
// q / a and c / q, so that neither subtracts nearly equal numbers, and
// c = (|P0| - R0)(|P0| + R0) avoids cancelling the two Gpc-scale squares.
__device__ __forceinline__ double cone_crossing(const double P0[3], const double V[3], double R0,
                                                double vv) {
  const double a = vv - 1.0;
  const double b = ((P0[0] * V[0] + P0[1] * V[1]) + P0[2] * V[2]) + R0;
  const double r = sqrt((P0[0] * P0[0] + P0[1] * P0[1]) + P0[2] * P0[2]);
  const double c = (r - R0) * (r + R0);
  double disc = b * b - a * c;
  disc = disc > 0.0 ? disc : 0.0;
  const double sq = sqrt(disc);
  const double q = (b >= 0.0) ? -(b + sq) : (sq - b);
  if (q == 0.0) return 0.0;   // double root at D = 0 (b = 0 and c = 0)
  const double r1 = q / a, r2 = c / q;
  return r1 < r2 ? r1 : r2;
}

// Event of a snapshot segment in the slab [eta_lo, eta_hi): its crossing D,
// and whether 0 <= D < eta_hi - eta_lo (|V| >= 1 records no event).
__device__ __forceinline__ bool snapshot_event(const double P0[3], const double V[3],
                                               double eta0, double eta_lo, double eta_hi,
                                               double vv, double& D) {
  if (!(vv < 1.0)) {
    D = __builtin_nan("");
    return false;
  }
  D = cone_crossing(P0, V, eta0 - eta_lo, vv);
  return D >= 0.0 && D < eta_hi - eta_lo;
}

// Geometry of segment i and whether it lies in its box's slab (the cone test
// of a stacked box is separate: cone_state).
__device__ __forceinline__ SegGeom seg_geom(const DevBox& bx, const char* raw, int64_t i,
                                            double eta0) {
  // Raw layout of a box: x_rel (n x 3), xdot (n x 3), xprime (n x 3), dsigma (n).
  const int dt = bx.dtype;
  const int64_t n = bx.n;
  SegGeom g;
  if (bx.rotated) {
    // A box placed in a healpix cone: its arrays are in box coordinates and
    // the box is turned onto the sky by rot (Sec. II.C).
    double x[3], v[3], t[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k] = raw_at(raw, dt, 3 * i + k);
      v[k] = raw_at(raw, dt, 3 * n + 3 * i + k);
      t[k] = raw_at(raw, dt, 6 * n + 3 * i + k);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.P[k] = bx.origin[k] + rot_row(bx.rot, k, x);
      g.V[k] = rot_row(bx.rot, k, v);
      g.T[k] = rot_row(bx.rot, k, t);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.P[k] = bx.origin[k] + raw_at(raw, dt, 3 * i + k);
      g.V[k] = raw_at(raw, dt, 3 * n + 3 * i + k);
      g.T[k] = raw_at(raw, dt, 6 * n + 3 * i + k);
    }
  }
  g.ds = raw_at(raw, dt, 9 * n + i);
  const double tt = (g.T[0] * g.T[0] + g.T[1] * g.T[1]) + g.T[2] * g.T[2];
  const double vv = (g.V[0] * g.V[0] + g.V[1] * g.V[1]) + g.V[2] * g.V[2];
  if (bx.snapshot) {
    // Positions are at the slab start: the event is where the worldline
    // meets the past light cone, if that happens inside the slab.
    double D;
    const bool in = snapshot_event(g.P, g.V, eta0, bx.eta_lo, bx.eta_hi, vv, D);
    if (in) {
#pragma unroll
      for (int k = 0; k < 3; ++k) g.P[k] = g.P[k] + g.V[k] * D;
    }
    g.R = sqrt((g.P[0] * g.P[0] + g.P[1] * g.P[1]) + g.P[2] * g.P[2]);
    g.keep = in && (g.R > 0.0);
  } else {
    g.R = sqrt((g.P[0] * g.P[0] + g.P[1] * g.P[1]) + g.P[2] * g.P[2]);
    const double eta = eta0 - g.R;
    g.keep = (g.R > 0.0) && (eta >= bx.eta_lo) && (eta < bx.eta_hi);
  }
  g.eps = sqrt(tt / (1.0 - vv));
  return g;
}

// Position, distance and slab test of segment i of a box of on-cone events:
// the same operations as seg_geom, without the velocity and tangent (the
// count pass of such boxes needs nothing else).
__device__ __forceinline__ SegGeom seg_pos(const DevBox& bx, const char* raw, int64_t i,
                                           double eta0) {
  const int dt = bx.dtype;
  SegGeom g;
  double x[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = raw_at(raw, dt, 3 * i + k);
  if (bx.rotated) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g.P[k] = bx.origin[k] + rot_row(bx.rot, k, x);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) g.P[k] = bx.origin[k] + x[k];
  }
  g.R = sqrt((g.P[0] * g.P[0] + g.P[1] * g.P[1]) + g.P[2] * g.P[2]);
  const double eta = eta0 - g.R;
  g.keep = (g.R > 0.0) && (eta >= bx.eta_lo) && (eta < bx.eta_hi);
  return g;
}

// Stacking: only the strings inside the box's healpix cone are kept.  The
// caps that bracket the pixel with a wide margin settle most directions
// (0 outside, 1 inside); the rest (2) need the pixel test.  Comparing the
// unnormalised cosine with the caps' cosines times R keeps a division out.
__device__ __forceinline__ int cone_state(const DevBox& bx, const SegGeom& g) {
  const double c = (bx.cone_dir[0] * g.P[0] + bx.cone_dir[1] * g.P[1]) + bx.cone_dir[2] * g.P[2];
  if (c < bx.cone_cos_out * g.R) return 0;
  if (c > bx.cone_cos_in * g.R) return 1;
  return 2;
}

// Copy a wave-uniform value into a vector register: an FP32 operation whose
// operands are all vector registers issues at twice the rate of one that
// reads a scalar register.
__device__ __forceinline__ float to_vgpr(float x) {
  float y;
  asm("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
  return y;
}

// Kahan update of (s, c) by x: s - c carries the sum.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

}  // namespace csmap
