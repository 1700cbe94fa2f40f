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
  return r;   // the cone test's data is read where it is used (ConeTest)
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
template <typename T>
__device__ __forceinline__ SegGeom seg_geom_t(const DevBox& bx, const T* raw, int64_t i,
                                              double eta0) {
  // Raw layout of a box: x_rel (n x 3), xdot (n x 3), xprime (n x 3), dsigma
  // (n), all of type T; every element is requested before any is used.
  const int64_t n = bx.n;
  double x[3], v[3], t[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    x[k] = (double)raw[3 * i + k];
    v[k] = (double)raw[3 * n + 3 * i + k];
    t[k] = (double)raw[6 * n + 3 * i + k];
  }
  SegGeom g;
  g.ds = (double)raw[9 * n + i];
  if (bx.rotated) {
    // A box placed in a healpix cone: its arrays are in box coordinates and
    // the box is turned onto the sky by rot (Sec. II.C).
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.P[k] = bx.origin[k] + rot_row(bx.rot, k, x);
      g.V[k] = rot_row(bx.rot, k, v);
      g.T[k] = rot_row(bx.rot, k, t);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.P[k] = bx.origin[k] + x[k];
      g.V[k] = v[k];
      g.T[k] = t[k];
    }
  }
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

__device__ __forceinline__ SegGeom seg_geom(const DevBox& bx, const char* raw, int64_t i,
                                            double eta0) {
  return bx.dtype == 0 ? seg_geom_t(bx, (const float*)raw, i, eta0)
                       : seg_geom_t(bx, (const double*)raw, i, eta0);
}

// Position, distance and slab test of a box of on-cone events from a
// segment's stored position x (box or sky coordinates, as the box holds
// them): the same operations as seg_geom, without the velocity and tangent
// (the count pass of such boxes needs nothing else).
__device__ __forceinline__ SegGeom seg_pos_at(const DevBox& bx, const double x[3], double eta0) {
  SegGeom g;
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

// The same for segment i of the box's raw arrays.
__device__ __forceinline__ SegGeom seg_pos(const DevBox& bx, const char* raw, int64_t i,
                                           double eta0) {
  double x[3];
  if (bx.dtype == 0) {
    const float* r = (const float*)raw;
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = (double)r[3 * i + k];
  } else {
    const double* r = (const double*)raw;
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = r[3 * i + k];
  }
  return seg_pos_at(bx, x, eta0);
}

// Stacking: only the strings inside the box's healpix cone are kept.  The
// caps that bracket the pixel with a wide margin settle the directions far
// from its boundary (0 outside, 1 inside), the four edge planes most of the
// others; the rest (2), within a thin band around the edges, need the pixel
// test.  Comparing unnormalised dot products with thresholds times R keeps
// a division out.  The data sits in LDS (25 doubles per box): held in
// scalar registers with the rest of the box it overflowed them.
struct ConeTest {
  double dir[3];
  double cos_out, cos_in;
  double n[4][3];
  double hi[4], lo[4];
};

// Threads 0 .. 24 of the block copy box b's cone data into t.
__device__ __forceinline__ void load_cone(const DevBox* boxes, int64_t b, ConeTest& t) {
  const DevBox& q = boxes[b];
  const int k = threadIdx.x;
  if (k < 3) t.dir[k] = q.cone_dir[k];
  else if (k == 3) t.cos_out = q.cone_cos_out;
  else if (k == 4) t.cos_in = q.cone_cos_in;
  else if (k < 17) t.n[(k - 5) / 3][(k - 5) % 3] = q.cone_n[(k - 5) / 3][(k - 5) % 3];
  else if (k < 21) t.hi[k - 17] = q.cone_hi[k - 17];
  else if (k < 25) t.lo[k - 21] = q.cone_lo[k - 21];
}

__device__ __forceinline__ int cone_state(const ConeTest& t, const SegGeom& g) {
  const double c = (t.dir[0] * g.P[0] + t.dir[1] * g.P[1]) + t.dir[2] * g.P[2];
  if (c < t.cos_out * g.R) return 0;
  if (c > t.cos_in * g.R) return 1;
  bool inside = true;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double f = (t.n[e][0] * g.P[0] + t.n[e][1] * g.P[1]) + t.n[e][2] * g.P[2];
    if (f < t.lo[e] * g.R) return 0;
    inside = inside && f > t.hi[e] * g.R;
  }
  return inside ? 1 : 2;
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
