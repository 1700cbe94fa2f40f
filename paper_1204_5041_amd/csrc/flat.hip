// flat.hip -- flat-sky small-angle maps on a gnomonic patch.
//
// The small-angle, flat-sky form of Eq. (1) (Sec. II.A: X n -> X, every
// photon path parallel to the patch axis c; Sec. III.B, Fig. 3 compares such
// maps with a gnomonic projection of the full-sky map).  A segment at P, at
// depth D = c.P, is seen at the plane position s = (e1.P, e2.P)/D; with u
// built from c instead of n, u = Xdot - (c.X')/(1 + c.Xdot) X', pixel t
// receives -4 eps dsigma (u_perp . (t - s)) / (D |t - s|^2).
//
//   records : per kept segment (the light-cone stage, with the patch's
//             acceptance cone, has compacted them), the plane position in
//             pixel units as an FP32 pair hi + lo and the two weights
//             a = -4 eps dsigma u_perp / (D h), from FP64 geometry;
//   pairs   : one wavefront owns 64 x 8 pixels of one row (8 consecutive
//             pixels per lane, sharing their row offset), records stream
//             through scalar registers two at a time (the next pair
//             requested before the current one is used), and the two terms
//             of a pixel are folded into one fraction before the division.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "segment_dev.h"

namespace csmap {

constexpr int kFlatK = 8;            // pixels per lane
constexpr int kFlatChunk = 32;       // records per FP32 partial sum
constexpr float kFlatTiny = 1e-18f;  // floor of |t - s|^2 (pixel units): an exact hit gives 0

// 1/x for x in [2^-125, 2^125] on the ordinary FP32 pipeline: the hardware
// reciprocal is a transcendental instruction that costs the pair loop about
// ten ordinary ones.  Subtracting the bits of x = 2^E (1 + f) from those of
// 2^127 would negate the exponent and map the mantissa to 2 - f, a seed y0
// with x y0 in [1, 1.125]; the constant used, 0x7EF311C2, is that one less
// 847422, the shift that minimises max |1 - x y0| over all mantissas (5.05e-2).
// A Newton step of third order, y <- y + y (e + e^2) with e = 1 - x y, cubes
// the relative error (to 1.3e-4), one of second order, y <- y + y e, squares
// it (to 1.7e-8), which leaves the result within 0.8 ulp of 1/x (the hardware
// reciprocal is within 1 ulp).
__device__ __forceinline__ float recip_newton(float x) {
  float y = __uint_as_float(0x7EF311C2u - __float_as_uint(x));
  float e = fmaf(-x, y, 1.0f);
  y = fmaf(y, fmaf(e, e, e), y);
  e = fmaf(-x, y, 1.0f);
  return fmaf(y, e, y);
}

// Exclusive prefix over boxes of their kept counts; the total is padded to
// an even count with one zero-weight record.
__global__ void __launch_bounds__(256) k_flat_scan(FlatArgs A) {
  __shared__ int64_t sh[256];
  int64_t running = 0;
  for (int64_t c0 = 0; c0 < A.nbox; c0 += 256) {
    const int64_t b = c0 + threadIdx.x;
    const int64_t v = (b < A.nbox) ? A.box_count[b].kept : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < A.nbox) A.flat_off[b] = running + sh[threadIdx.x] - v;
    const int64_t tot = sh[255];
    __syncthreads();
    running += tot;
  }
  if (threadIdx.x == 0) {
    if (running & 1) {
      float* z = A.rec + (size_t)running * kFlatRec;
      for (int k = 0; k < kFlatRec; ++k) z[k] = 0.f;
      ++running;
    }
    A.flat_off[A.nbox] = running;
  }
}

// One thread per kept record (four per thread, as the emit pass).
__global__ void __launch_bounds__(kPreThreads) k_flat_rec(FlatArgs A) {
  const int64_t blk = blockIdx.x;
  const int b = ((ci32p)A.blk_box)[blk];
  const DevBox bx = load_box(A.boxes, b);
  const int64_t kept = load_kept(A.box_count, b);
  const int64_t base = (blk - bx.blk_off) * kPreBlock;
  if (base >= kept) return;
  const char* raw = (const char*)A.raw + A.raw_byte_off[b];
  const int64_t out0 = A.flat_off[b];
  for (int j = 0; j < kPreBlock / kPreThreads; ++j) {
    const int64_t li = base + threadIdx.x + kPreThreads * j;
    if (li >= kept) break;
    const int64_t i = A.orig_index[bx.rec_off + li];
    const SegGeom g = seg_geom(bx, raw, i, A.eta0);
    const double D = (A.c[0] * g.P[0] + A.c[1] * g.P[1]) + A.c[2] * g.P[2];
    const double ca = (A.c[0] * g.T[0] + A.c[1] * g.T[1]) + A.c[2] * g.T[2];
    const double cb = 1.0 + ((A.c[0] * g.V[0] + A.c[1] * g.V[1]) + A.c[2] * g.V[2]);
    double u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = g.V[k] - (ca / cb) * g.T[k];
    const double kap = -4.0 * g.eps * g.ds / D * A.inv_h;
    const double sx = ((A.e1[0] * g.P[0] + A.e1[1] * g.P[1]) + A.e1[2] * g.P[2]) / D * A.inv_h +
                      A.off_x;
    const double sy = ((A.e2[0] * g.P[0] + A.e2[1] * g.P[1]) + A.e2[2] * g.P[2]) / D * A.inv_h +
                      A.off_y;
    const float sxh = (float)sx, syh = (float)sy;
    const float ax = (float)(kap * ((A.e1[0] * u[0] + A.e1[1] * u[1]) + A.e1[2] * u[2]));
    const float ay = (float)(kap * ((A.e2[0] * u[0] + A.e2[1] * u[1]) + A.e2[2] * u[2]));
    float4* o = (float4*)(A.rec + (size_t)(out0 + li) * kFlatRec);
    o[0] = make_float4(sxh, (float)(sx - (double)sxh), syh, (float)(sy - (double)syh));
    o[1] = make_float4(ax, ay, 0.f, 0.f);
  }
}

// Pair kernel: work item w = 4 blockIdx.x + (wavefront) is tile w mod ntiles
// (row y, columns 512 c .. 512 c + 511; lane l holds 512 c + 8 l + j) and
// record range s = w / ntiles of nsplit equal ranges (even bounds).  With one
// range the sums go to the map, else to parts[s][pixel] for k_flat_combine.
__global__ void __launch_bounds__(256) k_flat32(FlatArgs A, int64_t ntiles, int64_t tpr,
                                               int64_t nsplit, double* parts) {
  const int lane = threadIdx.x & 63;
  // The wavefront's index through readfirstlane: everything derived from it
  // (tile, record range, record addresses) then lives in scalar registers and
  // the records arrive by scalar loads.
  const int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (item >= ntiles * nsplit) return;
  const int64_t split = item / ntiles, tile = item - split * ntiles;
  const int64_t y = tile / tpr;
  const int64_t x0 = (tile - y * tpr) * (64 * kFlatK) + (int64_t)lane * kFlatK;
  const float fy = (float)y, fx = (float)x0;
  const int64_t nrec_all = ((const int64_t __attribute__((address_space(4)))*)A.flat_off)[A.nbox];
  const int64_t half = nrec_all / 2;
  const int64_t rbeg = 2 * (half * split / nsplit), rend = 2 * (half * (split + 1) / nsplit);
  const int64_t nrec = rend - rbeg;
  const cf4p recs = (cf4p)A.rec + 2 * rbeg;
  float acc[kFlatK], cmp[kFlatK], part[kFlatK];
#pragma unroll
  for (int j = 0; j < kFlatK; ++j) {
    acc[j] = 0.f;
    cmp[j] = 0.f;
    part[j] = 0.f;
  }
  int in_chunk = 0;
  // The next window's records are requested before this window's arithmetic
  // (an empty range reads the first window and uses none of it).
  const cf4p rec0 = nrec > 0 ? recs : (cf4p)A.rec;
  v4f pa = rec0[0], wa = rec0[1], pb = rec0[2], wb = rec0[3];
  for (int64_t r = 0; r < nrec; r += 2) {
    const int64_t rn = (r + 2 < nrec) ? r + 2 : r;
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this window's records have arrived
    const v4f npa = recs[2 * rn], nwa = recs[2 * rn + 1];
    const v4f npb = recs[2 * rn + 2], nwb = recs[2 * rn + 3];
    __builtin_amdgcn_sched_barrier(0);    // issue the requests before the arithmetic
    // x - s = ((x0 - s_hi) + j) - s_lo: the first two steps are exact for
    // a pixel near the segment, so s_lo is subtracted at the scale of the
    // pixel's own offset (subtracting it before adding j would round at the
    // scale of x0 - s and cost nearly-coincident pairs their accuracy).
    const float hxa = fx - pa.x, dya = (fy - pa.z) - pa.w;
    const float hxb = fx - pb.x, dyb = (fy - pb.z) - pb.w;
    const float ya2 = fmaf(dya, dya, kFlatTiny), yb2 = fmaf(dyb, dyb, kFlatTiny);
    const float aya = wa.y * dya, ayb = wb.y * dyb;
    const float sla = to_vgpr(pa.y), slb = to_vgpr(pb.y);
    const float uxa = to_vgpr(wa.x), uxb = to_vgpr(wb.x);
    // Each stage runs over the lane's K pixels before the next starts, so
    // that K independent operations separate dependent ones.
    float xa[kFlatK], xb[kFlatK], qa[kFlatK], qb[kFlatK], rq[kFlatK];
#pragma unroll
    for (int j = 0; j < kFlatK; ++j) {
      xa[j] = (hxa + (float)j) - sla;
      xb[j] = (hxb + (float)j) - slb;
    }
#pragma unroll
    for (int j = 0; j < kFlatK; ++j) {
      qa[j] = fmaf(xa[j], xa[j], ya2);
      qb[j] = fmaf(xb[j], xb[j], yb2);
    }
#pragma unroll
    // qa qb >= kFlatTiny^2 = 1e-36 > 2^-125, and below 2^122 because the
    // entry point admits only patches whose pixel offsets stay below 2^30:
    // inside recip_newton's range.
    for (int j = 0; j < kFlatK; ++j) rq[j] = recip_newton(qa[j] * qb[j]);
#pragma unroll
    for (int j = 0; j < kFlatK; ++j) {
      const float na = fmaf(uxa, xa[j], aya), nb = fmaf(uxb, xb[j], ayb);
      const float num = fmaf(na, qb[j], nb * qa[j]);
      part[j] = fmaf(num, rq[j], part[j]);
    }
    pa = npa;
    wa = nwa;
    pb = npb;
    wb = nwb;
    in_chunk += 2;
    if (in_chunk == kFlatChunk) {
#pragma unroll
      for (int j = 0; j < kFlatK; ++j) {
        kahan_add(acc[j], cmp[j], part[j]);
        part[j] = 0.f;
      }
      in_chunk = 0;
    }
  }
  double* out = (nsplit == 1 ? A.map : parts + split * (A.nx * A.ny)) + y * A.nx;
#pragma unroll
  for (int j = 0; j < kFlatK; ++j) {
    kahan_add(acc[j], cmp[j], part[j]);
    if (x0 + j < A.nx) out[x0 + j] = (double)acc[j] - (double)cmp[j];
  }
}

// map[p] = sum over record ranges of part[s][p], in range order.
__global__ void k_flat_combine(int64_t npix, int64_t nsplit, const double* part, double* map) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double v = part[p];
  for (int64_t s = 1; s < nsplit; ++s) v += part[s * npix + p];
  map[p] = v;
}

// Caller directions (n x 3, any positive length) as unit vectors in three
// arrays, the layout the forward kernels read pixel directions from.
__global__ void k_dirs_soa(int64_t n, const double* xyz, double* x, double* y, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = xyz[3 * i], b = xyz[3 * i + 1], c = xyz[3 * i + 2];
  const double r = sqrt((a * a + b * b) + c * c);
  x[i] = a / r;
  y[i] = b / r;
  z[i] = c / r;
}

hipError_t launch_dirs_soa(int64_t n, const double* xyz, double* x, double* y, double* z,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_dirs_soa<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(n, xyz, x, y, z);
  return hipGetLastError();
}

hipError_t launch_flat(const FlatArgs& A, hipStream_t st) {
  k_flat_scan<<<1, 256, 0, st>>>(A);
  if (A.nblk) k_flat_rec<<<dim3((unsigned)A.nblk), dim3(kPreThreads), 0, st>>>(A);
  return hipGetLastError();
}

// Record ranges per tile: enough that the launch has about 32768
// wavefronts (32 per SIMD), at most 16.  Each wavefront's chain of
// dependent operations leaves the SIMD idle unless several others are
// resident; on the 1024 x 1024 patch (2048 tiles) 1, 2, 4, 8 and 16 ranges
// measured 445, 407, 384, 372 and 366 ms with the hardware reciprocal, and
// 8, 16 and 32 ranges 317, 311 and 308 ms with recip_newton (32 would double
// the partial maps for 1%).  With more than one range, part holds that many
// maps of nx ny doubles, summed in range order.
int64_t flat_splits(int64_t nx, int64_t ny) {
  const int64_t tpr = (nx + 64 * kFlatK - 1) / (64 * kFlatK);
  const int64_t ntiles = tpr * ny;
  int64_t ns = (32768 + ntiles - 1) / ntiles;
  return ns < 1 ? 1 : (ns > 16 ? 16 : ns);
}

hipError_t launch_flat_pairs(const FlatArgs& A, int64_t nsplit, double* part, hipStream_t st) {
  const int64_t tpr = (A.nx + 64 * kFlatK - 1) / (64 * kFlatK);
  const int64_t ntiles = tpr * A.ny;
  k_flat32<<<dim3((unsigned)((ntiles * nsplit + 3) / 4)), dim3(256), 0, st>>>(A, ntiles, tpr,
                                                                             nsplit, part);
  if (nsplit > 1) {
    const int64_t npix = A.nx * A.ny;
    k_flat_combine<<<dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st>>>(npix, nsplit,
                                                                               part, A.map);
  }
  return hipGetLastError();
}

}  // namespace csmap
