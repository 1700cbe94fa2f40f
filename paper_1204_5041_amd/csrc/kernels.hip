// kernels.hip -- gfx950 kernels of libcsmap.
//
// Hot path (paper Sec. II.A, Eq. (1)-(2), summed over every segment for every
// pixel of the HEALPix sky of Sec. II.D):
//
//   precompute : per segment, P = origin + x_rel, R = |P|, the light-cone slab
//                test eta_lo <= eta0 - R < eta_hi, eps, and the per-segment
//                constants of the pair formula, all in FP64; kept segments
//                are compacted in their original order.
//   forward    : one wavefront owns a tile of 64*K consecutive RING pixels
//                (K per lane), computes their directions in-kernel, and
//                streams the segment records of every box the tile sees
//                through scalar registers: each record is fetched once per
//                wavefront with scalar loads and used by all 64 lanes.
//   adjoint    : the transpose -- one lane owns one segment, pixels stream
//                through scalar registers -- so a segment's 13 running sums
//                stay in its lane and no cross-lane reduction is needed in
//                the loop; partial sums of pixel chunks are combined by a
//                separate kernel in a fixed order.
//
// Pair formula.  With d = R n - P = R (n - Ph), Ph = P/R, and
// m = (Xdot.d') b - a (X'.d'), d' = n - Ph, a = n.X', b = 1 + n.Xdot,
// Eq. (1)-(2) give the summand -4 eps dsigma (u.d)/|d|^2 = kappa m/(b q),
// q = |n - Ph|^2, kappa = -4 eps dsigma / R.  Since n and Ph are unit
// vectors, q = 2 w with w = 1 - n.Ph, and
//   kappa/2 * (Xdot.d') = kappa/2 * b - kappa/2 (1 + Ph.Xdot)
//   kappa/2 * (X'.d')   = kappa/2 * a - kappa/2 (Ph.X')
// so the FP32 form needs only the three dot products n.Ph, n.X', n.Xdot per
// pair and two per-segment constants.  That form loses accuracy as w -> 0
// (cancellation in 1 - n.Ph), so pairs with w below a threshold take the
// direction difference n - Ph in FP64 instead.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "healpix_dev.h"
#include "internal.h"
#include "segment_dev.h"

namespace csmap {

// Pixel visibility of a box (decided in FP64 with a fixed operation order).
__device__ __forceinline__ bool sees_box(double nx, double ny, double nz, const DevBox& bx,
                                         double eta0) {
  if (bx.vis == 0) return true;
  if (bx.vis == 2) {
    const double dot = (nx * bx.cap_dir[0] + ny * bx.cap_dir[1]) + nz * bx.cap_dir[2];
    return dot >= bx.cap_cos;
  }
  const double r_lo = eta0 - bx.eta_hi;
  const double r_hi = eta0 - bx.eta_lo;
  const double n3[3] = {nx, ny, nz};
  double t_in = 0.0, t_out = __builtin_inf();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double lo = bx.origin[k];
    const double hi = bx.origin[k] + bx.ext[k];
    if (n3[k] == 0.0) {
      if (lo > 0.0 || hi < 0.0) return false;
      continue;
    }
    const double ta = lo / n3[k];
    const double tb = hi / n3[k];
    const double tmin = (ta < tb) ? ta : tb;
    const double tmax = (ta < tb) ? tb : ta;
    if (tmin > t_in) t_in = tmin;
    if (tmax < t_out) t_out = tmax;
  }
  return (t_in <= t_out) && (t_out > r_lo) && (t_in <= r_hi);
}

// ---------------------------------------------------------------------------
// Precompute: count kept segments per block, scan per box, emit records.
// ---------------------------------------------------------------------------
// Thread t of a block handles segments base + t + kPreThreads j, j < 4, so
// that every pass of the wavefront reads consecutive segments; the four
// segments' loads are in flight together.
constexpr int kPrePer = kPreBlock / kPreThreads;

// The pixel tests a block still needs are queued in LDS and run with every
// lane busy, rather than by the few lanes of each wavefront that need them.
// The few directions that neither the caps nor the edge planes settle
// (about 0.3% of the segments of a stacked grid) are queued in LDS by their
// position in the block and tested once the block's segments are done: their
// geometry is formed again and ang2pix runs with every lane busy.  Queuing
// positions rather than event coordinates keeps the block's LDS at 4 KB.
// A block belongs to one box, so its storage type and kind are uniform: the
// body is specialised on them, and the common case (positions stored, not
// slab-start snapshots) requests all of a thread's positions before using
// any of them.
struct PreShared {
  unsigned long long flags[kPreWords];
  int qpos[kPreBlock];
  int nq;
  ConeTest cone;
};

__device__ __forceinline__ void pre_keep(const PreArgs& A, const DevBox& bx, PreShared& sh,
                                         const SegGeom& g, int pos, bool& keep) {
  keep = g.keep;
  if (keep && A.flat_on) {
    const double D = (A.flat_dir[0] * g.P[0] + A.flat_dir[1] * g.P[1]) + A.flat_dir[2] * g.P[2];
    keep = (D > 0.0) && (D > A.flat_cos * g.R);
  }
  if (keep && bx.cone_nside > 0) {
    const int st = cone_state(sh.cone, g);
    keep = st == 1;
    if (st == 2) sh.qpos[atomicAdd(&sh.nq, 1)] = pos;
  }
}

template <typename T>
__device__ __forceinline__ void pre_count_pos(const PreArgs& A, const DevBox& bx, PreShared& sh,
                                              const T* x, int64_t base) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // Indices past the box's end read its last segment (a block of the box
  // starts below n) and are not used: the loads carry no branch and are all
  // in flight together.
  T v[kPrePer][3];
#pragma unroll
  for (int j = 0; j < kPrePer; ++j) {
    const int64_t i = base + threadIdx.x + kPreThreads * j;
    const int64_t ic = i < bx.n ? i : bx.n - 1;
#pragma unroll
    for (int k = 0; k < 3; ++k) v[j][k] = x[3 * ic + k];
  }
#pragma unroll
  for (int j = 0; j < kPrePer; ++j) {
    const int pos = threadIdx.x + kPreThreads * j;
    bool keep = false;
    if (base + pos < bx.n) {
      const double xd[3] = {(double)v[j][0], (double)v[j][1], (double)v[j][2]};
      pre_keep(A, bx, sh, seg_pos_at(bx, xd, A.eta0), pos, keep);
    }
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) sh.flags[(kPreThreads / 64) * j + wave] = bal;
  }
}

__device__ __forceinline__ void pre_count_snap(const PreArgs& A, const DevBox& bx, PreShared& sh,
                                               const char* raw, int64_t base) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < kPrePer; ++j) {
    const int pos = threadIdx.x + kPreThreads * j;
    bool keep = false;
    if (base + pos < bx.n) pre_keep(A, bx, sh, seg_geom(bx, raw, base + pos, A.eta0), pos, keep);
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) sh.flags[(kPreThreads / 64) * j + wave] = bal;
  }
}

__global__ void __launch_bounds__(kPreThreads) k_pre_count(PreArgs A) {
  const int64_t blk = blockIdx.x;
  const int b = ((ci32p)A.blk_box)[blk];
  const DevBox bx = load_box(A.boxes, b);
  const int64_t base = (blk - bx.blk_off) * kPreBlock;
  const char* raw = (const char*)A.raw + A.raw_byte_off[b];
  __shared__ PreShared sh;
  if (threadIdx.x == 0) sh.nq = 0;
  if (bx.cone_nside > 0) load_cone(A.boxes, b, sh.cone);
  __syncthreads();
  if (bx.snapshot) pre_count_snap(A, bx, sh, raw, base);
  else if (bx.dtype == 0) pre_count_pos(A, bx, sh, (const float*)raw, base);
  else pre_count_pos(A, bx, sh, (const double*)raw, base);
  __syncthreads();
  for (int q = threadIdx.x; q < sh.nq; q += kPreThreads) {
    const int pos = sh.qpos[q];
    const SegGeom g = bx.snapshot ? seg_geom(bx, raw, base + pos, A.eta0)
                                  : seg_pos(bx, raw, base + pos, A.eta0);
    if (ang2pix_ring(bx.cone_nside, g.P[0], g.P[1], g.P[2]) == bx.cone_pix)
      atomicOr(&sh.flags[pos >> 6], 1ull << (pos & 63));
  }
  __syncthreads();
  if (threadIdx.x < kPreWords) {
    const unsigned long long w = sh.flags[threadIdx.x];
    A.blk_mask[blk * kPreWords + threadIdx.x] = w;
    int c = __popcll(w);
#pragma unroll
    for (int off = 1; off < kPreWords; off <<= 1) c += __shfl_xor(c, off);
    if (threadIdx.x == 0) A.blk_count[blk] = c;
  }
}

// Position of the set bit of rank r (0-based) in a 64-bit word holding more
// than r set bits.
__device__ __forceinline__ int select_bit(uint64_t w, int r) {
  int pos = 0;
#pragma unroll
  for (int width = 32; width >= 1; width >>= 1) {
    const int c = __popcll(w & ((1ull << width) - 1ull));
    if (r >= c) {
      r -= c;
      w >>= width;
      pos += width;
    }
  }
  return pos;
}

// One workgroup per box: exclusive prefix of the block counts of the box.
__global__ void __launch_bounds__(256) k_pre_scan(PreArgs A, int64_t nbox) {
  const int b = blockIdx.x;
  if (b >= nbox) return;
  const DevBox bx = A.boxes[b];
  const int64_t nb = (bx.n + kPreBlock - 1) / kPreBlock;
  __shared__ int64_t sh[256];
  int64_t running = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 256) {
    const int64_t k = c0 + threadIdx.x;
    const int64_t v = (k < nb) ? (int64_t)A.blk_count[bx.blk_off + k] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (k < nb) A.blk_prefix[bx.blk_off + k] = running + sh[threadIdx.x] - v;
    const int64_t tot = sh[255];
    __syncthreads();
    running += tot;
  }
  if (threadIdx.x == 0) {
    A.box_count[b].kept = running;
    A.box_count[b].pad = 0;
  }
}

// Records by rank: record li of box b (li < kept) is the kept segment of
// rank li among the box's segments in index order.  Its block k is the last
// with exclusive prefix <= li; its rank inside the block selects a set bit of
// the block's keep flags.  A thread writes records base + t + kPreThreads j,
// j < 4, so consecutive threads write consecutive records.
__device__ __forceinline__ void emit_record(const PreArgs& A, const DevBox& bx, const char* raw,
                                            int64_t li, int64_t k0);

// Last block k in [lo, hi] with pre[k] <= li (pre[lo] <= li must hold).
__device__ __forceinline__ int64_t block_of_rank(const int64_t* pre, int64_t lo, int64_t hi,
                                                 int64_t li) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= li) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The workgroup's records (ranks base .. base + kPreBlock - 1) come from a
// short run of consecutive source blocks: two searches over the box's block
// prefixes find the run, whose prefixes are then staged in LDS, and each
// record's block is found there (a run longer than the staging buffer is
// searched in global memory, within the run).
constexpr int kEmitStage = 1024;

__global__ void __launch_bounds__(kPreThreads) k_pre_emit(PreArgs A) {
  const int64_t blk = blockIdx.x;
  const int b = ((ci32p)A.blk_box)[blk];
  const DevBox bx = load_box(A.boxes, b);
  const int64_t kept = load_kept(A.box_count, b);
  const int64_t base = (blk - bx.blk_off) * kPreBlock;
  if (base >= kept) return;
  const char* raw = (const char*)A.raw + A.raw_byte_off[b];
  const int64_t nb = (bx.n + kPreBlock - 1) / kPreBlock;
  const int64_t* pre = A.blk_prefix + bx.blk_off;
  const int64_t last = (base + kPreBlock < kept ? base + kPreBlock : kept) - 1;
  __shared__ int64_t run[2];
  __shared__ int64_t spre[kEmitStage];
  if (threadIdx.x < 2) run[threadIdx.x] = block_of_rank(pre, 0, nb - 1, threadIdx.x ? last : base);
  __syncthreads();
  const int64_t r0 = run[0], r1 = run[1];
  const bool staged = r1 - r0 < kEmitStage;
  if (staged)
    for (int64_t k = threadIdx.x; k <= r1 - r0; k += kPreThreads) spre[k] = pre[r0 + k];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPrePer; ++j) {
    const int64_t li = base + threadIdx.x + kPreThreads * j;
    if (li < kept) {
      int64_t k0;
      if (staged) {
        int lo = 0, hi = (int)(r1 - r0);
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (spre[mid] <= li) lo = mid;
          else hi = mid - 1;
        }
        k0 = r0 + lo;
      } else {
        k0 = block_of_rank(pre, r0, r1, li);
      }
      emit_record(A, bx, raw, li, k0);
    }
  }
}

// Record li, from the kept segment of rank li - pre[k0] in block k0.
__device__ __forceinline__ void emit_record(const PreArgs& A, const DevBox& bx, const char* raw,
                                            int64_t li, int64_t k0) {
  const int64_t* pre = A.blk_prefix + bx.blk_off;
  int rank = (int)(li - pre[k0]);
  // The block's keep flags are requested together (128 contiguous bytes)
  // and scanned in registers.
  const uint64_t* mask = A.blk_mask + (bx.blk_off + k0) * kPreWords;
  uint64_t mw[kPreWords];
#pragma unroll
  for (int w = 0; w < kPreWords; ++w) mw[w] = mask[w];
  int word = 0;
  uint64_t bits = mw[0];
  bool found = false;
#pragma unroll
  for (int w = 0; w < kPreWords; ++w) {
    const int c = __popcll(mw[w]);
    if (!found) {
      if (rank < c || w == kPreWords - 1) {
        found = true;
        word = w;
        bits = mw[w];
      } else {
        rank -= c;
      }
    }
  }
  const int64_t i = k0 * kPreBlock + word * 64 + select_bit(bits, rank);
  if (i >= bx.n) return;   // unreachable when the counts and flags agree
  const SegGeom g = seg_geom(bx, raw, i, A.eta0);
  const int64_t r = bx.rec_off + li;
  double Ph[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Ph[k] = g.P[k] / g.R;
  const double kappa = -4.0 * g.eps * g.ds / g.R;
  A.orig_index[r] = (int32_t)i;
  if (A.rec32) {
    const double kh = 0.5 * kappa;
    const double pv = (Ph[0] * g.V[0] + Ph[1] * g.V[1]) + Ph[2] * g.V[2];
    const double pt = (Ph[0] * g.T[0] + Ph[1] * g.T[1]) + Ph[2] * g.T[2];
    float4* o = (float4*)(A.rec32 + (size_t)r * kRec32);
    o[0] = make_float4((float)Ph[0], (float)Ph[1], (float)Ph[2], (float)g.T[0]);
    o[1] = make_float4((float)g.T[1], (float)g.T[2], (float)g.V[0], (float)g.V[1]);
    o[2] = make_float4((float)g.V[2], (float)kh, (float)(kh * (1.0 + pv)), (float)(kh * pt));
    const double vv = (g.V[0] * g.V[0] + g.V[1] * g.V[1]) + g.V[2] * g.V[2];
    const float force_near = (1.0 - sqrt(vv) < 0.05) ? 1.0f : 0.0f;
    o[3] = make_float4(__int_as_float((int)i), force_near, 0.f, 0.f);
    if (A.adjc) {
      // The adjoint's constants, without kappa (every adjoint sum is linear
      // in kappa, which the finalize step applies in FP64).
      ((float4*)A.adjc)[r] = make_float4((float)(1.0 + pv), (float)pt, 0.f, 0.f);
    }
    double2* h = (double2*)(A.phat64 + (size_t)r * 4);
    h[0] = make_double2(Ph[0], Ph[1]);
    h[1] = make_double2(Ph[2], g.R);
  }
  if (A.rec64) {
    double2* o = (double2*)(A.rec64 + (size_t)r * kRec64);
    o[0] = make_double2(Ph[0], Ph[1]);
    o[1] = make_double2(Ph[2], g.T[0]);
    o[2] = make_double2(g.T[1], g.T[2]);
    o[3] = make_double2(g.V[0], g.V[1]);
    o[4] = make_double2(g.V[2], kappa);
    // P/R carried as an unevaluated sum hi + lo: lo is the exact remainder
    // of the rounded quotient divided by R, so that n - P/R can be formed
    // accurately for directions close to the event.
    double lo[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) lo[k] = fma(-Ph[k], g.R, g.P[k]) / g.R;
    o[5] = make_double2((double)i, g.R);
    o[6] = make_double2(lo[0], lo[1]);
    o[7] = make_double2(lo[2], 0.0);
  }
}

// ---------------------------------------------------------------------------
// Light-cone events of a snapshot box, on their own (the same crossing as the
// render path): per segment the observer-relative event position, D, and
// whether the event falls inside the slab.
// ---------------------------------------------------------------------------
// One segment per thread: any alignment of the caller's arrays.
__global__ void k_cone_events_1(int64_t n, int dtype, const void* x_rel, const void* xdot,
                                double o0, double o1, double o2, double eta0, double eta_lo,
                                double eta_hi, double* pos, double* delta, uint8_t* keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const char* xr = (const char*)x_rel;
  const char* xd = (const char*)xdot;
  double P0[3], V[3];
  const double o[3] = {o0, o1, o2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P0[k] = o[k] + raw_at(xr, dtype, 3 * i + k);
    V[k] = raw_at(xd, dtype, 3 * i + k);
  }
  const double vv = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
  double D;
  const bool in = snapshot_event(P0, V, eta0, eta_lo, eta_hi, vv, D);
  const double nan = __builtin_nan("");
#pragma unroll
  for (int k = 0; k < 3; ++k) pos[3 * i + k] = in ? P0[k] + V[k] * D : nan;
  delta[i] = in ? D : nan;
  keep[i] = in ? 1 : 0;
}

// Thread t handles segments 2t and 2t + 1: their six coordinates are
// contiguous, so loads and stores move 8- and 16-byte vectors (positions
// 48 bytes, D 16 bytes, keep flags 2 bytes per thread).
template <typename Tin, typename Tin2>
__global__ void k_cone_events(int64_t n, const Tin* x_rel, const Tin* xdot, double o0, double o1,
                              double o2, double eta0, double eta_lo, double eta_hi, double* pos,
                              double* delta, uint8_t* keep) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = 2 * t;
  if (i0 >= n) return;
  const bool pair = i0 + 1 < n;
  double x[6], v[6];
  if (pair) {
    const Tin2* xr = (const Tin2*)(x_rel + 3 * i0);
    const Tin2* xd = (const Tin2*)(xdot + 3 * i0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const Tin2 a = xr[k], c = xd[k];
      x[2 * k] = (double)a.x;
      x[2 * k + 1] = (double)a.y;
      v[2 * k] = (double)c.x;
      v[2 * k + 1] = (double)c.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k] = (double)x_rel[3 * i0 + k];
      v[k] = (double)xdot[3 * i0 + k];
      x[3 + k] = 0.0;
      v[3 + k] = 0.0;
    }
  }
  const double o[3] = {o0, o1, o2};
  const double nan = __builtin_nan("");
  double p[6], d[2];
  bool in[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double P0[3], V[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      P0[k] = o[k] + x[3 * s + k];
      V[k] = v[3 * s + k];
    }
    const double vv = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
    double D;
    in[s] = snapshot_event(P0, V, eta0, eta_lo, eta_hi, vv, D);
#pragma unroll
    for (int k = 0; k < 3; ++k) p[3 * s + k] = in[s] ? P0[k] + V[k] * D : nan;
    d[s] = in[s] ? D : nan;
  }
  if (pair) {
    double2* po = (double2*)(pos + 3 * i0);
    po[0] = make_double2(p[0], p[1]);
    po[1] = make_double2(p[2], p[3]);
    po[2] = make_double2(p[4], p[5]);
    *(double2*)(delta + i0) = make_double2(d[0], d[1]);
    *(uint16_t*)(keep + i0) = (uint16_t)((in[0] ? 1u : 0u) | (in[1] ? 0x100u : 0u));
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) pos[3 * i0 + k] = p[k];
    delta[i0] = d[0];
    keep[i0] = in[0] ? 1 : 0;
  }
}

hipError_t launch_cone_events(int64_t n, int dtype, const void* x_rel, const void* xdot,
                              const double origin[3], double eta0, double eta_lo, double eta_hi,
                              double* pos, double* delta, uint8_t* keep, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t es = dtype == 0 ? 4 : 8;
  const bool aligned = ((uintptr_t)x_rel % (2 * es)) == 0 && ((uintptr_t)xdot % (2 * es)) == 0 &&
                       ((uintptr_t)pos % 16) == 0 && ((uintptr_t)delta % 16) == 0 &&
                       ((uintptr_t)keep % 2) == 0;
  if (!aligned) {
    k_cone_events_1<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(
        n, dtype, x_rel, xdot, origin[0], origin[1], origin[2], eta0, eta_lo, eta_hi, pos, delta,
        keep);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)(((n + 1) / 2 + 255) / 256)), block(256);
  if (dtype == 0)
    k_cone_events<float, float2><<<grid, block, 0, st>>>(n, (const float*)x_rel,
                                                         (const float*)xdot, origin[0], origin[1],
                                                         origin[2], eta0, eta_lo, eta_hi, pos,
                                                         delta, keep);
  else
    k_cone_events<double, double2><<<grid, block, 0, st>>>(
        n, (const double*)x_rel, (const double*)xdot, origin[0], origin[1], origin[2], eta0,
        eta_lo, eta_hi, pos, delta, keep);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utility kernels (plain stores; used instead of memset so that the
// launches can be captured in a graph).
// ---------------------------------------------------------------------------
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = v;
}

__global__ void k_zero_counters(unsigned long long* c, int n, uint32_t* work) {
  if (threadIdx.x < (unsigned)n) c[threadIdx.x] = 0ull;
  if (threadIdx.x == 0 && work) *work = 0u;
}

// Direction table in structure-of-arrays form (x, y, z each npix doubles).
__global__ void k_dir_table(int64_t nside, int64_t npix, double* x, double* y, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  double a, b, c;
  pix2vec_ring(nside, i, &a, &b, &c);
  x[i] = a;
  y[i] = b;
  z[i] = c;
}

__global__ void k_ang2pix(int64_t nside, int64_t n, const double* xyz, int64_t* pix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pix[i] = ang2pix_ring(nside, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}

__global__ void k_pix2vec(int64_t nside, int64_t first, int64_t count, double* xyz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double x, y, z;
  pix2vec_ring(nside, first + i, &x, &y, &z);
  xyz[3 * i + 0] = x;
  xyz[3 * i + 1] = y;
  xyz[3 * i + 2] = z;
}

// ---------------------------------------------------------------------------
// Forward pair kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t next_item(const FwdArgs& A, bool persistent, int lane,
                                             int64_t cur, int64_t stride) {
  if (!persistent) return cur + stride;
  uint32_t it = 0;
  if (lane == 0) it = atomicAdd(A.work_counter, 1u);
  return (int64_t)__builtin_amdgcn_readfirstlane(__shfl(it, 0));
}

__device__ __forceinline__ int32_t tile_of(const FwdArgs& A, int64_t item) {
  return A.items ? ((ci32p)A.items)[item] : (int32_t)item;
}

// The pixels of one lane in a tile: slot j is pixel first + pos0 + j step,
// present when pos0 + j step < cnt.  Ring-block tilings give each ring of
// the tile 64 / G lanes (G rings per tile) and read the ring's row from the
// table, so all K pixels of a lane lie on one ring; strips are 64 K
// consecutive pixels cut at the end of the map.  An empty row reports pixel
// 0 as its first, so that loads through it stay inside the map.
struct LaneRow {
  int64_t first;
  int32_t cnt, pos0, step;
};

template <int K>
__device__ __forceinline__ LaneRow lane_row(const FwdArgs& A, int64_t tile, int lane) {
  LaneRow r;
  if (A.rows) {
    const int g = lane >> A.ring_shift;
    const int64_t e = A.rows[tile * A.ring_g + g];
    r.first = e >> kRowCountBits;
    r.cnt = (int32_t)(e & ((1 << kRowCountBits) - 1));
    r.pos0 = lane - (g << A.ring_shift);
    r.step = 1 << A.ring_shift;
  } else {
    r.first = tile * (64 * K);
    const int64_t room = A.npix - r.first;
    r.cnt = room >= 64 * K ? 64 * K : (room > 0 ? (int32_t)room : 0);
    if (r.cnt == 0) r.first = 0;
    r.pos0 = lane;
    r.step = 64;
  }
  return r;
}

// Offset of slot j of a lane inside its row; slots past the end repeat the
// row's last pixel (or pixel `first` of an empty row).
__device__ __forceinline__ int32_t slot_off(const LaneRow& r, int j) {
  const int32_t pos = r.pos0 + j * r.step;
  return pos < r.cnt ? pos : (r.cnt > 0 ? r.cnt - 1 : 0);
}

// Fold the term m/d into the running fraction fp/fq of a window; the first
// slot of a window starts it.
__device__ __forceinline__ void fold_term(bool first, float& fp, float& fq, float m, float d) {
  if (first) {
    fp = m;
    fq = d;
  } else {
    fp = fmaf(fp, d, m * fq);
    fq = fq * d;
  }
}

// A 64-bit value every lane holds alike, moved to scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Terms of one segment for close pairs: the direction difference n - P/R
// is taken in FP64 (n from this wavefront's LDS slice, P/R from the FP64
// record) and the rest in FP32.  An exact coincidence gives m = 0 and a
// finite reciprocal, so that term is 0.
template <int K>
__device__ __forceinline__ void near_terms(const float (&nf)[K][3], const double* sdir, int lane,
                                           const v4f r0, const v4f r1, const v4f r2,
                                           const float (&a)[K], const float (&b)[K], cd2p hp,
                                           float (&part)[K]) {
  const v2d h0 = hp[0];
  const v2d h1 = hp[1];
  const float tx = r0.w, ty = r1.x, tz = r1.y;
  const float vx = r1.z, vy = r1.w, vz = r2.x;
  const float kap = r2.y;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float dx = (float)(sdir[(j * 3 + 0) * 64 + lane] - h0.x);
    const float dy = (float)(sdir[(j * 3 + 1) * 64 + lane] - h0.y);
    const float dz = (float)(sdir[(j * 3 + 2) * 64 + lane] - h1.x);
    const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float t1 = kap * fmaf(vz, dz, fmaf(vy, dy, vx * dx));
    const float t2 = kap * fmaf(tz, dz, fmaf(ty, dy, tx * dx));
    const float m = fmaf(-a[j], t2, t1 * b[j]);
    const float den = b[j] * fmaxf(0.5f * q, 1e-30f);
    part[j] = fmaf(m, __builtin_amdgcn_rcpf(den), part[j]);
  }
  (void)nf;
}

// One box's kept records [r0, r1) against a wavefront's pixels, with the
// terms m/d of a pixel folded into one fraction over windows of four
// consecutive segments, (p/q) + m/d = (p d + m q)/(q d), divided once per
// window.  Folded terms have d = b w >= 0.05 near_w (b >= 0.05 unless the
// segment is flagged), so a product of four stays inside the FP32 range.
// Terms of the FP64 path are added one by one.  Each window slot is a
// separate copy of the step, so its update of (p, q) is fixed at compile
// time.  RING: the K pixels of every lane lie on one HEALPix ring and share
// z, so each dot product n.X takes its z part from a per-segment constant.
template <int K, bool RING>
__device__ __forceinline__ void frac_box(const FwdArgs& A, cf4p recs, cd2p ph64, int64_t r0,
                                         int64_t r1, const float (&nf)[K][3],
                                         const double* sdir, int lane, const float (&vis)[K],
                                         float (&S)[K], float (&C)[K],
                                         unsigned long long& near_steps,
                                         unsigned long long& mid_steps) {
  const float near_w = A.near_w, far_w = A.far_w;
  // 32-bit counts (a box holds fewer than 2^31 records) keep the loop tests
  // on the scalar unit, which has no 64-bit ordered compare.
  const int32_t nseg = (int32_t)(r1 - r0);
  const int32_t nwin = (nseg + 3) >> 2;
  const cf4p last = recs + 4 * (r1 - 1);
  cf4p rp = recs + 4 * r0;
  v4f q0 = rp[0], q1 = rp[1], q2 = rp[2], q3 = rp[3];
  float part[K], fp[K], fq[K];
#pragma unroll
  for (int j = 0; j < K; ++j) { part[j] = 0.f; fp[j] = 0.f; fq[j] = 1.f; }
  int32_t left = A.chunk;   // segments until the next Kahan update (multiple of 4)
  for (int32_t win = 0; win < nwin; ++win) {
    const int32_t nslot = (win + 1 < nwin) ? 4 : nseg - 4 * win;
#pragma unroll
    for (int slot = 0; slot < 4; ++slot) {
      if (slot < nslot) {
        const cf4p pf = (rp != last) ? rp + 4 : rp;
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): q0..q3 have arrived
        const v4f n0 = pf[0], n1 = pf[1], n2 = pf[2], n3 = pf[3];
        // Segment constants copied to vector registers once per step: FMAs
        // whose operands are all vector registers issue at twice the rate of
        // those reading a scalar register.
        const float px = to_vgpr(q0.x), py = to_vgpr(q0.y);
        const float tx = to_vgpr(q0.w), ty = to_vgpr(q1.x);
        const float vx = to_vgpr(q1.z), vy = to_vgpr(q1.w);
        const float kap = to_vgpr(q2.y), c1v = to_vgpr(q2.z), c2v = to_vgpr(q2.w);
        float pz, tz, vz;
        float w[K], a[K], bb[K];
        bool nearp = false;
        if constexpr (RING) {
          pz = q0.z;
          tz = q1.y;
          vz = q2.x;
          const float zz = nf[0][2];
          const float cw = fmaf(-zz, pz, 1.0f), ca = zz * tz, cb = fmaf(zz, vz, 1.0f);
#pragma unroll
          for (int j = 0; j < K; ++j) {
            w[j] = fmaf(-nf[j][1], py, fmaf(-nf[j][0], px, cw));
            a[j] = fmaf(nf[j][1], ty, fmaf(nf[j][0], tx, ca));
            bb[j] = fmaf(nf[j][1], vy, fmaf(nf[j][0], vx, cb));
            nearp |= (w[j] < far_w);
          }
        } else {
          pz = to_vgpr(q0.z);
          tz = to_vgpr(q1.y);
          vz = to_vgpr(q2.x);
#pragma unroll
          for (int j = 0; j < K; ++j) {
            w[j] = fmaf(-nf[j][2], pz, fmaf(-nf[j][1], py, fmaf(-nf[j][0], px, 1.0f)));
            a[j] = fmaf(nf[j][2], tz, fmaf(nf[j][1], ty, nf[j][0] * tx));
            bb[j] = fmaf(nf[j][2], vz, fmaf(nf[j][1], vy, fmaf(nf[j][0], vx, 1.0f)));
            nearp |= (w[j] < far_w);
          }
        }
        const bool force = __float_as_int(q3.y) != 0;
        // The far step is marked likely so that it runs without a taken
        // branch (1-2% on a full-sky launch).
        if (__builtin_expect(!force && !__any(nearp), 1)) {
          // Far step: kappa/2 times Xdot.(n - Ph) and X'.(n - Ph) from the
          // dot products.
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float t1 = fmaf(kap, bb[j], -c1v);
            const float t2 = fmaf(kap, a[j], -c2v);
            const float m = fmaf(-a[j], t2, t1 * bb[j]);   // kappa/2 * m
            fold_term(slot == 0, fp[j], fq[j], m, bb[j] * w[j]);
          }
        } else {
          bool n64 = force;
#pragma unroll
          for (int j = 0; j < K; ++j) n64 |= (w[j] < near_w);
          if (!__any(n64)) {
            // Middle step: the direction difference in FP32 (its error,
            // about 1e-7 absolute, is small against |n - Ph| >= 0.01).
            ++mid_steps;
#pragma unroll
            for (int j = 0; j < K; ++j) {
              const float dx = nf[j][0] - px, dy = nf[j][1] - py, dz = nf[j][2] - pz;
              const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
              const float t1 = kap * fmaf(vz, dz, fmaf(vy, dy, vx * dx));
              const float t2 = kap * fmaf(tz, dz, fmaf(ty, dy, tx * dx));
              const float m = fmaf(-a[j], t2, t1 * bb[j]);
              fold_term(slot == 0, fp[j], fq[j], m, bb[j] * (0.5f * q));
            }
          } else {
            ++near_steps;
            near_terms<K>(nf, sdir, lane, q0, q1, q2, a, bb, ph64 + 2 * ((rp - recs) >> 2), part);
            if (slot == 0) {
#pragma unroll
              for (int j = 0; j < K; ++j) { fp[j] = 0.f; fq[j] = 1.f; }
            }
          }
        }
        q0 = n0;
        q1 = n1;
        q2 = n2;
        q3 = n3;
        rp = pf;
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) part[j] = fmaf(fp[j], __builtin_amdgcn_rcpf(fq[j]), part[j]);
    left -= 4;
    if (left <= 0 || win + 1 == nwin) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        kahan_add(S[j], C[j], part[j] * vis[j]);
        part[j] = 0.f;
      }
      left = A.chunk;
    }
  }
}

template <int K, bool PERSISTENT, bool FRAC>
__global__ void __launch_bounds__(256) k_fwd32(FwdArgs A) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  // The wavefront index is uniform; say so, so that everything derived from
  // it (tile, box, segment index) lives in scalar registers.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t item = PERSISTENT ? next_item(A, true, lane, 0, 0) : (int64_t)blockIdx.x * wpb + wave;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  unsigned long long near_steps = 0, mid_steps = 0, all_steps = 0;
  const float near_w = A.near_w, far_w = A.far_w;
  cf4p recs = (cf4p)A.rec32;
  cd2p ph64 = (cd2p)A.phat64;
  // Dynamic LDS: K x 3 x 64 doubles per wavefront of the workgroup.
  extern __shared__ double sdir_all[];
  double* const sdir = sdir_all + wave * (K * 3 * 64);
  while (item < A.nitems) {
    const int64_t tile = tile_of(A, item);
    // Pixel directions come from the table written by the RING pix2vec
    // kernel.  Slots past the end of a lane's row repeat its last pixel
    // (they are masked out of every sum and never written).  The FP64
    // directions are parked in this wavefront's slice of LDS for the
    // close-pair steps and visibility tests; only the FP32 copies stay in
    // registers across the segment loop.
    float nf[K][3];
    bool inmap[K];
    bool same_ring = true;   // this lane's K pixels share one ring (one z)
    double z0 = 0.0;
    const LaneRow lr = lane_row<K>(A, tile, lane);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      inmap[j] = lr.pos0 + j * lr.step < lr.cnt;
      const int64_t p = lr.first + slot_off(lr, j);
      const double x = A.dirx[p], y = A.diry[p], z = A.dirz[p];
      if (j == 0) z0 = z;
      same_ring = same_ring && z == z0;
      sdir[(j * 3 + 0) * 64 + lane] = x;
      sdir[(j * 3 + 1) * 64 + lane] = y;
      sdir[(j * 3 + 2) * 64 + lane] = z;
      nf[j][0] = (float)x;
      nf[j][1] = (float)y;
      nf[j][2] = (float)z;
    }
    // Ring z is computed from integers, so equal z means one ring.
    const bool ring = __all(same_ring);
    float S[K], C[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { S[j] = 0.f; C[j] = 0.f; }

    int32_t b0 = 0, b1 = A.nbox;
    if (A.only_box >= 0) { b0 = A.only_box; b1 = A.only_box + 1; }
    else if (!A.all_boxes) { b0 = ((ci32p)A.tile_ptr)[tile]; b1 = ((ci32p)A.tile_ptr)[tile + 1]; }
    for (int32_t bi = b0; bi < b1; ++bi) {
      const int32_t b = (A.all_boxes || A.only_box >= 0) ? bi : ((ci32p)A.tile_boxes)[bi];
      const DevBox bx = load_box(A.boxes, b);
      // Visibility as a per-lane 0/1 weight: partial sums of pixels that do
      // not see the box are multiplied by 0 before they reach the running
      // sum (the arithmetic on those lanes stays finite).
      float vis[K];
      unsigned long long nvis = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const bool v = inmap[j] && (bx.vis == 0 || sees_box(sdir[(j * 3 + 0) * 64 + lane],
                                                             sdir[(j * 3 + 1) * 64 + lane],
                                                             sdir[(j * 3 + 2) * 64 + lane], bx,
                                                             A.eta0));
        vis[j] = v ? 1.0f : 0.0f;
        nvis += __popcll(__ballot(v));
      }
      if (nvis == 0) continue;
      const int64_t r0 = bx.rec_off;
      int64_t r1 = r0 + load_kept(A.box_count, b);
      if (A.seg_cap > 0 && r1 - r0 > A.seg_cap) r1 = r0 + A.seg_cap;
      if (lane == 0 && r1 > r0) atomicAdd(A.pairs, nvis * (unsigned long long)(r1 - r0));
      if (r1 == r0) continue;
      all_steps += (unsigned long long)(r1 - r0);
      if constexpr (FRAC) {
        if (ring)
          frac_box<K, true>(A, recs, ph64, r0, r1, nf, sdir, lane, vis, S, C, near_steps, mid_steps);
        else
          frac_box<K, false>(A, recs, ph64, r0, r1, nf, sdir, lane, vis, S, C, near_steps, mid_steps);
      } else {
      // Segment records stream through scalar registers.  The record of the
      // next step is requested before the current one is used; the explicit
      // wait at the top of each step covers exactly the previous request.
      cf4p rp = recs + 4 * r0;
      const cf4p re = recs + 4 * r1;
      v4f q0 = rp[0], q1 = rp[1], q2 = rp[2], q3 = rp[3];
      float part[K];
#pragma unroll
      for (int j = 0; j < K; ++j) part[j] = 0.f;
      int32_t left = A.chunk;   // steps until the next Kahan update
      while (true) {
        const cf4p nxt = rp + 4;
        const bool more = nxt != re;
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): q0..q2 have arrived
        const cf4p pf = more ? nxt : rp;
        const v4f n0 = pf[0], n1 = pf[1], n2 = pf[2], n3 = pf[3];
        const float px = q0.x, py = q0.y, pz = q0.z;
        const float tx = q0.w, ty = q1.x, tz = q1.y;
        const float vx = q1.z, vy = q1.w, vz = q2.x;
        const float kap = q2.y, c1v = q2.z, c2v = q2.w;
        float w[K], a[K], bb[K];
        bool nearp = false;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          w[j] = fmaf(-nf[j][2], pz, fmaf(-nf[j][1], py, fmaf(-nf[j][0], px, 1.0f)));
          a[j] = fmaf(nf[j][2], tz, fmaf(nf[j][1], ty, nf[j][0] * tx));
          bb[j] = fmaf(nf[j][2], vz, fmaf(nf[j][1], vy, fmaf(nf[j][0], vx, 1.0f)));
          nearp |= (w[j] < far_w);
        }
        // Segments flagged at precompute (|Xdot| close to 1, where b = 1 + n.Xdot
        // may be tiny) always take the FP64 form.
        const bool force = __float_as_int(q3.y) != 0;
        bool n64 = force;
        if (!force && __any(nearp)) {
#pragma unroll
          for (int j = 0; j < K; ++j) n64 |= (w[j] < near_w);
        }
        if (__builtin_expect(!force && !__any(nearp), 1)) {
          // kappa/2 times Xdot.(n - Ph) and X'.(n - Ph) from the dot products.
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float t1 = fmaf(kap, bb[j], -c1v);
            const float t2 = fmaf(kap, a[j], -c2v);
            const float m = fmaf(-a[j], t2, t1 * bb[j]);   // kappa/2 * m
            part[j] = fmaf(m, __builtin_amdgcn_rcpf(bb[j] * w[j]), part[j]);
          }
        } else if (!__any(n64)) {
          // Middle pairs: the direction difference in FP32.
          ++mid_steps;
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float dx = nf[j][0] - px, dy = nf[j][1] - py, dz = nf[j][2] - pz;
            const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float t1 = kap * fmaf(vz, dz, fmaf(vy, dy, vx * dx));
            const float t2 = kap * fmaf(tz, dz, fmaf(ty, dy, tx * dx));
            const float m = fmaf(-a[j], t2, t1 * bb[j]);
            part[j] = fmaf(m, __builtin_amdgcn_rcpf(bb[j] * (0.5f * q)), part[j]);
          }
        } else {
          // Close pairs: the difference of directions in FP64.  An exact
          // coincidence (n == Ph) gives m = 0 and a finite reciprocal, so
          // the term is 0.
          ++near_steps;
          const cd2p hp = ph64 + 2 * ((rp - recs) >> 2);
          const v2d h0 = hp[0];
          const v2d h1 = hp[1];
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float dx = (float)(sdir[(j * 3 + 0) * 64 + lane] - h0.x);
            const float dy = (float)(sdir[(j * 3 + 1) * 64 + lane] - h0.y);
            const float dz = (float)(sdir[(j * 3 + 2) * 64 + lane] - h1.x);
            const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float t1 = kap * fmaf(vz, dz, fmaf(vy, dy, vx * dx));
            const float t2 = kap * fmaf(tz, dz, fmaf(ty, dy, tx * dx));
            const float m = fmaf(-a[j], t2, t1 * bb[j]);
            const float den = bb[j] * fmaxf(0.5f * q, 1e-30f);
            part[j] = fmaf(m, __builtin_amdgcn_rcpf(den), part[j]);
          }
        }
        --left;
        if (left == 0 || !more) {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            kahan_add(S[j], C[j], part[j] * vis[j]);
            part[j] = 0.f;
          }
          left = A.chunk;
        }
        if (!more) break;
        q0 = n0;
        q1 = n1;
        q2 = n2;
        q3 = n3;
        rp = nxt;
      }
      }
    }
    const LaneRow lw = lane_row<K>(A, tile, lane);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (lw.pos0 + j * lw.step < lw.cnt) {
        // The running sum s carries the result; c is the negated rounding
        // error still owed to it, so the value is s - c.
        const int64_t p = lw.first + lw.pos0 + j * lw.step;
        const double v = (double)S[j] - (double)C[j];
        A.map[p] = A.accumulate ? A.map[p] + v : v;
      }
    }
    item = PERSISTENT ? next_item(A, true, lane, item, stride) : item + stride;
  }
  if (lane == 0 && near_steps) atomicAdd(A.near_steps, near_steps);
  if (lane == 0 && mid_steps) atomicAdd(A.mid_steps, mid_steps);
  if (lane == 0 && all_steps) atomicAdd(A.steps, all_steps);
}

__device__ __forceinline__ double rcp_f64(double x) {
  // The hardware estimate r (relative error e = 1 - x r below 2^-24)
  // refined by one third-order step: 1/x = r / (1 - e) = r (1 + e + e^2 +
  // ...), truncated after e^2, leaves e^3 < 2^-72.  Three FMAs where two
  // Newton steps take four; both measure within 1 ulp of 1/x over 2^22
  // random operands spanning 2^-40 to 2^10.
  double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  r = fma(r, fma(e, e, e), r);
  return r;
}

// The FP64 pair steps over nk consecutive records (16 doubles each) into
// part[j].  kRing: every lane's K pixels share one z (ring-block tiles keep
// a lane on one ring), so the z parts of n - Ph, |n - Ph|^2, n.X', 1 + n.Xdot,
// Xdot.(n - Ph) and X'.(n - Ph) are formed once per record for the lane
// (3.5 fewer FP64 instructions per pair at K = 2; the sums are associated
// differently, within an ulp).
template <int K, bool kRing>
__device__ __forceinline__ void fwd64_steps(cd2p rp, int32_t nk, const double (&nd)[K][3],
                                            double (&part)[K]) {
  for (int32_t k = 0; k < nk; ++k, rp += 8) {
    const v2d q0 = rp[0];
    const v2d q1 = rp[1];
    const v2d q2 = rp[2];
    const v2d q3 = rp[3];
    const v2d q4 = rp[4];
    const v2d q6 = rp[6];
    const v2d q7 = rp[7];
    const double px = q0.x, py = q0.y, pz = q1.x;
    const double lx = q6.x, ly = q6.y, lz = q7.x;
    const double tx = q1.y, ty = q2.x, tz = q2.y;
    const double vx = q3.x, vy = q3.y, vz = q4.x;
    const double kap = q4.y;
    // (n - hi) is exact for nearby directions; the lo part then enters with
    // a single rounding.
    double dz0 = 0.0, qz = 0.0, az = 0.0, bz = 1.0, vdz = 0.0, tdz = 0.0;
    if constexpr (kRing) {
      dz0 = (nd[0][2] - pz) - lz;
      qz = dz0 * dz0;
      az = nd[0][2] * tz;
      bz = fma(nd[0][2], vz, 1.0);
      vdz = vz * dz0;
      tdz = tz * dz0;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double dx = (nd[j][0] - px) - lx;
      const double dy = (nd[j][1] - py) - ly;
      double q, a, b, vd, td;
      if constexpr (kRing) {
        q = fma(dy, dy, fma(dx, dx, qz));
        a = fma(nd[j][1], ty, fma(nd[j][0], tx, az));
        b = fma(nd[j][1], vy, fma(nd[j][0], vx, bz));
        vd = fma(vy, dy, fma(vx, dx, vdz));
        td = fma(ty, dy, fma(tx, dx, tdz));
      } else {
        const double dz = (nd[j][2] - pz) - lz;
        q = fma(dz, dz, fma(dy, dy, dx * dx));
        a = fma(nd[j][2], tz, fma(nd[j][1], ty, nd[j][0] * tx));
        b = fma(nd[j][2], vz, fma(nd[j][1], vy, fma(nd[j][0], vx, 1.0)));
        vd = fma(vz, dz, fma(vy, dy, vx * dx));
        td = fma(tz, dz, fma(ty, dy, tx * dx));
      }
      const double m = fma(vd, b, -(a * td));
      const double r = (q > 0.0) ? rcp_f64(b * q) : 0.0;
      part[j] = fma(kap * m, r, part[j]);
    }
  }
}

template <int K, bool PERSISTENT>
__global__ void __launch_bounds__(256) k_fwd64(FwdArgs A) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  // The wavefront index is uniform; say so, so that everything derived from
  // it (tile, box, segment index) lives in scalar registers.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t item = PERSISTENT ? next_item(A, true, lane, 0, 0) : (int64_t)blockIdx.x * wpb + wave;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  cd2p recs = (cd2p)A.rec64;
  while (item < A.nitems) {
    const int64_t tile = tile_of(A, item);
    double nd[K][3];
    bool inmap[K];
    bool same_ring = true;   // this lane's K pixels share one ring (one z)
    const LaneRow lr = lane_row<K>(A, tile, lane);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      inmap[j] = lr.pos0 + j * lr.step < lr.cnt;
      const int64_t pc = lr.first + slot_off(lr, j);
      nd[j][0] = A.dirx[pc];
      nd[j][1] = A.diry[pc];
      nd[j][2] = A.dirz[pc];
      same_ring = same_ring && nd[j][2] == nd[0][2];
    }
    // Ring z is computed from integers, so equal z means one ring.
    const bool ring = __all(same_ring);
    double S[K], C[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { S[j] = 0.0; C[j] = 0.0; }
    int32_t b0 = 0, b1 = A.nbox;
    if (A.only_box >= 0) { b0 = A.only_box; b1 = A.only_box + 1; }
    else if (!A.all_boxes) { b0 = ((ci32p)A.tile_ptr)[tile]; b1 = ((ci32p)A.tile_ptr)[tile + 1]; }
    for (int32_t bi = b0; bi < b1; ++bi) {
      const int32_t b = (A.all_boxes || A.only_box >= 0) ? bi : ((ci32p)A.tile_boxes)[bi];
      const DevBox bx = load_box(A.boxes, b);
      bool vis[K];
      bool anyv = false;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        vis[j] = inmap[j] && (bx.vis == 0 || sees_box(nd[j][0], nd[j][1], nd[j][2], bx, A.eta0));
        anyv |= vis[j];
      }
      if (!__any(anyv)) continue;
      const int64_t r0 = bx.rec_off;
      int64_t r1 = r0 + load_kept(A.box_count, b);
      if (A.seg_cap > 0 && r1 - r0 > A.seg_cap) r1 = r0 + A.seg_cap;
      {
        unsigned long long nvis = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) nvis += __popcll(__ballot(vis[j]));
        if (lane == 0 && r1 > r0) atomicAdd(A.pairs, nvis * (unsigned long long)(r1 - r0));
      }
      for (int64_t c0 = r0; c0 < r1; c0 += A.chunk) {
        const int64_t c1 = (c0 + A.chunk < r1) ? c0 + A.chunk : r1;
        double part[K];
#pragma unroll
        for (int j = 0; j < K; ++j) part[j] = 0.0;
        const int32_t nk = (int32_t)(c1 - c0);
        const cd2p rp = recs + 8 * c0;
        if (ring)
          fwd64_steps<K, true>(rp, nk, nd, part);
        else
          fwd64_steps<K, false>(rp, nk, nd, part);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const double y = part[j] - C[j];
          const double t = S[j] + y;
          const double cn = (t - S[j]) - y;
          S[j] = vis[j] ? t : S[j];
          C[j] = vis[j] ? cn : C[j];
        }
      }
    }
    const LaneRow lw = lane_row<K>(A, tile, lane);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (lw.pos0 + j * lw.step < lw.cnt) {
        const int64_t p = lw.first + lw.pos0 + j * lw.step;
        const double v = S[j] - C[j];
        A.map[p] = A.accumulate ? A.map[p] + v : v;
      }
    }
    item = PERSISTENT ? next_item(A, true, lane, item, stride) : item + stride;
  }
}

// ---------------------------------------------------------------------------
// Adjoint.
// ---------------------------------------------------------------------------
// Pixel table: direction (FP32) and cotangent (FP32) per pixel, plus the FP64
// direction for close pairs and visibility decisions.
// The adjoint's pixel table: per pixel n (FP32) and the cotangent, and n in
// FP64 with the cotangent; one zero record past the last pixel lets the
// pixel loop read one record ahead without a bound.
__global__ void k_pixtab(int64_t nside, int64_t npix, const double* dmap, float* tab32,
                         double* tab64) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p == npix) {
    ((float4*)tab32)[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  if (p > npix) return;
  double x, y, z;
  pix2vec_ring(nside, p, &x, &y, &z);
  ((float4*)tab32)[p] = make_float4((float)x, (float)y, (float)z, (float)dmap[p]);
  ((double2*)tab64)[2 * p + 0] = make_double2(x, y);
  ((double2*)tab64)[2 * p + 1] = make_double2(z, dmap[p]);
}

// Accumulators of one segment (see the finalize kernel for their use).  All
// of them are linear in kappa' = -2 eps dsigma / R, which is left out here
// and applied in FP64 by the finalize step.  With s the pixel's cotangent,
// d = n - Ph the direction difference of the pair, w = 1 - n.Ph = |d|^2/2,
// a = n.X', b = 1 + n.Xdot, v = Xdot.d, u = X'.d, r = 1/(b w) and
// m = v b - a u (the Eq. (1) term is kappa' m r):
//   0 S1  = sum s/w                      1 S2 = sum s a r
//   2 SF  = sum s m r                    3 C2 = sum s a u r/b
//   4 C4  = sum s u r                    5..7   D3 = sum (s m r/w) d
//   8..10 DV = sum (s/w + s a u r/b) d   11..13 DT = sum s r (u + a) d
// Every vector sum multiplies d rather than n: the n-weighted sums of the
// close pixels are each of order 1/theta larger than the result and would
// cancel against Ph times a scalar sum.
constexpr int kAcc = 14;

// Add one pair to the accumulators (see their list above): s the pixel's
// cotangent, a, b, w, v = Xdot.d, u = X'.d, r = 1/(b w), d = n - Ph.
// With g = s r: S1 += g b, S2 += g a, SF += g m, C4 += g u,
// C2 += (g u) a (w r), D3 += (g m)(b r) d, DV += (g b + C2 term) d,
// DT += (g a + g u) d: 28 instructions.
__device__ __forceinline__ void adj_accumulate(float (&pa)[kAcc], float s, float a, float bb,
                                               float w, float v, float u, float r, float dx,
                                               float dy, float dz) {
  const float g = s * r;
  const float m = fmaf(-a, u, v * bb);
  const float gm = g * m;                       // s m r
  pa[2] += gm;
  pa[0] = fmaf(g, bb, pa[0]);
  pa[1] = fmaf(g, a, pa[1]);
  const float gu = g * u;                       // s u r
  pa[4] += gu;
  const float c2 = (gu * a) * (w * r);          // s a u r / b
  pa[3] += c2;
  const float d3 = gm * (bb * r);               // s m r / w
  pa[5] = fmaf(d3, dx, pa[5]);
  pa[6] = fmaf(d3, dy, pa[6]);
  pa[7] = fmaf(d3, dz, pa[7]);
  const float dv = fmaf(g, bb, c2);             // s/w + s a u r/b
  pa[8] = fmaf(dv, dx, pa[8]);
  pa[9] = fmaf(dv, dy, pa[9]);
  pa[10] = fmaf(dv, dz, pa[10]);
  const float c3 = fmaf(g, a, gu);              // s r (u + a)
  pa[11] = fmaf(c3, dx, pa[11]);
  pa[12] = fmaf(c3, dy, pa[12]);
  pa[13] = fmaf(c3, dz, pa[13]);
}

// Per-lane constants of the adjoint's segment (see k_adj32).
struct AdjSeg {
  float px, py, pz, tx, ty, tz, vx, vy, vz;
  float c1, c2;   // 1 + Ph.Xdot, Ph.X'
  double hx, hy, hz;   // Ph in FP64
};

// The adjoint's pixel loop over [p0, p1): pixel records stream through
// scalar registers one step ahead (the table holds one padding record past
// the last pixel, so the read ahead needs no bound); the values are copied
// to vector registers so that the per-pair FMAs read vector operands only
// (twice the issue rate of scalar operands).  kVis: the box has a
// visibility rule, tested per pixel.  kForce: the group takes the FP64 form
// against every pixel.  Without it the close-pair path is marked unlikely,
// so that the far path runs straight through with the loop's back edge as
// its one taken branch (with the uniform flag tested in the loop, it took
// four to five per pixel, and the launch was 4% slower).
template <bool kVis, bool kForce>
__device__ __forceinline__ void adj_pixels(const AdjArgs& A, const DevBox& bx, const AdjSeg& g,
                                           int64_t p0, int64_t p1, double (&acc)[kAcc]) {
  const float near_w = A.near_w, far_w = A.far_w;
  cf4p tab = (cf4p)A.pixtab;
  cd2p tab64 = (cd2p)A.pix64;
  // The pixels of a ring share z: the z parts of w, a, b and d are formed
  // once per ring (whenever the z of the next pixel differs).
  uint32_t zbits = 0x40000000u;   // the bits of 2.0f: no pixel has z = 2
  float wz = 0.f, az = 0.f, bz = 0.f, dzr = 0.f;
  constexpr int J = 64;
  v4f cur = tab[p0];
  for (int64_t pc = p0; pc < p1; pc += J) {
    const int64_t pe = (pc + J < p1) ? pc + J : p1;
    float pa[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) pa[k] = 0.f;
    // A 32-bit count keeps the loop test on the scalar unit (it has no
    // 64-bit ordered compare).
    const int32_t np = (int32_t)(pe - pc);   // at most J
    for (int32_t i = 0; i < np; ++i) {
      const int64_t p = pc + i;
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): cur has arrived
      const v4f pt = cur;
      cur = tab[p + 1];
      if (kVis) {
        const v2d e0 = tab64[2 * p + 0];
        const v2d e1 = tab64[2 * p + 1];
        if (!sees_box(e0.x, e0.y, e1.x, bx, A.eta0)) continue;
      }
      // A new ring (compared as bits, so that the test stays in scalar
      // registers).
      if (__float_as_uint(pt.z) != zbits) {
        zbits = __float_as_uint(pt.z);
        const float z = to_vgpr(pt.z);
        wz = fmaf(-z, g.pz, 1.0f);
        az = z * g.tz;
        bz = fmaf(z, g.vz, 1.0f);
        dzr = z - g.pz;
      }
      const float nx = to_vgpr(pt.x), ny = to_vgpr(pt.y);
      float s = to_vgpr(pt.w);
      float w = fmaf(-ny, g.py, fmaf(-nx, g.px, wz));
      const float a = fmaf(ny, g.ty, fmaf(nx, g.tx, az));
      const float bb = fmaf(ny, g.vy, fmaf(nx, g.vx, bz));
      // The far form's values: Xdot.d = b - (1 + Ph.Xdot), X'.d = a - Ph.X'.
      // A close pixel (for some lane) overwrites them in place, which lets
      // the far form run without register copies.
      float dx = nx - g.px, dy = ny - g.py, dz = dzr;
      float v = bb - g.c1, u = a - g.c2;
      if (kForce || __builtin_expect(__any(w < far_w), 0)) {
        // Middle form: the direction difference in FP32 (see the forward
        // kernel); FP64 form: from the FP64 directions.
        if (kForce || __any(w < near_w)) {
          const v2d e0 = tab64[2 * p + 0];
          const v2d e1 = tab64[2 * p + 1];
          dx = (float)(e0.x - g.hx);
          dy = (float)(e0.y - g.hy);
          dz = (float)(e1.x - g.hz);
        }
        const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        v = fmaf(g.vz, dz, fmaf(g.vy, dy, g.vx * dx));
        u = fmaf(g.tz, dz, fmaf(g.ty, dy, g.tx * dx));
        // An exact coincidence (q = 0) contributes nothing.
        w = (q > 0.0f) ? 0.5f * q : 1.0f;
        s = (q > 0.0f) ? s : 0.0f;
      }
      adj_accumulate(pa, s, a, bb, w, v, u, __builtin_amdgcn_rcpf(bb * w), dx, dy, dz);
    }
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] += (double)pa[k];
  }
}

// Work item: a group of 64 consecutive kept records of one box (one per
// lane) and one of `nsplit` contiguous pixel ranges.
__global__ void __launch_bounds__(256) k_adj32(AdjArgs A) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t item = (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (item >= A.nitems) return;
  const int32_t b = ((ci32p)A.items)[3 * item + 0];
  const int32_t grp = ((ci32p)A.items)[3 * item + 1];
  const int32_t split = ((ci32p)A.items)[3 * item + 2];
  const DevBox bx = load_box(A.boxes, b);
  const int64_t kept = load_kept(A.box_count, b);
  const int64_t li = (int64_t)grp * 64 + lane;
  const bool active = li < kept;
  const int64_t rec = bx.rec_off + (active ? li : 0);
  // Segment constants (per lane).
  const float4* R4 = (const float4*)(A.rec32 + (size_t)rec * kRec32);
  const float4 q0 = R4[0], q1 = R4[1], q2 = R4[2], q3 = R4[3];
  // 1 + Ph.Xdot and Ph.X' (the sums leave out kappa' = -2 eps dsigma / R,
  // which the finalize step applies, so they stay finite at dsigma = 0).
  const float4 cu = ((const float4*)A.adjc)[rec];
  const double2 h0 = ((const double2*)A.phat64)[2 * rec + 0];
  const double2 h1 = ((const double2*)A.phat64)[2 * rec + 1];
  const AdjSeg g = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x,
                    cu.x, cu.y, h0.x, h0.y, h1.x};
  // The pixel range is uniform; computing it through readfirstlane keeps it
  // (and the loop bound) in scalar registers.
  const int64_t p0 = uniform_i64(A.npix * split / A.nsplit);
  const int64_t p1 = uniform_i64(A.npix * (split + 1) / A.nsplit);
  // A group holding a segment flagged at precompute takes the FP64 form
  // against every pixel.
  const bool force = __any(active && __float_as_int(q3.y) != 0);
  double acc[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k) acc[k] = 0.0;
  if (force) {
    if (bx.vis != 0)
      adj_pixels<true, true>(A, bx, g, p0, p1, acc);
    else
      adj_pixels<false, true>(A, bx, g, p0, p1, acc);
  } else {
    if (bx.vis != 0)
      adj_pixels<true, false>(A, bx, g, p0, p1, acc);
    else
      adj_pixels<false, false>(A, bx, g, p0, p1, acc);
  }
  if (active) {
    double* o = A.partial + ((size_t)rec * A.nsplit + split) * kAcc;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) o[k] = acc[k];
  }
}

struct GradPtrs {
  double* x;
  double* xd;
  double* xp;
  double* ds;
};

// Combine the pixel-chunk partials of each kept record (in chunk order) and
// apply the per-segment chain rule, then scatter to the caller's arrays.
// The partial sums leave out kappa' = -2 eps dsigma / R; with S the sums
// times k = -2 eps / R (kappa' per unit dsigma):
//   G_d   = V S1 - T S2 - D3                   (sum of s df/d(n - Ph))
//   dL/dP = dsigma [-(G_d - Ph (Ph.G_d))/R - SF Ph / R] (Ph = P/R, dR/dP = Ph)
//   dL/dV = dsigma [DV + Ph C2 + SF V/(1 - V^2)]        (the last term from eps)
//   dL/dT = dsigma [-DT - Ph C4 + SF T/T^2]             (the last term from eps)
//   dL/ddsigma = SF                            (Eq. (1) is linear in dsigma)
__global__ void k_adj_finalize(const DevBox* boxes, const DevBoxCount* counts, int32_t b,
                               const char* raw, const int32_t* orig_index,
                               const double* phat64, const double* partial, int32_t nsplit,
                               GradPtrs out) {
  const DevBox bx = boxes[b];
  const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= counts[b].kept) return;
  const int64_t rec = bx.rec_off + li;
  double S[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k) S[k] = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* pp = partial + ((size_t)rec * nsplit + sp) * kAcc;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) S[k] += pp[k];
  }
  const int64_t i = orig_index[rec];
  const int dt = bx.dtype;
  const int64_t n = bx.n;
  double V[3], T[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V[k] = raw_at(raw, dt, 3 * n + 3 * i + k);
    T[k] = raw_at(raw, dt, 6 * n + 3 * i + k);
  }
  if (bx.rotated) {
    const double v[3] = {V[0], V[1], V[2]}, t[3] = {T[0], T[1], T[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      V[k] = rot_row(bx.rot, k, v);
      T[k] = rot_row(bx.rot, k, t);
    }
  }
  const double ds = raw_at(raw, dt, 9 * n + i);
  const double Ph[3] = {phat64[4 * rec + 0], phat64[4 * rec + 1], phat64[4 * rec + 2]};
  const double R = phat64[4 * rec + 3];
  const double vv = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
  const double tt = (T[0] * T[0] + T[1] * T[1]) + T[2] * T[2];
  const double kunit = -2.0 * sqrt(tt / (1.0 - vv)) / R;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) S[k] *= kunit;
  double G[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) G[k] = V[k] * S[0] - T[k] * S[1] - S[5 + k];
  const double pg = (Ph[0] * G[0] + Ph[1] * G[1]) + Ph[2] * G[2];
  const double SF = S[2];
  double gx[3], gv[3], gt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gx[k] = ds * (-(G[k] - Ph[k] * pg) / R - SF * Ph[k] / R);
    gv[k] = ds * (S[8 + k] + Ph[k] * S[3] + SF * V[k] / (1.0 - vv));
    gt[k] = ds * (-S[11 + k] - Ph[k] * S[4] + SF * T[k] / tt);
  }
  // A rotated box: sky = rot * box, so d/d(box) = rot^T d/d(sky).
  const bool rot = bx.rotated != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (out.x) out.x[3 * i + k] = rot ? rot_col(bx.rot, k, gx) : gx[k];
    if (out.xd) out.xd[3 * i + k] = rot ? rot_col(bx.rot, k, gv) : gv[k];
    if (out.xp) out.xp[3 * i + k] = rot ? rot_col(bx.rot, k, gt) : gt[k];
  }
  if (out.ds) out.ds[i] = SF;
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the API layer).
// ---------------------------------------------------------------------------
hipError_t launch_precompute(const PreArgs& A, int64_t nbox, hipStream_t st) {
  if (nbox == 0) return hipSuccess;
  // The scan runs for every box, also when no box has segments, so that every
  // kept count the pair kernels read has been written.
  if (A.nblk) k_pre_count<<<dim3((unsigned)A.nblk), dim3(kPreThreads), 0, st>>>(A);
  k_pre_scan<<<dim3((unsigned)nbox), dim3(256), 0, st>>>(A, nbox);
  if (A.nblk) k_pre_emit<<<dim3((unsigned)A.nblk), dim3(kPreThreads), 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_f64<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned long long* c, int n, uint32_t* work, hipStream_t st) {
  k_zero_counters<<<1, 64, 0, st>>>(c, n, work);
  return hipGetLastError();
}

hipError_t launch_dir_table(int64_t nside, int64_t npix, double* x, double* y, double* z,
                           hipStream_t st) {
  k_dir_table<<<dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st>>>(nside, npix, x, y, z);
  return hipGetLastError();
}

hipError_t launch_ang2pix(int64_t nside, int64_t n, const double* xyz, int64_t* pix,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_ang2pix<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(nside, n, xyz, pix);
  return hipGetLastError();
}

hipError_t launch_pix2vec(int64_t nside, int64_t first, int64_t count, double* xyz,
                          hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_pix2vec<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(nside, first, count,
                                                                          xyz);
  return hipGetLastError();
}

static size_t fwd32_lds(int K, unsigned block) {
  return sizeof(double) * 3 * 64 * (size_t)K * (block / 64);
}

template <int K, bool P>
static void fwd_launch(bool fp64, const FwdArgs& A, unsigned grid, unsigned block,
                       hipStream_t st) {
  if (fp64)
    k_fwd64<K, P><<<dim3(grid), dim3(block), 0, st>>>(A);
  else if (A.frac)
    k_fwd32<K, P, true><<<dim3(grid), dim3(block), fwd32_lds(K, block), st>>>(A);
  else
    k_fwd32<K, P, false><<<dim3(grid), dim3(block), fwd32_lds(K, block), st>>>(A);
}

template <int K, bool P>
static int fwd_occupancy(bool fp64, bool frac, unsigned block) {
  int nb = 0;
  hipError_t e;
  if (fp64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd64<K, P>, (int)block, 0);
  else if (frac)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd32<K, P, true>, (int)block,
                                                      fwd32_lds(K, block));
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd32<K, P, false>, (int)block,
                                                      fwd32_lds(K, block));
  return e == hipSuccess ? nb : 0;
}

// Workgroups of the persistent forward kernel that fit on one CU at once.
int forward_blocks_per_cu(bool fp64, bool frac, int K, unsigned block) {
  switch (K) {
    case 1: return fwd_occupancy<1, true>(fp64, frac, block);
    case 2: return fwd_occupancy<2, true>(fp64, frac, block);
    case 4: return fwd_occupancy<4, true>(fp64, frac, block);
    case 8: return fwd_occupancy<8, true>(fp64, frac, block);
  }
  return 0;
}

hipError_t launch_forward(bool fp64, int K, bool persistent, const FwdArgs& A, unsigned grid,
                          unsigned block, hipStream_t st) {
  switch (K) {
    case 1: persistent ? fwd_launch<1, true>(fp64, A, grid, block, st)
                       : fwd_launch<1, false>(fp64, A, grid, block, st); break;
    case 2: persistent ? fwd_launch<2, true>(fp64, A, grid, block, st)
                       : fwd_launch<2, false>(fp64, A, grid, block, st); break;
    case 4: persistent ? fwd_launch<4, true>(fp64, A, grid, block, st)
                       : fwd_launch<4, false>(fp64, A, grid, block, st); break;
    case 8: persistent ? fwd_launch<8, true>(fp64, A, grid, block, st)
                       : fwd_launch<8, false>(fp64, A, grid, block, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pixtab(int64_t nside, int64_t npix, const double* dmap, float* tab32,
                         double* tab64, hipStream_t st) {
  k_pixtab<<<dim3((unsigned)((npix + 256) / 256)), dim3(256), 0, st>>>(nside, npix, dmap, tab32,
                                                                        tab64);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs& A, hipStream_t st) {
  if (A.nitems == 0) return hipSuccess;
  const unsigned grid = (unsigned)((A.nitems + 3) / 4);
  k_adj32<<<dim3(grid), dim3(256), 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_adj_finalize(const DevBox* boxes, const DevBoxCount* counts, int32_t b,
                               int64_t nseg, const char* raw, const int32_t* orig_index,
                               const double* phat64, const double* partial, int32_t nsplit,
                               double* gx, double* gxd, double* gxp, double* gds,
                               hipStream_t st) {
  if (nseg <= 0) return hipSuccess;
  GradPtrs o{gx, gxd, gxp, gds};
  k_adj_finalize<<<dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st>>>(
      boxes, counts, b, raw, orig_index, phat64, partial, nsplit, o);
  return hipGetLastError();
}

}  // namespace csmap
