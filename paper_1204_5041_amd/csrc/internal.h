// internal.h -- data layout shared by the host scheduler and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tiling.h"

namespace csmap {

constexpr int kMaxNside = 8192;

// Device copy of one box descriptor.
struct DevBox {
  double origin[3];
  double ext[3];
  double eta_lo, eta_hi;
  double cap_dir[3];
  double cap_cos;
  int32_t vis;       // 0 all, 1 ray crosses box inside slab radii, 2 cap
  int32_t dtype;     // 0 f32, 1 f64 raw arrays
  int32_t snapshot;  // 1: positions at eta_lo, events are the worldlines' light-cone crossings
  int32_t rotated;   // 1: raw arrays are in box coordinates; sky = rot * box
  int64_t n;         // raw segments
  int64_t raw_off;   // offset (in segments) of the raw arrays of this box
  int64_t rec_off;   // offset (in records) of this box's compacted records
  int64_t blk_off;   // first precompute block of this box
  int64_t cone_pix;  // cone_nside > 0: RING pixel of the box's healpix cone
  int32_t cone_nside;  // > 0: keep only events whose direction lies in cone_pix
  int32_t pad;
  double rot[9];     // row-major box-to-sky rotation (rotated == 1)
  // cone_nside > 0: caps around the cone axis that bracket the pixel with a
  // wide margin: cos(angle to cone_dir) < cone_cos_out is certainly outside,
  // > cone_cos_in certainly inside; in between, the planes through the ends
  // of the pixel's four edges decide most directions: n_e.d > cone_hi[e] for
  // every e is inside, n_e.d < cone_lo[e] for some e outside; only the rest
  // need ang2pix.
  double cone_dir[3];
  double cone_cos_out, cone_cos_in;
  double cone_n[4][3];
  double cone_hi[4], cone_lo[4];
};

// Per-box result of the light-cone compaction, written on the device.
struct DevBoxCount {
  int64_t kept;
  int64_t pad;
};

// FP32C segment record: 16 floats (one 64-byte scalar load).
//   [0..2]  P/R rounded to float          (unit vector towards the event)
//   [3..5]  X'                             (T)
//   [6..8]  Xdot                           (V)
//   [9]     kappa = -2 eps dsigma / R      (half of the Eq. (1) prefactor over R)
//   [10]    kappa (1 + (P/R).V)            (c1, FP64 then rounded)
//   [11]    kappa (P/R).T                  (c2, FP64 then rounded)
//   [12]    index of the segment inside its box (bit pattern of an int32)
//   [13]    1 if the segment must always take the close-pair form
//           (1 - |Xdot| < 0.05), else 0
//   [14..15] unused
constexpr int kRec32 = 16;
// FP64 record: 16 doubles.
//   [0..2] P/R rounded (hi), [3..5] X', [6..8] Xdot, [9] -4 eps dsigma / R,
//   [10] index of the segment inside its box, [11] R,
//   [12..14] P/R - hi (lo), [15] unused
constexpr int kRec64 = 16;

constexpr int kPreThreads = 256;   // threads per precompute workgroup
constexpr int kPreBlock = 1024;    // segments per precompute workgroup (4 per thread)
constexpr int kPreWords = kPreBlock / 64;  // 64-bit keep-flag words per block

struct PreArgs {
  const DevBox* boxes;
  const int32_t* blk_box;      // box of each precompute block
  int64_t nblk;
  const void* raw;             // raw segment storage (bytes)
  const int64_t* raw_byte_off; // byte offset of each box's raw arrays
  double eta0;
  int32_t* blk_count;          // kept segments per block
  uint64_t* blk_mask;          // keep flags of each block's segments (kPreBlock bits)
  int64_t* blk_prefix;         // exclusive prefix within the box
  DevBoxCount* box_count;
  float* rec32;                // FP32C records (or null)
  double* phat64;              // FP32C: P/R in FP64, 4 doubles per record
  double* rec64;               // FP64 records (or null)
  int32_t* orig_index;         // record -> index of the segment in its box
  // Adjoint only (or null): per record the FP32C constants per unit dsigma,
  // (k, k (1 + Ph.Xdot), k Ph.X', 0) with k = -2 eps / R.
  float* adjc;
  // Flat-sky patch (csmap_render_flat): when flat_on, a segment is kept only
  // if D = flat_dir.P > 0 and D > flat_cos R.
  double flat_dir[3];
  double flat_cos;
  int32_t flat_on;
};

// Arguments of the flat-sky kernels.
struct FlatArgs {
  const DevBox* boxes;
  const DevBoxCount* box_count;
  const int32_t* blk_box;
  int64_t nblk, nbox;
  const void* raw;
  const int64_t* raw_byte_off;
  const int32_t* orig_index;
  double eta0;
  double c[3], e1[3], e2[3];   // patch axis and plane axes
  double inv_h;                // 1 / pixel size (radians)
  double off_x, off_y;         // pixel coordinate of the axis: n/2 - 1/2
  int64_t nx, ny;
  int64_t* flat_off;           // [nbox + 1]: first flat record of each box; [nbox]: total (even)
  float* rec;                  // kFlatRec floats per flat record
  double* map;                 // ny x nx, row-major
};
constexpr int kFlatRec = 8;

// Arguments of the forward pair kernels.
struct FwdArgs {
  const DevBox* boxes;
  const DevBoxCount* box_count;
  int32_t nbox;
  int32_t all_boxes;           // 1: every tile sees every box (no lists)
  const int32_t* tile_ptr;     // CSR over tiles: boxes of tile t are
  const int32_t* tile_boxes;   //   tile_boxes[tile_ptr[t] .. tile_ptr[t+1])
  const int64_t* rows;         // ring-block row table, ring_g per tile (null: strips)
  int32_t ring_g;              // rings per tile (1 for strips)
  int32_t ring_shift;          // log2 of the lanes per ring, 64 / ring_g
  const int32_t* items;        // tile of each work item (null: item == tile)
  int64_t nitems;
  uint32_t* work_counter;      // persistent schedule: next item
  int64_t nside, npix;
  double eta0;
  const double* dirx;          // pixel direction table (RING order, FP64)
  const double* diry;
  const double* dirz;
  const float* rec32;
  const double* phat64;
  const double* rec64;
  float near_w;                // FP32C: pairs with 1 - n.Ph below this take the FP64 difference
  float far_w;                 // FP32C: pairs with 1 - n.Ph at or above this use dot products
  int32_t chunk;
  int32_t accumulate;          // 1: map += contribution (per-box schedule)
  int32_t only_box;            // per-box schedule: the one box (else -1)
  int32_t frac;                // FP32C: fold far pairs into a running fraction
  int32_t seg_cap;             // >0: at most this many segments per box (tuning samples)
  double* map;
  unsigned long long* pairs;   // pair counter
  unsigned long long* near_steps;
  unsigned long long* mid_steps;
  unsigned long long* steps;     // FP32C: (wavefront, segment) steps of every form
};

// Arguments of the adjoint kernels.
struct AdjArgs {
  const DevBox* boxes;
  const DevBoxCount* box_count;
  int32_t nbox;
  int64_t nside, npix;
  double eta0;
  const float* pixtab;         // per pixel: n (3 floats), dL/dTheta as float
  const double* pix64;         // per pixel: n in FP64 (4 doubles)
  const float* rec32;
  const double* phat64;
  const float* adjc;           // per record: constants per unit dsigma (see PreArgs)
  const int32_t* items;        // (box, segment group, pixel chunk) triples
  int64_t nitems;
  int32_t nsplit;              // pixel chunks per segment group
  float near_w;
  float far_w;
  double* partial;             // [record][split][13] accumulators
  const double* dmap;
};

}  // namespace csmap
