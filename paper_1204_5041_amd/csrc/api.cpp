// api.cpp -- the C ABI of libcsmap (include/csmap.h): sky state, argument
// validation, device memory, launch planning, graph capture and tuning.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/csmap.h"
#include "internal.h"
#include "cones.h"
#include "sched.h"

namespace csmap {
hipError_t launch_precompute(const PreArgs& A, int64_t nbox, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_zero_counters(unsigned long long* c, int n, uint32_t* work, hipStream_t st);
hipError_t launch_pix2vec(int64_t nside, int64_t first, int64_t count, double* xyz,
                          hipStream_t st);
hipError_t launch_ang2pix(int64_t nside, int64_t n, const double* xyz, int64_t* pix,
                          hipStream_t st);
hipError_t launch_flat(const FlatArgs& A, hipStream_t st);
hipError_t launch_dirs_soa(int64_t n, const double* xyz, double* x, double* y, double* z,
                           hipStream_t st);
hipError_t launch_flat_pairs(const FlatArgs& A, int64_t nsplit, double* part, hipStream_t st);
int64_t flat_splits(int64_t nx, int64_t ny);
hipError_t launch_dir_table(int64_t nside, int64_t npix, double* x, double* y, double* z,
                            hipStream_t st);
hipError_t launch_cone_events(int64_t n, int dtype, const void* x_rel, const void* xdot,
                              const double origin[3], double eta0, double eta_lo, double eta_hi,
                              double* pos, double* delta, uint8_t* keep, hipStream_t st);
size_t map2alm_scratch_bytes(int64_t nside, int64_t lmax);
size_t map2alm_noalloc_max_bytes();
hipError_t map2alm_noalloc_scratch(void** ptr);
hipError_t launch_valu_probe(int kind, int64_t blocks, int64_t iters, void* out, hipStream_t st);
int64_t valu_probe_chains();
hipError_t launch_map2alm(int64_t nside, int64_t lmax, const double* map, double* alm,
                          void* scratch, hipStream_t st);
hipError_t launch_alm2cl(int64_t lmax, const double* alm, double* cl, hipStream_t st);
hipError_t launch_forward(bool fp64, int K, bool persistent, const FwdArgs& A, unsigned grid,
                          unsigned block, hipStream_t st);
int forward_blocks_per_cu(bool fp64, bool frac, int K, unsigned block);
hipError_t launch_pixtab(int64_t nside, int64_t npix, const double* dmap, float* tab32,
                         double* tab64, hipStream_t st);
hipError_t launch_adjoint(const AdjArgs& A, hipStream_t st);
hipError_t launch_adj_finalize(const DevBox* boxes, const DevBoxCount* counts, int32_t b,
                               int64_t nseg, const char* raw, const int32_t* orig_index,
                               const double* phat64, const double* partial, int32_t nsplit,
                               double* gx, double* gxd, double* gxp, double* gds,
                               hipStream_t st);
}  // namespace csmap

using namespace csmap;

namespace {

thread_local std::string g_err;

csmap_status fail(csmap_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// Device allocation that only grows; contents are not preserved on growth.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

struct HostBox {
  HostBoxGeom geom;
  int snapshot;     // 1: positions at the slab start (csmap_add_snapshot_box)
  int rotated = 0;  // 1: box-frame arrays turned onto the sky by rot (csmap_add_cone_box)
  int64_t cone_nside = 0, cone_pix = 0;
  double rot[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double cone_dir[3] = {0, 0, 1};
  double cone_cos_out = -2.0, cone_cos_in = 2.0;
  ConeEdges cone_edge = {};
  int dtype;
  int64_t n;
  int64_t raw_byte_off;
};

}  // namespace

struct csmap_sky {
  int64_t nside = 0, npix = 0;
  double eta0 = 0.0;
  csmap_form form = CSMAP_FORM_FP32C;
  hipStream_t stream = nullptr;
  bool failed = false;

  // options (defaults: the fastest measured shape for the FP32C form)
  int K = 8;
  int waves = 4;
  int schedule = 1;
  int graph = 0;
  int chunk = 32;
  double near_w = 5e-5;
  double far_w = 5e-3;
  int adj_split = 0;
  int frac = 1;
  int tiling = 0;   // 0 auto, 1 strips, 2 ring blocks
  int block_rings = 0;  // ring blocks: rings per tile (0: chosen from K)

  // boxes and raw segment storage (append-only)
  std::vector<HostBox> boxes;
  DevBuf raw;
  size_t raw_used = 0;
  int64_t total_seg = 0;

  // derived device state, rebuilt when `dirty`
  bool dirty = true;
  int planned_K = -1;
  int planned_tiling = -1;
  int planned_rings = -1;
  Tiling plan;
  DevBuf d_rows;     // ring-block row table (empty for strips)
  DevBuf d_boxes, d_blk_box, d_blk_count, d_blk_prefix, d_box_count, d_raw_off, d_blk_mask;
  DevBuf d_flat_off, d_flat_rec, d_flat_part;
  DevBuf d_udir;      // caller directions of csmap_render_dirs, x | y | z
  DevBuf d_rec32, d_phat64, d_rec64, d_orig;
  DevBuf d_tile_ptr, d_tile_boxes, d_items, d_box_items;
  std::vector<int64_t> box_items_off;  // per box offset into d_box_items (+ end)
  int64_t nblk = 0;
  int64_t ntiles = 0;
  int64_t nitems_sorted = 0;
  bool all_boxes = true;
  DevBuf d_counters;  // [0] pairs, [1] FP64 steps, [2] work counter (uint32), [3] middle steps,
                      // [4] all steps
  DevBuf d_dir;       // pixel directions, x | y | z (npix doubles each)
  bool dir_ready = false;

  // adjoint scratch
  DevBuf d_pixtab32, d_pix64, d_partial, d_adj_items, d_adjc;

  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph_h = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double* graph_map = nullptr;
  uint64_t graph_version = ~0ull;
  uint64_t version = 1;

  // timing
  hipEvent_t ev[6] = {};
  double ms_pre = 0, ms_fwd = 0, ms_bwd = 0;
  bool have_fwd_time = false, have_bwd_time = false;
  bool timed_graph = false;
};

namespace {

csmap_status dev_fail(csmap_sky* s, hipError_t e, const char* what) {
  if (s) s->failed = true;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(e == hipErrorOutOfMemory ? CSMAP_E_NOMEM : CSMAP_E_DEVICE, m);
}

#define HIPCHK(sky, call, what)                         \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return dev_fail(sky, e_, what); \
  } while (0)

csmap_status check_sky(csmap_sky* s) {
  if (!s) return fail(CSMAP_E_INVALID, "sky is NULL");
  if (s->failed) return fail(CSMAP_E_STATE, "sky is unusable after an earlier device error");
  return CSMAP_OK;
}

void drop_graph(csmap_sky* s) {
  if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
  if (s->graph_h) (void)hipGraphDestroy(s->graph_h);
  s->graph_exec = nullptr;
  s->graph_h = nullptr;
  s->graph_version = ~0ull;
  s->graph_map = nullptr;
}

int64_t tile_pixels(const csmap_sky* s) { return 64 * (int64_t)s->K; }

// Compact ring blocks by default.  With visibility rules a tile on the rim
// of a box's region carries lanes that do not see it, and a strip of
// consecutive RING pixels would carry far more of them; where every box
// sees every pixel they measured about 3% faster than strips as well (one
// 400,000-segment box at Nside 2048: 5.85 s against 6.02 s), every lane's
// pixels lying on one ring.
bool use_blocks(const csmap_sky* s) { return s->tiling != 1; }

// Rings per ring-block tile: 2 K rows of 32 pixels unless set.
int block_rings(const csmap_sky* s) { return s->block_rings > 0 ? s->block_rings : 2 * s->K; }

// Rebuild descriptors, compaction tables, record storage and the tile plan.
csmap_status prepare(csmap_sky* s) {
  if (!s->dirty && s->planned_K == s->K && s->planned_tiling == s->tiling &&
      s->planned_rings == block_rings(s))
    return CSMAP_OK;
  const int64_t nbox = (int64_t)s->boxes.size();
  hipStream_t st = s->stream;
  // Box descriptors and precompute blocks.
  std::vector<DevBox> db(nbox);
  std::vector<int32_t> blk_box;
  std::vector<int64_t> raw_off(nbox);
  int64_t rec = 0;
  for (int64_t b = 0; b < nbox; ++b) {
    const HostBox& h = s->boxes[b];
    DevBox& d = db[b];
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) {
      d.origin[k] = h.geom.origin[k];
      d.ext[k] = h.geom.ext[k];
      d.cap_dir[k] = h.geom.cap_dir[k];
    }
    d.eta_lo = h.geom.eta_lo;
    d.eta_hi = h.geom.eta_hi;
    d.cap_cos = h.geom.cap_cos;
    d.vis = h.geom.vis;
    d.dtype = h.dtype;
    d.snapshot = h.snapshot;
    d.rotated = h.rotated;
    d.cone_nside = (int32_t)h.cone_nside;
    d.cone_pix = h.cone_pix;
    for (int k = 0; k < 9; ++k) d.rot[k] = h.rot[k];
    for (int k = 0; k < 3; ++k) d.cone_dir[k] = h.cone_dir[k];
    d.cone_cos_out = h.cone_cos_out;
    d.cone_cos_in = h.cone_cos_in;
    for (int e = 0; e < 4; ++e) {
      for (int k = 0; k < 3; ++k) d.cone_n[e][k] = h.cone_edge.n[e][k];
      d.cone_hi[e] = h.cone_edge.hi[e];
      d.cone_lo[e] = h.cone_edge.lo[e];
    }
    d.n = h.n;
    d.raw_off = 0;
    d.rec_off = rec;
    d.blk_off = (int64_t)blk_box.size();
    const int64_t nb = (h.n + kPreBlock - 1) / kPreBlock;
    for (int64_t k = 0; k < nb; ++k) blk_box.push_back((int32_t)b);
    raw_off[b] = h.raw_byte_off;
    rec += h.n;
  }
  s->nblk = (int64_t)blk_box.size();
  const int64_t nrec = std::max<int64_t>(rec, 1);
  HIPCHK(s, s->d_boxes.ensure(sizeof(DevBox) * std::max<int64_t>(nbox, 1)), "alloc boxes");
  HIPCHK(s, s->d_blk_box.ensure(sizeof(int32_t) * std::max<int64_t>(s->nblk, 1)), "alloc blocks");
  HIPCHK(s, s->d_blk_count.ensure(sizeof(int32_t) * std::max<int64_t>(s->nblk, 1)), "alloc blocks");
  HIPCHK(s, s->d_blk_prefix.ensure(sizeof(int64_t) * std::max<int64_t>(s->nblk, 1)), "alloc blocks");
  HIPCHK(s, s->d_blk_mask.ensure(sizeof(uint64_t) * kPreWords *
                                 std::max<int64_t>(s->nblk, 1)), "alloc blocks");
  HIPCHK(s, s->d_box_count.ensure(sizeof(DevBoxCount) * std::max<int64_t>(nbox, 1)), "alloc counts");
  HIPCHK(s, s->d_raw_off.ensure(sizeof(int64_t) * std::max<int64_t>(nbox, 1)), "alloc offsets");
  HIPCHK(s, s->d_orig.ensure(sizeof(int32_t) * nrec), "alloc records");
  if (s->form == CSMAP_FORM_FP32C) {
    HIPCHK(s, s->d_rec32.ensure(sizeof(float) * kRec32 * nrec), "alloc records");
    HIPCHK(s, s->d_phat64.ensure(sizeof(double) * 4 * nrec), "alloc records");
  } else {
    HIPCHK(s, s->d_rec64.ensure(sizeof(double) * kRec64 * nrec), "alloc records");
    HIPCHK(s, s->d_phat64.ensure(sizeof(double) * 4 * nrec), "alloc records");
  }
  HIPCHK(s, s->d_counters.ensure(64), "alloc counters");
  if (!s->dir_ready) {
    HIPCHK(s, s->d_dir.ensure(sizeof(double) * 3 * (size_t)s->npix), "alloc direction table");
    double* d = s->d_dir.as<double>();
    HIPCHK(s, launch_dir_table(s->nside, s->npix, d, d + s->npix, d + 2 * s->npix, st),
           "direction table");
    s->dir_ready = true;
  }
  if (nbox) {
    HIPCHK(s, hipMemcpyAsync(s->d_boxes.p, db.data(), sizeof(DevBox) * nbox,
                             hipMemcpyHostToDevice, st), "upload boxes");
    HIPCHK(s, hipMemcpyAsync(s->d_raw_off.p, raw_off.data(), sizeof(int64_t) * nbox,
                             hipMemcpyHostToDevice, st), "upload offsets");
  }
  if (s->nblk)
    HIPCHK(s, hipMemcpyAsync(s->d_blk_box.p, blk_box.data(), sizeof(int32_t) * s->nblk,
                             hipMemcpyHostToDevice, st), "upload blocks");

  // Tile plan.
  std::vector<int64_t> rows;
  if (use_blocks(s)) {
    const int G = block_rings(s);
    make_ring_blocks(s->nside, G, 64 * (int64_t)s->K / G, s->plan);
    ring_block_rows(s->plan, rows);
    HIPCHK(s, s->d_rows.ensure(sizeof(int64_t) * rows.size()), "alloc rows");
    HIPCHK(s, hipMemcpyAsync(s->d_rows.p, rows.data(), sizeof(int64_t) * rows.size(),
                             hipMemcpyHostToDevice, st), "upload rows");
  } else {
    make_strips(s->nside, tile_pixels(s), s->plan);
    s->d_rows.release();
  }
  s->ntiles = s->plan.ntiles;
  s->all_boxes = true;
  for (auto& h : s->boxes)
    if (h.geom.vis != 0) s->all_boxes = false;
  std::vector<std::vector<std::pair<int64_t, int64_t>>> ranges(nbox);
  std::vector<int64_t> cnt(s->ntiles + 1, 0);
  std::vector<double> cost(s->ntiles, 0.0);
  for (int64_t b = 0; b < nbox; ++b) {
    box_tiles(s->plan, s->boxes[b].geom, s->eta0, ranges[b]);
    for (auto& r : ranges[b])
      for (int64_t t = r.first; t <= r.second; ++t) {
        cnt[t + 1] += 1;
        cost[t] += (double)s->boxes[b].n;
      }
  }
  std::vector<int32_t> tile_ptr(s->ntiles + 1, 0), tile_boxes;
  if (!s->all_boxes) {
    for (int64_t t = 0; t < s->ntiles; ++t) tile_ptr[t + 1] = (int32_t)(tile_ptr[t] + cnt[t + 1]);
    tile_boxes.resize(std::max<int64_t>(tile_ptr[s->ntiles], 1));
    std::vector<int32_t> fillp(tile_ptr.begin(), tile_ptr.end() - 1);
    for (int64_t b = 0; b < nbox; ++b)
      for (auto& r : ranges[b])
        for (int64_t t = r.first; t <= r.second; ++t) tile_boxes[fillp[t]++] = (int32_t)b;
    HIPCHK(s, s->d_tile_ptr.ensure(sizeof(int32_t) * tile_ptr.size()), "alloc tiles");
    HIPCHK(s, s->d_tile_boxes.ensure(sizeof(int32_t) * tile_boxes.size()), "alloc tiles");
    HIPCHK(s, hipMemcpyAsync(s->d_tile_ptr.p, tile_ptr.data(), sizeof(int32_t) * tile_ptr.size(),
                             hipMemcpyHostToDevice, st), "upload tiles");
    HIPCHK(s, hipMemcpyAsync(s->d_tile_boxes.p, tile_boxes.data(),
                             sizeof(int32_t) * tile_boxes.size(), hipMemcpyHostToDevice, st),
           "upload tiles");
  }
  // Persistent schedule: tiles ordered by decreasing work.
  std::vector<int32_t> order(s->ntiles);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  s->nitems_sorted = s->ntiles;
  HIPCHK(s, s->d_items.ensure(sizeof(int32_t) * std::max<int64_t>(s->ntiles, 1)), "alloc items");
  HIPCHK(s, hipMemcpyAsync(s->d_items.p, order.data(), sizeof(int32_t) * s->ntiles,
                           hipMemcpyHostToDevice, st), "upload items");
  // Per-box schedule: the tiles of each box.
  std::vector<int32_t> bitems;
  s->box_items_off.assign(nbox + 1, 0);
  for (int64_t b = 0; b < nbox; ++b) {
    for (auto& r : ranges[b])
      for (int64_t t = r.first; t <= r.second; ++t) bitems.push_back((int32_t)t);
    s->box_items_off[b + 1] = (int64_t)bitems.size();
  }
  HIPCHK(s, s->d_box_items.ensure(sizeof(int32_t) * std::max<size_t>(bitems.size(), 1)),
         "alloc items");
  if (!bitems.empty())
    HIPCHK(s, hipMemcpyAsync(s->d_box_items.p, bitems.data(), sizeof(int32_t) * bitems.size(),
                             hipMemcpyHostToDevice, st), "upload items");
  // Host staging vectors go out of scope below: wait for the copies.
  HIPCHK(s, hipStreamSynchronize(st), "upload plan");
  s->dirty = false;
  s->planned_K = s->K;
  s->planned_tiling = s->tiling;
  s->planned_rings = block_rings(s);
  return CSMAP_OK;
}

PreArgs pre_args(csmap_sky* s) {
  PreArgs A;
  memset(&A, 0, sizeof(A));
  A.boxes = s->d_boxes.as<DevBox>();
  A.blk_box = s->d_blk_box.as<int32_t>();
  A.nblk = s->nblk;
  A.raw = s->raw.p;
  A.raw_byte_off = s->d_raw_off.as<int64_t>();
  A.eta0 = s->eta0;
  A.blk_count = s->d_blk_count.as<int32_t>();
  A.blk_prefix = s->d_blk_prefix.as<int64_t>();
  A.blk_mask = s->d_blk_mask.as<uint64_t>();
  A.box_count = s->d_box_count.as<DevBoxCount>();
  if (s->form == CSMAP_FORM_FP32C) {
    A.rec32 = s->d_rec32.as<float>();
  } else {
    A.rec64 = s->d_rec64.as<double>();
  }
  A.phat64 = s->d_phat64.as<double>();
  A.orig_index = s->d_orig.as<int32_t>();
  return A;
}

FwdArgs fwd_args(csmap_sky* s, double* map) {
  FwdArgs A;
  memset(&A, 0, sizeof(A));
  A.boxes = s->d_boxes.as<DevBox>();
  A.box_count = s->d_box_count.as<DevBoxCount>();
  A.nbox = (int32_t)s->boxes.size();
  A.all_boxes = s->all_boxes ? 1 : 0;
  A.tile_ptr = s->d_tile_ptr.as<int32_t>();
  A.tile_boxes = s->d_tile_boxes.as<int32_t>();
  A.rows = s->plan.blocks ? s->d_rows.as<int64_t>() : nullptr;
  A.ring_g = s->plan.blocks ? s->plan.rings : 1;
  A.ring_shift = 0;   // log2(64 / ring_g): lane l serves ring l >> ring_shift of its tile
  while ((1 << A.ring_shift) * A.ring_g < 64) ++A.ring_shift;
  A.items = nullptr;
  A.nitems = s->ntiles;
  A.work_counter = (uint32_t*)(s->d_counters.as<unsigned long long>() + 2);
  A.nside = s->nside;
  A.npix = s->npix;
  A.eta0 = s->eta0;
  A.dirx = s->d_dir.as<double>();
  A.diry = A.dirx + s->npix;
  A.dirz = A.dirx + 2 * s->npix;
  A.rec32 = s->d_rec32.as<float>();
  A.phat64 = s->d_phat64.as<double>();
  A.rec64 = s->d_rec64.as<double>();
  A.near_w = (float)s->near_w;
  A.far_w = (float)std::max(s->far_w, s->near_w);
  A.frac = s->frac;
  A.chunk = s->chunk;
  A.accumulate = 0;
  A.only_box = -1;
  A.map = map;
  A.pairs = s->d_counters.as<unsigned long long>();
  A.near_steps = s->d_counters.as<unsigned long long>() + 1;
  A.mid_steps = s->d_counters.as<unsigned long long>() + 3;
  A.steps = s->d_counters.as<unsigned long long>() + 4;
  return A;
}

// Host check, before any forward launch, that the plan matches what the
// kernels index with: tile count, pixels per lane and the ring-block row
// table (64 / ring_g lanes per ring, ring_g rows per tile).
csmap_status check_forward(const csmap_sky* s, const FwdArgs& A, int K) {
  const Tiling& t = s->plan;
  if (K != s->planned_K || t.ntiles != s->ntiles)
    return fail(CSMAP_E_STATE, "forward launch does not match the tile plan");
  if (A.rows) {
    if (!t.blocks || A.ring_g != t.rings || (1 << A.ring_shift) * A.ring_g != 64 ||
        t.width * t.rings != 64 * (int64_t)K ||
        s->d_rows.cap < sizeof(int64_t) * (size_t)t.ntiles * (size_t)t.rings)
      return fail(CSMAP_E_STATE, "ring-block row table does not match the launch");
  } else if (t.blocks || t.tile_px != 64 * (int64_t)K) {
    return fail(CSMAP_E_STATE, "strip tiling does not match the launch");
  }
  if (!A.items && A.nitems > t.ntiles)
    return fail(CSMAP_E_STATE, "more work items than tiles");
  return CSMAP_OK;
}

unsigned persistent_grid(const csmap_sky* s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // Exactly the workgroups that are resident at once: every wavefront pulls
  // tiles until the queue is empty.
  int per_cu = forward_blocks_per_cu(s->form == CSMAP_FORM_FP64, s->frac != 0, s->K,
                                     64u * (unsigned)s->waves);
  if (per_cu <= 0) per_cu = 1;
  return (unsigned)std::max(1, cus * per_cu);
}

// Enqueue the whole render on stream st (no synchronisation, no events).
csmap_status enqueue_render(csmap_sky* s, double* map, hipStream_t st, bool with_events) {
  const bool fp64 = s->form == CSMAP_FORM_FP64;
  const PreArgs P = pre_args(s);
  FwdArgs A = fwd_args(s, map);
  const csmap_status cs = check_forward(s, A, s->K);
  if (cs != CSMAP_OK) return cs;
  if (with_events) HIPCHK(s, hipEventRecord(s->ev[0], st), "event");
  HIPCHK(s, launch_precompute(P, (int64_t)s->boxes.size(), st), "precompute launch");
  HIPCHK(s, launch_zero_counters(s->d_counters.as<unsigned long long>(), 5,
                                 (uint32_t*)(s->d_counters.as<unsigned long long>() + 2), st),
         "counter reset");
  if (with_events) HIPCHK(s, hipEventRecord(s->ev[1], st), "event");
  const unsigned block = 64u * (unsigned)s->waves;
  if (s->schedule == 2) {
    HIPCHK(s, launch_fill(map, s->npix, 0.0, st), "map clear");
    A.accumulate = 1;
    for (int64_t b = 0; b < (int64_t)s->boxes.size(); ++b) {
      const int64_t n = s->box_items_off[b + 1] - s->box_items_off[b];
      if (n == 0 || s->boxes[b].n == 0) continue;
      A.only_box = (int32_t)b;
      A.items = s->d_box_items.as<int32_t>() + s->box_items_off[b];
      A.nitems = n;
      const unsigned grid = (unsigned)((n + s->waves - 1) / s->waves);
      HIPCHK(s, launch_forward(fp64, s->K, false, A, grid, block, st), "forward launch");
    }
  } else if (s->schedule == 1) {
    A.items = s->d_items.as<int32_t>();
    A.nitems = s->nitems_sorted;
    HIPCHK(s, launch_forward(fp64, s->K, true, A, persistent_grid(s), block, st),
           "forward launch");
  } else {
    const unsigned grid = (unsigned)((s->ntiles + s->waves - 1) / s->waves);
    HIPCHK(s, launch_forward(fp64, s->K, false, A, grid, block, st), "forward launch");
  }
  if (with_events) HIPCHK(s, hipEventRecord(s->ev[2], st), "event");
  return CSMAP_OK;
}

bool valid_pow_choice(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

size_t dtype_size(int dt) { return dt == CSMAP_F32 ? 4 : 8; }

}  // namespace

extern "C" {

int64_t csmap_npix(int64_t nside) {
  if (nside < 1 || nside > kMaxNside) return -1;
  return 12 * nside * nside;
}

const char* csmap_last_error(void) { return g_err.c_str(); }

csmap_status csmap_create_sky(int64_t nside, double eta0, csmap_form form, void* hip_stream,
                              csmap_sky** out) {
  g_err.clear();
  if (!out) return fail(CSMAP_E_INVALID, "out is NULL");
  *out = nullptr;
  if (nside < 1 || nside > kMaxNside)
    return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (!isfinite(eta0)) return fail(CSMAP_E_INVALID, "eta0 must be finite");
  if (form != CSMAP_FORM_FP64 && form != CSMAP_FORM_FP32C)
    return fail(CSMAP_E_INVALID, "unknown form");
  csmap_sky* s = new (std::nothrow) csmap_sky();
  if (!s) return fail(CSMAP_E_NOMEM, "host allocation failed");
  s->nside = nside;
  s->npix = 12 * nside * nside;
  s->eta0 = eta0;
  s->form = form;
  s->stream = (hipStream_t)hip_stream;
  s->chunk = (form == CSMAP_FORM_FP64) ? 64 : 32;
  // FP64: four pixels per lane, which the per-ring sharing of the z terms
  // makes pay (K = 2 without it was as fast as K = 4).
  if (form == CSMAP_FORM_FP64) s->K = 4;
  for (auto& e : s->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      csmap_destroy_sky(s);
      return dev_fail(nullptr, r, "event create");
    }
  }
  hipError_t r = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (r != hipSuccess) {
    csmap_destroy_sky(s);
    return dev_fail(nullptr, r, "stream create");
  }
  *out = s;
  return CSMAP_OK;
}

csmap_status csmap_destroy_sky(csmap_sky* s) {
  g_err.clear();
  if (!s) return CSMAP_OK;
  if (s->stream || s->cap_stream) (void)hipDeviceSynchronize();
  drop_graph(s);
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  DevBuf* bufs[] = {&s->raw, &s->d_boxes, &s->d_blk_box, &s->d_blk_count, &s->d_blk_prefix,
                    &s->d_blk_mask, &s->d_flat_off, &s->d_flat_rec, &s->d_udir, &s->d_flat_part,
                    &s->d_box_count, &s->d_raw_off, &s->d_rec32, &s->d_phat64, &s->d_rec64,
                    &s->d_orig, &s->d_tile_ptr, &s->d_tile_boxes, &s->d_items,
                    &s->d_box_items, &s->d_counters, &s->d_pixtab32, &s->d_pix64,
                    &s->d_partial, &s->d_adj_items, &s->d_adjc, &s->d_dir};
  for (DevBuf* b : bufs) b->release();
  delete s;
  return CSMAP_OK;
}

static csmap_status check_cone(const csmap_cone* c) {
  if (c->nside < 0 || c->nside > kMaxNside)
    return fail(CSMAP_E_INVALID, "cone nside must be in [0, 8192]");
  if (c->nside > 0 && (c->pix < 0 || c->pix >= 12 * c->nside * c->nside))
    return fail(CSMAP_E_INVALID, "cone pix must be in [0, 12 nside^2)");
  for (int k = 0; k < 9; ++k)
    if (!isfinite(c->rot[k])) return fail(CSMAP_E_INVALID, "rot must be finite");
  const double* m = c->rot;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double g = m[i] * m[j] + m[3 + i] * m[3 + j] + m[6 + i] * m[6 + j];
      if (fabs(g - (i == j ? 1.0 : 0.0)) > 1e-9)
        return fail(CSMAP_E_INVALID, "rot must be orthonormal");
    }
  const double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                     m[2] * (m[3] * m[7] - m[4] * m[6]);
  if (!(det > 0.0)) return fail(CSMAP_E_INVALID, "rot must be a proper rotation (det +1)");
  return CSMAP_OK;
}

static csmap_status add_box_impl(csmap_sky* s, const csmap_box* box, int snapshot,
                                 const csmap_cone* cone, int64_t* box_id) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!box) return fail(CSMAP_E_INVALID, "box is NULL");
  if (snapshot && box->vis == CSMAP_VIS_BOX)
    return fail(CSMAP_E_UNSUPPORTED,
                "CSMAP_VIS_BOX is not provided for snapshot boxes (their events leave the box)");
  if (cone && box->vis == CSMAP_VIS_BOX)
    return fail(CSMAP_E_UNSUPPORTED,
                "CSMAP_VIS_BOX is not provided for cone boxes (the rule's box is axis-aligned)");
  if (cone) {
    cs = check_cone(cone);
    if (cs != CSMAP_OK) return cs;
  }
  if (box->n < 0) return fail(CSMAP_E_INVALID, "segment count must be >= 0");
  if (box->n > (int64_t)INT32_MAX) return fail(CSMAP_E_INVALID, "at most 2^31-1 segments per box");
  if (box->dtype != CSMAP_F32 && box->dtype != CSMAP_F64)
    return fail(CSMAP_E_INVALID, "unknown dtype");
  if (box->n > 0 && (!box->x_rel || !box->xdot || !box->xprime || !box->dsigma))
    return fail(CSMAP_E_INVALID, "segment array pointer is NULL");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(box->origin[k]) || !isfinite(box->ext[k]))
      return fail(CSMAP_E_INVALID, "origin and ext must be finite");
  if (!isfinite(box->eta_lo) || !isfinite(box->eta_hi) || !(box->eta_lo < box->eta_hi))
    return fail(CSMAP_E_INVALID, "slab must satisfy eta_lo < eta_hi (finite)");
  if (box->vis != CSMAP_VIS_ALL && box->vis != CSMAP_VIS_BOX && box->vis != CSMAP_VIS_CAP)
    return fail(CSMAP_E_INVALID, "unknown visibility rule");
  if (box->vis == CSMAP_VIS_BOX)
    for (int k = 0; k < 3; ++k)
      if (!(box->ext[k] > 0.0)) return fail(CSMAP_E_INVALID, "ext must be > 0 for CSMAP_VIS_BOX");
  if (box->vis == CSMAP_VIS_CAP) {
    const double nn = box->cap_dir[0] * box->cap_dir[0] + box->cap_dir[1] * box->cap_dir[1] +
                      box->cap_dir[2] * box->cap_dir[2];
    if (!(fabs(nn - 1.0) < 1e-9)) return fail(CSMAP_E_INVALID, "cap_dir must be a unit vector");
    if (!(box->cap_cos >= -1.0 && box->cap_cos <= 1.0))
      return fail(CSMAP_E_INVALID, "cap_cos must be in [-1, 1]");
  }
  const size_t es = dtype_size(box->dtype);
  const size_t nbytes = es * 10 * (size_t)box->n;
  // Grow raw storage (geometrically), preserving what is there.
  const size_t need = s->raw_used + ((nbytes + 255) & ~(size_t)255);
  if (need > s->raw.cap) {
    size_t want = std::max(need, s->raw.cap + s->raw.cap / 2);
    void* np = nullptr;
    hipError_t e = hipMalloc(&np, want);
    if (e != hipSuccess) return fail(CSMAP_E_NOMEM, "device allocation of segment storage failed");
    if (s->raw_used) {
      HIPCHK(s, hipMemcpyAsync(np, s->raw.p, s->raw_used, hipMemcpyDeviceToDevice, s->stream),
             "grow storage");
      HIPCHK(s, hipStreamSynchronize(s->stream), "grow storage");
    }
    if (s->raw.p) (void)hipFree(s->raw.p);
    s->raw.p = np;
    s->raw.cap = want;
  }
  char* dst = (char*)s->raw.p + s->raw_used;
  const size_t n3 = es * 3 * (size_t)box->n;
  if (box->n > 0) {
    HIPCHK(s, hipMemcpyAsync(dst, box->x_rel, n3, hipMemcpyDefault, s->stream), "copy x_rel");
    HIPCHK(s, hipMemcpyAsync(dst + n3, box->xdot, n3, hipMemcpyDefault, s->stream), "copy xdot");
    HIPCHK(s, hipMemcpyAsync(dst + 2 * n3, box->xprime, n3, hipMemcpyDefault, s->stream),
           "copy xprime");
    HIPCHK(s, hipMemcpyAsync(dst + 3 * n3, box->dsigma, es * (size_t)box->n, hipMemcpyDefault,
                             s->stream), "copy dsigma");
  }
  HostBox h;
  h.snapshot = snapshot;
  if (cone) {
    h.rotated = 1;
    h.cone_nside = cone->nside;
    h.cone_pix = cone->pix;
    for (int k = 0; k < 9; ++k) h.rot[k] = cone->rot[k];
    if (cone->nside > 0) {
      cone_caps(cone->nside, cone->pix, h.cone_dir, h.cone_cos_out, h.cone_cos_in);
      cone_edges(cone->nside, cone->pix, h.cone_edge);
    }
  }
  for (int k = 0; k < 3; ++k) {
    h.geom.origin[k] = box->origin[k];
    h.geom.ext[k] = box->ext[k];
    h.geom.cap_dir[k] = box->cap_dir[k];
  }
  h.geom.eta_lo = box->eta_lo;
  h.geom.eta_hi = box->eta_hi;
  h.geom.vis = (int)box->vis;
  h.geom.cap_cos = box->cap_cos;
  h.dtype = (int)box->dtype;
  h.n = box->n;
  h.raw_byte_off = (int64_t)s->raw_used;
  s->raw_used = need;
  s->boxes.push_back(h);
  s->total_seg += box->n;
  s->dirty = true;
  s->version++;
  if (box_id) *box_id = (int64_t)s->boxes.size() - 1;
  return CSMAP_OK;
}

csmap_status csmap_add_box(csmap_sky* s, const csmap_box* box, int64_t* box_id) {
  return add_box_impl(s, box, 0, nullptr, box_id);
}

csmap_status csmap_add_snapshot_box(csmap_sky* s, const csmap_box* box, int64_t* box_id) {
  return add_box_impl(s, box, 1, nullptr, box_id);
}

csmap_status csmap_add_cone_box(csmap_sky* s, const csmap_box* box, const csmap_cone* cone,
                                int snapshot, int64_t* box_id) {
  g_err.clear();
  if (!cone) return fail(CSMAP_E_INVALID, "cone is NULL");
  if (snapshot != 0 && snapshot != 1) return fail(CSMAP_E_INVALID, "snapshot must be 0 or 1");
  return add_box_impl(s, box, snapshot, cone, box_id);
}

csmap_status csmap_precompute(csmap_sky* s) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  cs = prepare(s);
  if (cs != CSMAP_OK) return cs;
  hipStream_t st = s->stream;
  const PreArgs P = pre_args(s);
  HIPCHK(s, hipEventRecord(s->ev[0], st), "event");
  HIPCHK(s, launch_precompute(P, (int64_t)s->boxes.size(), st), "precompute launch");
  HIPCHK(s, launch_zero_counters(s->d_counters.as<unsigned long long>(), 5,
                                 (uint32_t*)(s->d_counters.as<unsigned long long>() + 2), st),
         "counter reset");
  HIPCHK(s, hipEventRecord(s->ev[1], st), "event");
  HIPCHK(s, hipEventRecord(s->ev[2], st), "event");
  s->timed_graph = false;
  s->have_fwd_time = true;
  return CSMAP_OK;
}

csmap_status csmap_ang2pix_ring(int64_t nside, int64_t n, const double* xyz, int64_t* pix,
                                void* hip_stream) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (n < 0) return fail(CSMAP_E_INVALID, "n must be >= 0");
  if (n > 0 && (!xyz || !pix)) return fail(CSMAP_E_INVALID, "xyz or pix is NULL");
  hipError_t e = launch_ang2pix(nside, n, xyz, pix, (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(nullptr, e, "ang2pix launch");
  return CSMAP_OK;
}

static csmap_status check_shell(double r_in, double r_out, double side) {
  if (!isfinite(r_in) || !isfinite(r_out) || !isfinite(side) || !(r_in > 0.0) ||
      !(r_in < r_out) || !(side > 0.0))
    return fail(CSMAP_E_INVALID, "need finite 0 < r_in < r_out and side > 0");
  return CSMAP_OK;
}

csmap_status csmap_cone_place(int64_t nside, int64_t pix, int axis, double r_in, double r_out,
                              double side, csmap_cone* cone, double origin[3], double* slack) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (pix < 0 || pix >= 12 * nside * nside)
    return fail(CSMAP_E_INVALID, "pix must be in [0, 12 nside^2)");
  if (axis < 0 || axis > 2) return fail(CSMAP_E_INVALID, "axis must be 0, 1 or 2");
  csmap_status cs = check_shell(r_in, r_out, side);
  if (cs != CSMAP_OK) return cs;
  if (!cone || !origin || !slack) return fail(CSMAP_E_INVALID, "output pointer is NULL");
  ConePlacement pl;
  cone_place(nside, pix, axis, r_in, r_out, side, pl);
  cone->nside = nside;
  cone->pix = pix;
  for (int k = 0; k < 9; ++k) cone->rot[k] = pl.rot[k];
  for (int k = 0; k < 3; ++k) origin[k] = pl.origin[k];
  *slack = pl.slack;
  return CSMAP_OK;
}

csmap_status csmap_cone_min_nside(double r_in, double r_out, double side, int64_t* nside) {
  g_err.clear();
  csmap_status cs = check_shell(r_in, r_out, side);
  if (cs != CSMAP_OK) return cs;
  if (!nside) return fail(CSMAP_E_INVALID, "nside is NULL");
  *nside = 0;
  // No cone fits once its depth alone exceeds the box.
  if (side < r_out - r_in) return CSMAP_OK;
  for (int64_t n = 1; n <= 256; n *= 2)
    if (cone_grid_slack(n, r_in, r_out, side) >= 0.0) {
      *nside = n;
      break;
    }
  return CSMAP_OK;
}

// The current device's stream-ordered pool for map2alm's scratch, created on
// first use.  Its release threshold is unbounded, so memory a call frees
// (in stream order) stays in the pool and the next call of the same or a
// smaller size takes it without a device allocation.
static hipError_t map2alm_pool(hipMemPool_t* out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!pools[dev]) {
    hipMemPoolProps props;
    memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t p = nullptr;
    e = hipMemPoolCreate(&p, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = UINT64_MAX;
    e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(p);
      return e;
    }
    pools[dev] = p;
  }
  *out = pools[dev];
  return hipSuccess;
}

csmap_status csmap_map2alm(int64_t nside, int64_t lmax, const double* map, double* alm,
                           void* hip_stream) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (lmax < 0 || lmax > 4 * nside) return fail(CSMAP_E_INVALID, "lmax must be in [0, 4 Nside]");
  if (!map || !alm) return fail(CSMAP_E_INVALID, "map or alm is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  hipMemPool_t pool = nullptr;
  hipError_t e = map2alm_pool(&pool);
  if (e != hipSuccess) return dev_fail(nullptr, e, "map2alm scratch pool");
  void* scratch = nullptr;
  e = hipMallocFromPoolAsync(&scratch, map2alm_scratch_bytes(nside, lmax), pool, st);
  if (e != hipSuccess || !scratch)
    return fail(CSMAP_E_NOMEM, "device allocation of map2alm scratch failed");
  e = launch_map2alm(nside, lmax, map, alm, scratch, st);
  const hipError_t e2 = hipFreeAsync(scratch, st);
  if (e != hipSuccess) return dev_fail(nullptr, e, "map2alm launch");
  if (e2 != hipSuccess) return dev_fail(nullptr, e2, "map2alm scratch release");
  return CSMAP_OK;
}

csmap_status csmap_map2alm_noalloc(int64_t nside, int64_t lmax, const double* map, double* alm,
                                   void* hip_stream) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (lmax < 0 || lmax > 4 * nside) return fail(CSMAP_E_INVALID, "lmax must be in [0, 4 Nside]");
  if (!map || !alm) return fail(CSMAP_E_INVALID, "map or alm is NULL");
  const size_t need = map2alm_scratch_bytes(nside, lmax);
  if (need > map2alm_noalloc_max_bytes())
    return fail(CSMAP_E_INVALID, "map2alm_noalloc: Nside " + std::to_string(nside) + ", lmax " +
                                     std::to_string(lmax) + " needs " + std::to_string(need) +
                                     " bytes of scratch; the fixed scratch holds " +
                                     std::to_string(map2alm_noalloc_max_bytes()));
  void* scratch = nullptr;
  hipError_t e = map2alm_noalloc_scratch(&scratch);
  if (e != hipSuccess) return dev_fail(nullptr, e, "map2alm_noalloc scratch address");
  e = launch_map2alm(nside, lmax, map, alm, scratch, (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(nullptr, e, "map2alm_noalloc launch");
  return CSMAP_OK;
}

csmap_status csmap_valu_probe(int kind, int64_t blocks, int64_t iters, void* out,
                              void* hip_stream, double* ms, double* fma_insts) {
  g_err.clear();
  if (kind < 0 || kind > 2) return fail(CSMAP_E_INVALID, "kind must be 0, 1 or 2");
  if (blocks < 1 || blocks > (int64_t)1 << 24 || iters < 1 || iters > (int64_t)1 << 30)
    return fail(CSMAP_E_INVALID, "need 1 <= blocks <= 2^24 and 1 <= iters <= 2^30");
  if (!out) return fail(CSMAP_E_INVALID, "out is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = launch_valu_probe(kind, blocks, iters, out, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return dev_fail(nullptr, e, "valu probe");
  if (ms) *ms = t;
  if (fma_insts) *fma_insts = (double)blocks * 4.0 * (double)iters * (double)valu_probe_chains();
  return CSMAP_OK;
}

csmap_status csmap_alm2cl(int64_t lmax, const double* alm, double* cl, void* hip_stream) {
  g_err.clear();
  if (lmax < 0 || lmax > 4 * kMaxNside) return fail(CSMAP_E_INVALID, "lmax out of range");
  if (!alm || !cl) return fail(CSMAP_E_INVALID, "alm or cl is NULL");
  hipError_t e = launch_alm2cl(lmax, alm, cl, (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(nullptr, e, "alm2cl launch");
  return CSMAP_OK;
}

csmap_status csmap_cone_events(const csmap_box* box, double eta0, double* pos, double* delta,
                               uint8_t* keep, void* hip_stream) {
  g_err.clear();
  if (!box) return fail(CSMAP_E_INVALID, "box is NULL");
  if (box->n < 0) return fail(CSMAP_E_INVALID, "segment count must be >= 0");
  if (box->dtype != CSMAP_F32 && box->dtype != CSMAP_F64)
    return fail(CSMAP_E_INVALID, "unknown dtype");
  if (box->n > 0 && (!box->x_rel || !box->xdot || !pos || !delta || !keep))
    return fail(CSMAP_E_INVALID, "array pointer is NULL");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(box->origin[k])) return fail(CSMAP_E_INVALID, "origin must be finite");
  if (!isfinite(eta0) || !isfinite(box->eta_lo) || !isfinite(box->eta_hi) ||
      !(box->eta_lo < box->eta_hi))
    return fail(CSMAP_E_INVALID, "eta0 and the slab must be finite with eta_lo < eta_hi");
  hipError_t e = launch_cone_events(box->n, (int)box->dtype, box->x_rel, box->xdot, box->origin,
                                    eta0, box->eta_lo, box->eta_hi, pos, delta, keep,
                                    (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(nullptr, e, "cone events launch");
  return CSMAP_OK;
}

csmap_status csmap_reset(csmap_sky* s) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  HIPCHK(s, hipStreamSynchronize(s->stream), "reset");
  s->boxes.clear();
  s->raw_used = 0;
  s->total_seg = 0;
  s->dirty = true;
  s->version++;
  drop_graph(s);
  return CSMAP_OK;
}

csmap_status csmap_set_option(csmap_sky* s, csmap_option opt, double value) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!isfinite(value)) return fail(CSMAP_E_INVALID, "option value must be finite");
  const int iv = (int)lround(value);
  switch (opt) {
    case CSMAP_OPT_SCHEDULE:
      if (iv < 0 || iv > 2) return fail(CSMAP_E_INVALID, "schedule must be 0, 1 or 2");
      s->schedule = iv;
      break;
    case CSMAP_OPT_GRAPH:
      if (iv < 0 || iv > 1) return fail(CSMAP_E_INVALID, "graph must be 0 or 1");
      s->graph = iv;
      break;
    case CSMAP_OPT_PIX_PER_LANE:
      if (!valid_pow_choice(iv)) return fail(CSMAP_E_INVALID, "pixels per lane must be 1, 2, 4 or 8");
      s->K = iv;
      break;
    case CSMAP_OPT_WAVES:
      if (iv != 1 && iv != 2 && iv != 4) return fail(CSMAP_E_INVALID, "waves must be 1, 2 or 4");
      s->waves = iv;
      break;
    case CSMAP_OPT_NEAR_W:
      if (!(value >= 1e-6)) return fail(CSMAP_E_INVALID, "near threshold must be >= 1e-6");
      s->near_w = value;
      break;
    case CSMAP_OPT_FAR_W:
      if (!(value >= 1e-6)) return fail(CSMAP_E_INVALID, "far threshold must be >= 1e-6");
      s->far_w = value;
      break;
    case CSMAP_OPT_ACCUM:
      if (iv < 0 || iv > 1) return fail(CSMAP_E_INVALID, "accumulation mode must be 0 or 1");
      s->frac = iv;
      break;
    case CSMAP_OPT_CHUNK:
      if (iv < 8 || iv > 4096 || (iv & 3))
        return fail(CSMAP_E_INVALID, "chunk must be a multiple of 4 in [8, 4096]");
      s->chunk = iv;
      break;
    case CSMAP_OPT_ADJ_SPLIT:
      if (iv < 0 || iv > 4096) return fail(CSMAP_E_INVALID, "split must be in [0, 4096]");
      s->adj_split = iv;
      break;
    case CSMAP_OPT_TILING:
      if (iv < 0 || iv > 2) return fail(CSMAP_E_INVALID, "tiling must be 0, 1 or 2");
      s->tiling = iv;
      break;
    case CSMAP_OPT_BLOCK_RINGS:
      if (iv != 0 && (iv < 1 || iv > 64 || (iv & (iv - 1))))
        return fail(CSMAP_E_INVALID, "rings per block must be 0 or a power of two in [1, 64]");
      s->block_rings = iv;
      break;
    default:
      return fail(CSMAP_E_INVALID, "unknown option");
  }
  s->version++;
  drop_graph(s);
  return CSMAP_OK;
}

csmap_status csmap_render(csmap_sky* s, double* map) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!map) return fail(CSMAP_E_INVALID, "map is NULL");
  cs = prepare(s);
  if (cs != CSMAP_OK) return cs;
  if (s->graph) {
    if (!s->graph_exec || s->graph_map != map || s->graph_version != s->version) {
      drop_graph(s);
      HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal),
             "begin capture");
      cs = enqueue_render(s, map, s->cap_stream, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
      if (cs != CSMAP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return cs;
      }
      if (e != hipSuccess) return dev_fail(s, e, "end capture");
      s->graph_h = g;
      HIPCHK(s, hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0), "instantiate graph");
      s->graph_map = map;
      s->graph_version = s->version;
    }
    HIPCHK(s, hipEventRecord(s->ev[0], s->stream), "event");
    HIPCHK(s, hipGraphLaunch(s->graph_exec, s->stream), "graph launch");
    HIPCHK(s, hipEventRecord(s->ev[2], s->stream), "event");
    s->timed_graph = true;
  } else {
    cs = enqueue_render(s, map, s->stream, true);
    if (cs != CSMAP_OK) return cs;
    s->timed_graph = false;
  }
  s->have_fwd_time = true;
  return CSMAP_OK;
}

static bool unit3(const double* v) {
  for (int k = 0; k < 3; ++k)
    if (!isfinite(v[k])) return false;
  return fabs(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - 1.0) < 1e-9;
}

static double dot3h(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

csmap_status csmap_render_flat(csmap_sky* s, const csmap_patch* patch, double* map) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!patch || !map) return fail(CSMAP_E_INVALID, "patch or map is NULL");
  const csmap_patch& P = *patch;
  if (!unit3(P.center) || !unit3(P.e1) || !unit3(P.e2))
    return fail(CSMAP_E_INVALID, "center, e1 and e2 must be unit vectors");
  if (fabs(dot3h(P.center, P.e1)) > 1e-9 || fabs(dot3h(P.center, P.e2)) > 1e-9 ||
      fabs(dot3h(P.e1, P.e2)) > 1e-9)
    return fail(CSMAP_E_INVALID, "center, e1 and e2 must be orthogonal");
  if (P.nx < 1 || P.ny < 1 || P.nx > (int64_t)1 << 31 || P.ny > (int64_t)1 << 31 ||
      P.nx * P.ny > (int64_t)1 << 31)
    return fail(CSMAP_E_INVALID, "need nx, ny >= 1 and nx * ny <= 2^31");
  if (!isfinite(P.pix) || !(P.pix > 0.0)) return fail(CSMAP_E_INVALID, "pix must be > 0");
  if (!(P.accept_cos > 0.0 && P.accept_cos <= 1.0))
    return fail(CSMAP_E_INVALID, "accept_cos must be in (0, 1]");
  // An accepted segment has |e.P|/D < tan(rho), so its plane position in
  // pixel units is below tan(rho)/pix + n/2, every pixel-segment offset below
  // tan(rho)/pix + n, and with that bound at 2^30 the pair kernel's product
  // of two squared distances stays below 4 (2^30)^4 = 2^122, inside the range
  // of its reciprocal ([2^-125, 2^125]).
  {
    const double c = P.accept_cos;
    const double tan_rho = sqrt((1.0 - c) * (1.0 + c)) / c;
    const double nmax = (double)std::max(P.nx, P.ny);
    if (!(tan_rho / P.pix + nmax <= 1073741824.0))
      return fail(CSMAP_E_INVALID,
                  "acceptance cone too wide for the pixel size: need "
                  "tan(acos(accept_cos))/pix + max(nx, ny) <= 2^30");
  }
  cs = prepare(s);
  if (cs != CSMAP_OK) return cs;
  const int64_t nbox = (int64_t)s->boxes.size();
  hipStream_t st = s->stream;
  HIPCHK(s, s->d_flat_off.ensure(sizeof(int64_t) * (nbox + 1)), "alloc flat offsets");
  HIPCHK(s, s->d_flat_rec.ensure(sizeof(float) * kFlatRec * (size_t)(s->total_seg + 2)),
         "alloc flat records");
  PreArgs pa = pre_args(s);
  pa.flat_on = 1;
  for (int k = 0; k < 3; ++k) pa.flat_dir[k] = P.center[k];
  pa.flat_cos = P.accept_cos;
  FlatArgs A;
  memset(&A, 0, sizeof(A));
  A.boxes = s->d_boxes.as<DevBox>();
  A.box_count = s->d_box_count.as<DevBoxCount>();
  A.blk_box = s->d_blk_box.as<int32_t>();
  A.nblk = s->nblk;
  A.nbox = nbox;
  A.raw = s->raw.p;
  A.raw_byte_off = s->d_raw_off.as<int64_t>();
  A.orig_index = s->d_orig.as<int32_t>();
  A.eta0 = s->eta0;
  for (int k = 0; k < 3; ++k) {
    A.c[k] = P.center[k];
    A.e1[k] = P.e1[k];
    A.e2[k] = P.e2[k];
  }
  A.inv_h = 1.0 / P.pix;
  A.off_x = 0.5 * (double)P.nx - 0.5;
  A.off_y = 0.5 * (double)P.ny - 0.5;
  A.nx = P.nx;
  A.ny = P.ny;
  A.flat_off = s->d_flat_off.as<int64_t>();
  A.rec = s->d_flat_rec.as<float>();
  A.map = map;
  HIPCHK(s, hipEventRecord(s->ev[0], st), "event");
  HIPCHK(s, launch_precompute(pa, nbox, st), "precompute launch");
  HIPCHK(s, launch_flat(A, st), "flat record launch");
  HIPCHK(s, hipEventRecord(s->ev[1], st), "event");
  const int64_t nsplit = flat_splits(P.nx, P.ny);
  if (nsplit > 1)
    HIPCHK(s, s->d_flat_part.ensure(sizeof(double) * (size_t)nsplit * (size_t)(P.nx * P.ny)),
           "alloc flat partial maps");
  HIPCHK(s, launch_flat_pairs(A, nsplit, s->d_flat_part.as<double>(), st), "flat pair launch");
  HIPCHK(s, hipEventRecord(s->ev[2], st), "event");
  s->timed_graph = false;
  s->have_fwd_time = true;
  return CSMAP_OK;
}

csmap_status csmap_render_dirs(csmap_sky* s, int64_t n, const double* xyz, double* out) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(CSMAP_E_INVALID, "n must be in [0, 2^31]");
  if (n > 0 && (!xyz || !out)) return fail(CSMAP_E_INVALID, "xyz or out is NULL");
  cs = prepare(s);
  if (cs != CSMAP_OK) return cs;
  hipStream_t st = s->stream;
  HIPCHK(s, s->d_udir.ensure(sizeof(double) * 3 * (size_t)std::max<int64_t>(n, 1)),
         "alloc direction table");
  double* d = s->d_udir.as<double>();
  const PreArgs P = pre_args(s);
  FwdArgs A = fwd_args(s, out);
  // Strips of 64 K directions in the caller's order; every tile walks every
  // box, and the per-pixel visibility test of the kernels applies each
  // box's rule to each direction.
  const int64_t tile_px = 64 * (int64_t)s->K;
  const int64_t ntiles = (n + tile_px - 1) / tile_px;
  A.all_boxes = 1;
  A.rows = nullptr;
  A.ring_g = 1;
  A.ring_shift = 6;
  A.items = nullptr;
  A.nitems = ntiles;
  A.nside = 0;
  A.npix = n;
  A.dirx = d;
  A.diry = d + n;
  A.dirz = d + 2 * n;
  HIPCHK(s, launch_dirs_soa(n, xyz, d, d + n, d + 2 * n, st), "direction launch");
  HIPCHK(s, hipEventRecord(s->ev[0], st), "event");
  HIPCHK(s, launch_precompute(P, (int64_t)s->boxes.size(), st), "precompute launch");
  HIPCHK(s, launch_zero_counters(s->d_counters.as<unsigned long long>(), 5,
                                 (uint32_t*)(s->d_counters.as<unsigned long long>() + 2), st),
         "counter reset");
  HIPCHK(s, hipEventRecord(s->ev[1], st), "event");
  if (ntiles > 0) {
    const unsigned block = 64u * (unsigned)s->waves;
    const unsigned grid = (unsigned)((ntiles + s->waves - 1) / s->waves);
    HIPCHK(s, launch_forward(s->form == CSMAP_FORM_FP64, s->K, false, A, grid, block, st),
           "forward launch");
  }
  HIPCHK(s, hipEventRecord(s->ev[2], st), "event");
  s->timed_graph = false;
  s->have_fwd_time = true;
  return CSMAP_OK;
}

csmap_status csmap_backward(csmap_sky* s, const double* dmap, const csmap_grad* grads,
                            int64_t nbox) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!dmap) return fail(CSMAP_E_INVALID, "dmap is NULL");
  if (nbox != (int64_t)s->boxes.size())
    return fail(CSMAP_E_INVALID, "nbox must equal the number of boxes");
  if (nbox > 0 && !grads) return fail(CSMAP_E_INVALID, "grads is NULL");
  if (s->form != CSMAP_FORM_FP32C)
    return fail(CSMAP_E_UNSUPPORTED, "backward is provided for the FP32C form");
  for (auto& h : s->boxes)
    if (h.snapshot)
      return fail(CSMAP_E_UNSUPPORTED, "backward is not provided for snapshot boxes");
  cs = prepare(s);
  if (cs != CSMAP_OK) return cs;
  hipStream_t st = s->stream;
  HIPCHK(s, hipEventRecord(s->ev[3], st), "event");
  HIPCHK(s, s->d_adjc.ensure(sizeof(float) * 4 * (size_t)std::max<int64_t>(1, s->total_seg)),
         "alloc adjoint constants");
  PreArgs P = pre_args(s);
  P.adjc = s->d_adjc.as<float>();
  HIPCHK(s, launch_precompute(P, nbox, st), "precompute launch");
  // Kept counts decide the work items.
  std::vector<DevBoxCount> kc(std::max<int64_t>(nbox, 1));
  if (nbox)
    HIPCHK(s, hipMemcpyAsync(kc.data(), s->d_box_count.p, sizeof(DevBoxCount) * nbox,
                             hipMemcpyDeviceToHost, st), "read counts");
  HIPCHK(s, hipStreamSynchronize(st), "read counts");
  int64_t groups = 0;
  for (int64_t b = 0; b < nbox; ++b) groups += (kc[b].kept + 63) / 64;
  int nsplit = s->adj_split;
  if (nsplit <= 0) {
    const int64_t target = 16384;  // work items wanted to fill the device
    nsplit = (int)std::min<int64_t>(256, std::max<int64_t>(1, (target + std::max<int64_t>(groups, 1) - 1) /
                                                                std::max<int64_t>(groups, 1)));
    nsplit = (int)std::min<int64_t>(nsplit, std::max<int64_t>(1, s->npix / 64));
  }
  std::vector<int32_t> items;
  items.reserve(3 * groups * nsplit);
  for (int64_t b = 0; b < nbox; ++b)
    for (int64_t g = 0; g < (kc[b].kept + 63) / 64; ++g)
      for (int sp = 0; sp < nsplit; ++sp) {
        items.push_back((int32_t)b);
        items.push_back((int32_t)g);
        items.push_back(sp);
      }
  const int64_t nitems = (int64_t)items.size() / 3;
  HIPCHK(s, s->d_pixtab32.ensure(sizeof(float) * 4 * (s->npix + 1)), "alloc pixel table");
  HIPCHK(s, s->d_pix64.ensure(sizeof(double) * 4 * s->npix), "alloc pixel table");
  HIPCHK(s, s->d_partial.ensure(sizeof(double) * 14 * (size_t)std::max<int64_t>(1, s->total_seg) *
                                nsplit), "alloc partials");
  HIPCHK(s, s->d_adj_items.ensure(sizeof(int32_t) * std::max<size_t>(items.size(), 1)),
         "alloc items");
  if (!items.empty())
    HIPCHK(s, hipMemcpyAsync(s->d_adj_items.p, items.data(), sizeof(int32_t) * items.size(),
                             hipMemcpyHostToDevice, st), "upload items");
  HIPCHK(s, launch_pixtab(s->nside, s->npix, dmap, s->d_pixtab32.as<float>(),
                          s->d_pix64.as<double>(), st), "pixel table");
  for (int64_t b = 0; b < nbox; ++b) {
    const int64_t n = s->boxes[b].n;
    if (grads[b].x_rel) HIPCHK(s, launch_fill(grads[b].x_rel, 3 * n, 0.0, st), "grad clear");
    if (grads[b].xdot) HIPCHK(s, launch_fill(grads[b].xdot, 3 * n, 0.0, st), "grad clear");
    if (grads[b].xprime) HIPCHK(s, launch_fill(grads[b].xprime, 3 * n, 0.0, st), "grad clear");
    if (grads[b].dsigma) HIPCHK(s, launch_fill(grads[b].dsigma, n, 0.0, st), "grad clear");
  }
  AdjArgs A;
  memset(&A, 0, sizeof(A));
  A.boxes = s->d_boxes.as<DevBox>();
  A.box_count = s->d_box_count.as<DevBoxCount>();
  A.nbox = (int32_t)nbox;
  A.nside = s->nside;
  A.npix = s->npix;
  A.eta0 = s->eta0;
  A.pixtab = s->d_pixtab32.as<float>();
  A.pix64 = s->d_pix64.as<double>();
  A.rec32 = s->d_rec32.as<float>();
  A.phat64 = s->d_phat64.as<double>();
  A.adjc = s->d_adjc.as<float>();
  A.items = s->d_adj_items.as<int32_t>();
  A.nitems = nitems;
  A.nsplit = nsplit;
  A.near_w = (float)s->near_w;
  A.far_w = (float)std::max(s->far_w, s->near_w);
  A.partial = s->d_partial.as<double>();
  A.dmap = dmap;
  HIPCHK(s, hipEventRecord(s->ev[4], st), "event");
  HIPCHK(s, launch_adjoint(A, st), "adjoint launch");
  HIPCHK(s, hipEventRecord(s->ev[5], st), "event");
  for (int64_t b = 0; b < nbox; ++b) {
    HIPCHK(s, launch_adj_finalize(s->d_boxes.as<DevBox>(), s->d_box_count.as<DevBoxCount>(),
                                  (int32_t)b, kc[b].kept,
                                  (const char*)s->raw.p + s->boxes[b].raw_byte_off,
                                  s->d_orig.as<int32_t>(), s->d_phat64.as<double>(),
                                  s->d_partial.as<double>(), nsplit, grads[b].x_rel,
                                  grads[b].xdot, grads[b].xprime, grads[b].dsigma, st),
           "finalize launch");
  }
  // The item list lives in host memory until the copy has completed.
  HIPCHK(s, hipStreamSynchronize(st), "backward");
  s->have_bwd_time = true;
  return CSMAP_OK;
}

csmap_status csmap_get_stats(csmap_sky* s, csmap_stats* out) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  if (!out) return fail(CSMAP_E_INVALID, "out is NULL");
  memset(out, 0, sizeof(*out));
  HIPCHK(s, hipStreamSynchronize(s->stream), "sync");
  out->nside = s->nside;
  out->npix = s->npix;
  out->nbox = (int64_t)s->boxes.size();
  out->segments = s->total_seg;
  if (!s->dirty && s->d_counters.p) {
    unsigned long long c[5] = {0, 0, 0, 0, 0};
    HIPCHK(s, hipMemcpy(c, s->d_counters.p, sizeof(c), hipMemcpyDeviceToHost), "read counters");
    out->pairs = (int64_t)c[0];
    out->near_steps = (int64_t)c[1];
    out->mid_steps = (int64_t)c[3];
    out->steps = (int64_t)c[4];
    std::vector<DevBoxCount> kc(s->boxes.size());
    if (!kc.empty())
      HIPCHK(s, hipMemcpy(kc.data(), s->d_box_count.p, sizeof(DevBoxCount) * kc.size(),
                          hipMemcpyDeviceToHost), "read counts");
    for (auto& k : kc) out->kept += k.kept;
  }
  float ms = 0.f;
  if (s->have_fwd_time) {
    if (s->timed_graph) {
      HIPCHK(s, hipEventElapsedTime(&ms, s->ev[0], s->ev[2]), "elapsed");
      out->ms_forward = ms;
      out->ms_precompute = 0.0;
    } else {
      HIPCHK(s, hipEventElapsedTime(&ms, s->ev[0], s->ev[1]), "elapsed");
      out->ms_precompute = ms;
      HIPCHK(s, hipEventElapsedTime(&ms, s->ev[1], s->ev[2]), "elapsed");
      out->ms_forward = ms;
    }
  }
  if (s->have_bwd_time) {
    HIPCHK(s, hipEventElapsedTime(&ms, s->ev[4], s->ev[5]), "elapsed");
    out->ms_backward = ms;
  }
  out->pix_per_lane = s->K;
  out->waves = s->waves;
  out->schedule = s->schedule;
  out->graph = s->graph;
  out->chunk = s->chunk;
  out->near_w = s->near_w;
  out->far_w = s->far_w;
  out->tiling = use_blocks(s) ? 2 : 1;
  return CSMAP_OK;
}

csmap_status csmap_pix2vec_ring(int64_t nside, int64_t first, int64_t count, double* xyz,
                                void* hip_stream) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  const int64_t npix = 12 * nside * nside;
  if (first < 0 || count < 0 || first > npix || count > npix - first)
    return fail(CSMAP_E_INVALID, "pixel range outside the map");
  if (count > 0 && !xyz) return fail(CSMAP_E_INVALID, "xyz is NULL");
  hipError_t e = launch_pix2vec(nside, first, count, xyz, (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(nullptr, e, "pix2vec launch");
  return CSMAP_OK;
}

static csmap_status write_cap_ranges(const Tiling& t, double cx, double cy, double cz,
                                     double rho, int64_t* ranges, int64_t max_ranges,
                                     int64_t* n_ranges) {
  std::vector<std::pair<int64_t, int64_t>> out;
  cap_tiles(t, cx, cy, cz, rho, out);
  *n_ranges = (int64_t)out.size();
  if ((int64_t)out.size() > max_ranges) return fail(CSMAP_E_INVALID, "max_ranges too small");
  for (size_t i = 0; i < out.size(); ++i) {
    ranges[2 * i] = out[i].first;
    ranges[2 * i + 1] = out[i].second;
  }
  return CSMAP_OK;
}

csmap_status csmap_cap_tiles(int64_t nside, int64_t tile, double cx, double cy, double cz,
                             double rho, int64_t* ranges, int64_t max_ranges,
                             int64_t* n_ranges) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (tile < 1) return fail(CSMAP_E_INVALID, "tile must be >= 1");
  if (!n_ranges || (max_ranges > 0 && !ranges)) return fail(CSMAP_E_INVALID, "NULL output");
  if (!isfinite(cx) || !isfinite(cy) || !isfinite(cz) || !isfinite(rho) || rho < 0)
    return fail(CSMAP_E_INVALID, "cap must be finite with rho >= 0");
  Tiling t;
  make_strips(nside, tile, t);
  return write_cap_ranges(t, cx, cy, cz, rho, ranges, max_ranges, n_ranges);
}

csmap_status csmap_ring_block_rows(int64_t nside, int64_t rings, int64_t width, int64_t* rows,
                                   int64_t max_tiles, int64_t* n_tiles) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (rings < 1 || rings > 64) return fail(CSMAP_E_INVALID, "rings must be in [1, 64]");
  if (width < 1 || width >= (1 << kRowCountBits))
    return fail(CSMAP_E_INVALID, "width must be in [1, 1023]");
  if (!n_tiles || (max_tiles > 0 && !rows)) return fail(CSMAP_E_INVALID, "NULL output");
  Tiling t;
  make_ring_blocks(nside, (int)rings, width, t);
  *n_tiles = t.ntiles;
  if (t.ntiles > max_tiles) return fail(CSMAP_E_INVALID, "max_tiles too small");
  std::vector<int64_t> r;
  ring_block_rows(t, r);
  std::copy(r.begin(), r.end(), rows);
  return CSMAP_OK;
}

csmap_status csmap_cap_block_tiles(int64_t nside, int64_t rings, int64_t width, double cx,
                                   double cy, double cz, double rho, int64_t* ranges,
                                   int64_t max_ranges, int64_t* n_ranges) {
  g_err.clear();
  if (nside < 1 || nside > kMaxNside) return fail(CSMAP_E_INVALID, "nside must be in [1, 8192]");
  if (rings < 1 || rings > 64) return fail(CSMAP_E_INVALID, "rings must be in [1, 64]");
  if (width < 1 || width >= (1 << kRowCountBits))
    return fail(CSMAP_E_INVALID, "width must be in [1, 1023]");
  if (!n_ranges || (max_ranges > 0 && !ranges)) return fail(CSMAP_E_INVALID, "NULL output");
  if (!isfinite(cx) || !isfinite(cy) || !isfinite(cz) || !isfinite(rho) || rho < 0)
    return fail(CSMAP_E_INVALID, "cap must be finite with rho >= 0");
  Tiling t;
  make_ring_blocks(nside, (int)rings, width, t);
  return write_cap_ranges(t, cx, cy, cz, rho, ranges, max_ranges, n_ranges);
}

csmap_status csmap_autotune(csmap_sky* s, const char* cache_path) {
  g_err.clear();
  csmap_status cs = check_sky(s);
  if (cs != CSMAP_OK) return cs;
  const bool fp64 = s->form == CSMAP_FORM_FP64;
  const int64_t nbox = (int64_t)s->boxes.size();
  int dev = 0;
  HIPCHK(s, hipGetDevice(&dev), "device");
  hipDeviceProp_t prop;
  HIPCHK(s, hipGetDeviceProperties(&prop, dev), "device properties");
  // Workload key: device, form, Nside, box count, the number of boxes under
  // each visibility rule, the caps' summed sky fraction (two significant
  // digits), and the segment count rounded to a power of two.
  int nrule[3] = {0, 0, 0};
  double cap_frac = 0.0;
  for (auto& h : s->boxes) {
    nrule[std::min(std::max(h.geom.vis, 0), 2)]++;
    if (h.geom.vis == CSMAP_VIS_CAP) cap_frac += 0.5 * (1.0 - h.geom.cap_cos);
  }
  int seg_log2 = 0;
  while (((int64_t)1 << seg_log2) < std::max<int64_t>(1, s->total_seg)) ++seg_log2;
  char frac_txt[32];
  snprintf(frac_txt, sizeof(frac_txt), "%.2g", cap_frac);
  std::ostringstream key;
  key << prop.gcnArchName << "|" << (fp64 ? "fp64" : "fp32c") << "|" << s->nside << "|" << nbox
      << "|vis" << nrule[0] << "," << nrule[1] << "," << nrule[2] << "|caps" << frac_txt << "|"
      << seg_log2;
  struct Cand {
    int K, W, S, F, tiling, rings, chunk;
    double near_w, far_w;
  };
  auto apply = [&](const Cand& c) {
    s->K = c.K;
    s->waves = c.W;
    s->schedule = c.S;
    s->frac = c.F;
    s->tiling = c.tiling;
    s->block_rings = c.rings;
    s->chunk = c.chunk;
    s->near_w = c.near_w;
    s->far_w = c.far_w;
    s->have_fwd_time = false;
    s->version++;
    drop_graph(s);
  };
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      Cand c;
      if (ls >> k >> c.K >> c.W >> c.S >> c.F >> c.tiling >> c.rings >> c.chunk >> c.near_w >>
          c.far_w &&
          k == key.str()) {
        apply(c);
        return CSMAP_OK;
      }
    }
  }
  if (nbox == 0 || s->total_seg == 0) return CSMAP_OK;
  // Sample: tiles spread evenly over the tile order (which follows the
  // rings, so over the sky), about 25M pixels in all (enough to give every
  // resident wavefront many work items), each tile limited to its first
  // 2,048 segments per box so that every candidate measures steady-state
  // throughput.  Candidates are ranked by pairs per second, since tiles of
  // different shapes cover slightly different pixels.
  const int64_t sample_px = 49152 * 512;
  DevBuf scratch, items;
  HIPCHK(s, scratch.ensure(sizeof(double) * (size_t)s->npix), "alloc scratch map");
  const Cand saved = {s->K,     s->waves, s->schedule, s->frac,  s->tiling,
                      s->block_rings, s->chunk, s->near_w, s->far_w};
  hipStream_t st = s->stream;
  const bool log = getenv("CSMAP_TUNE_LOG") != nullptr;
  // Pairs per second of one candidate on the sample; -1 if the planner
  // rejects its shape (the candidate is skipped, not an error).
  auto measure = [&](const Cand& c, double* rate, int seg_cap) -> csmap_status {
    *rate = -1.0;
    apply(c);
    csmap_status r = prepare(s);
    if (r == CSMAP_E_INVALID) {   // a shape the planner does not admit
      g_err.clear();
      return CSMAP_OK;
    }
    if (r != CSMAP_OK) return r;
    const int64_t nsample = std::max<int64_t>(
        1, std::min<int64_t>(s->ntiles, sample_px / (64 * (int64_t)c.K)));
    std::vector<int32_t> it(nsample);
    for (int64_t i = 0; i < nsample; ++i) it[i] = (int32_t)(i * s->ntiles / nsample);
    HIPCHK(s, items.ensure(sizeof(int32_t) * it.size()), "alloc items");
    HIPCHK(s, hipMemcpy(items.p, it.data(), sizeof(int32_t) * it.size(), hipMemcpyHostToDevice),
           "upload items");
    const PreArgs P = pre_args(s);
    HIPCHK(s, launch_precompute(P, nbox, st), "precompute launch");
    FwdArgs A = fwd_args(s, scratch.as<double>());
    A.items = items.as<int32_t>();
    A.nitems = (int64_t)it.size();
    A.seg_cap = seg_cap;
    r = check_forward(s, A, c.K);
    if (r == CSMAP_E_INVALID) {
      g_err.clear();
      return CSMAP_OK;
    }
    if (r != CSMAP_OK) return r;
    const unsigned block = 64u * (unsigned)c.W;
    const unsigned grid = c.S ? persistent_grid(s) : (unsigned)((A.nitems + c.W - 1) / c.W);
    double ms_min = 1e300;
    unsigned long long ctr[5] = {0, 0, 0, 0, 0};
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(s, launch_zero_counters(s->d_counters.as<unsigned long long>(), 5, A.work_counter, st),
             "counter reset");
      HIPCHK(s, hipEventRecord(s->ev[0], st), "event");
      HIPCHK(s, launch_forward(fp64, c.K, c.S == 1, A, grid, block, st), "forward launch");
      HIPCHK(s, hipEventRecord(s->ev[1], st), "event");
      HIPCHK(s, hipEventSynchronize(s->ev[1]), "sync");
      float ms = 0.f;
      HIPCHK(s, hipEventElapsedTime(&ms, s->ev[0], s->ev[1]), "elapsed");
      if (rep > 0) ms_min = std::min(ms_min, (double)ms);
    }
    HIPCHK(s, hipMemcpy(ctr, s->d_counters.p, sizeof(ctr), hipMemcpyDeviceToHost),
           "read counters");
    *rate = (double)ctr[0] / std::max(ms_min, 1e-6) * 1e3;
    if (log)
      fprintf(stderr,
              "csmap_autotune: K=%d waves=%d accum=%d tiling=%d rings=%d chunk=%d near_w=%g "
              "far_w=%g items=%lld %.3f ms %.4g pairs/s (FP64 steps %llu, middle %llu of "
              "%llu)\n",
              c.K, c.W, c.F, c.tiling, c.rings, c.chunk, c.near_w, c.far_w, (long long)it.size(),
              ms_min, *rate, ctr[1], ctr[3], ctr[4]);
    return CSMAP_OK;
  };
  Cand best = saved;
  best.S = 1;
  if (best.tiling == 0) best.tiling = 2;
  double best_rate = -1.0;
  std::vector<std::pair<Cand, double>> tried;
  auto consider = [&](const Cand& c) -> csmap_status {
    double rate = -1.0;
    csmap_status r = measure(c, &rate, 2048);
    if (r != CSMAP_OK) return r;
    tried.push_back({c, rate});
    if (rate > best_rate) {
      best_rate = rate;
      best = c;
    }
    return CSMAP_OK;
  };
  // Stage 1: launch shape (pixels per lane, wavefronts per workgroup,
  // accumulation mode) with the persistent schedule, which was never slower
  // than one-tile-per-wavefront launches on uniform skies and bounds the
  // tail on uneven ones.
  {
    const Cand base = best;
    for (int K : {1, 2, 4, 8})
      for (int W : {1, 2, 4})
        for (int F : {0, 1}) {
          if (fp64 && F) continue;
          if (!fp64 && K == 1) continue;
          Cand c = base;
          c.K = K;
          c.W = W;
          c.F = F;
          c.rings = 0;
          cs = consider(c);
          if (cs != CSMAP_OK) break;
        }
  }
  // Stage 1b: the short sample (2,048 segments per box and tile) weighs a
  // tile's fixed costs more than a full render does, and shapes within a few
  // percent of each other on it have differed by 5% on a whole sky (pixels
  // per lane 4 against 8 on the uneven 256-box workload).  The shapes within
  // 3% of the best are measured again on 8,192 segments per box and tile,
  // and the best of that measurement is kept.
  if (cs == CSMAP_OK) {
    std::vector<Cand> close;
    for (auto& t : tried)
      if (t.second >= 0.97 * best_rate) close.push_back(t.first);
    if (close.size() > 1) {
      double r_best = -1.0;
      Cand c_best = best;
      for (const Cand& c : close) {
        double rate = -1.0;
        cs = measure(c, &rate, 8192);
        if (cs != CSMAP_OK) break;
        if (rate > r_best) {
          r_best = rate;
          c_best = c;
        }
      }
      if (cs == CSMAP_OK && r_best > 0.0) {
        // Later stages compare their short-sample rates with the chosen
        // shape's own.
        for (auto& t : tried) {
          const Cand& a = t.first;
          if (a.K == c_best.K && a.W == c_best.W && a.S == c_best.S && a.F == c_best.F &&
              a.tiling == c_best.tiling && a.rings == c_best.rings && a.chunk == c_best.chunk &&
              a.near_w == c_best.near_w && a.far_w == c_best.far_w)
            best_rate = t.second;
        }
        best = c_best;
      }
    }
  }
  // Stage 2: from the best shape, one parameter at a time: the tiling and
  // rings per ring-block tile, the FP32 partial-sum length
  // before each compensated update (FP32C; at most 64 terms), and the pair
  // form thresholds among those whose per-term error bound is no larger
  // than the defaults' (far form 6e-8/far_w, middle form 1e-7/sqrt(2 near_w):
  // far_w >= 5e-3, near_w >= 5e-5), so that tuning never trades accuracy.
  if (cs == CSMAP_OK) {
    const Cand base = best;
    std::vector<Cand> cands;
    Cand c = base;
    c.tiling = base.tiling == 1 ? 2 : 1;
    c.rings = 0;
    cands.push_back(c);
    for (int g : {base.K, 4 * base.K, 8 * base.K})
      if (g >= 1 && g <= 64 && g != 2 * base.K) {
        c = base;
        c.tiling = 2;
        c.rings = g;
        cands.push_back(c);
      }
    for (const Cand& cc : cands) {
      cs = consider(cc);
      if (cs != CSMAP_OK) break;
    }
  }
  if (cs == CSMAP_OK && !fp64) {
    const Cand base = best;
    for (int ch : {16, 64}) {
      Cand c = base;
      c.chunk = ch;
      cs = consider(c);
      if (cs != CSMAP_OK) break;
    }
  }
  if (cs == CSMAP_OK && !fp64) {
    const Cand base = best;
    for (double fw : {1e-2, 2e-2}) {
      Cand c = base;
      c.far_w = std::max(fw, base.far_w);
      if (c.far_w != base.far_w) {
        cs = consider(c);
        if (cs != CSMAP_OK) break;
      }
    }
    for (double nw : {1e-4, 2e-4}) {
      if (cs != CSMAP_OK) break;
      Cand c = best;
      c.near_w = std::max(nw, best.near_w);
      if (c.near_w != best.near_w) cs = consider(c);
    }
  }
  scratch.release();
  items.release();
  if (best_rate < 0.0) best = saved;
  apply(best);
  if (cs != CSMAP_OK) return cs;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out.precision(17);
    out << key.str() << " " << best.K << " " << best.W << " " << best.S << " " << best.F << " "
        << best.tiling << " " << best.rings << " " << best.chunk << " " << best.near_w << " "
        << best.far_w << "\n";
  }
  return CSMAP_OK;
}

}  // extern "C"
