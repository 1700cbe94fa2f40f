// sched.cpp -- host-side work planning: how pixels are cut into tiles and
// which tiles can see a box.
//
// For boxes that do not see the whole sky the kernels test every pixel
// exactly; this file only has to produce a superset of the tiles that
// contain a visible pixel, so every quantity here carries a margin.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "sched.h"

namespace csmap {

namespace {

struct RingInfo {
  int64_t first;   // RING index of the ring's first pixel
  int64_t len;     // pixels in the ring
  double z;        // cos(colatitude) of the ring
  double offset;   // azimuth of pixel 0 in units of the pixel spacing
};

// Ring i (1 .. 4 Nside - 1) of the HEALPix RING scheme.
RingInfo ring_info(int64_t nside, int64_t i) {
  const int64_t N = nside;
  RingInfo r;
  if (i < N) {
    r.len = 4 * i;
    r.first = 2 * i * (i - 1);
    r.z = 1.0 - (double)(i * i) / (3.0 * N * N);
    r.offset = 0.5;
  } else if (i <= 3 * N) {
    r.len = 4 * N;
    r.first = 2 * N * (N - 1) + (i - N) * 4 * N;
    r.z = (double)(4 * N - 2 * i) / (3.0 * N);
    r.offset = ((i - N) % 2 == 0) ? 0.5 : 0.0;
  } else {
    const int64_t k = 4 * N - i;
    r.len = 4 * k;
    r.first = 12 * N * N - 2 * k * (k + 1);
    r.z = -(1.0 - (double)(k * k) / (3.0 * N * N));
    r.offset = 0.5;
  }
  return r;
}

int64_t ring_len(int64_t nside, int64_t i) {
  return 4 * std::min(std::min(i, nside), 4 * nside - i);
}

// Chunk of a ring block that holds offset j of a ring of `len` pixels, in a
// block whose longest ring has `maxlen`, chunks `width` wide: chunk c starts
// at floor(width c len / maxlen), so this is the largest c with that
// start <= j.
int64_t chunk_of(int64_t j, int64_t len, int64_t maxlen, int64_t width) {
  const int64_t num = (j + 1) * maxlen, den = width * len;
  return (num + den - 1) / den - 1;
}

}  // namespace

void make_strips(int64_t nside, int64_t tile_px, Tiling& t) {
  t = Tiling();
  t.nside = nside;
  t.tile_px = tile_px;
  t.blocks = false;
  const int64_t npix = 12 * nside * nside;
  t.ntiles = (npix + tile_px - 1) / tile_px;
}

void make_ring_blocks(int64_t nside, int rings, int64_t width, Tiling& t) {
  t = Tiling();
  t.nside = nside;
  t.rings = rings;
  t.width = width;
  t.blocks = true;
  const int64_t nring = 4 * nside - 1;
  const int64_t nblock = (nring + rings - 1) / rings;
  t.block_first.assign(nblock + 1, 0);
  t.block_maxlen.assign(nblock, 0);
  for (int64_t rb = 0; rb < nblock; ++rb) {
    int64_t maxlen = 0;
    for (int64_t i = 1 + rb * rings; i <= std::min(nring, (rb + 1) * rings); ++i)
      maxlen = std::max(maxlen, ring_len(nside, i));
    t.block_maxlen[rb] = maxlen;
    t.block_first[rb + 1] = t.block_first[rb] + (maxlen + width - 1) / width;
  }
  t.ntiles = t.block_first[nblock];
}

std::pair<int64_t, int64_t> Tiling::ring_span(int64_t i, int64_t j0, int64_t j1) const {
  const RingInfo r = ring_info(nside, i);
  if (!blocks) return {(r.first + j0) / tile_px, (r.first + j1) / tile_px};
  const int64_t rb = (i - 1) / rings;
  const int64_t maxlen = block_maxlen[rb];
  return {block_first[rb] + chunk_of(j0, r.len, maxlen, width),
          block_first[rb] + chunk_of(j1, r.len, maxlen, width)};
}

void ring_block_rows(const Tiling& t, std::vector<int64_t>& rows) {
  rows.assign((size_t)t.ntiles * t.rings, 0);
  const int64_t nring = 4 * t.nside - 1;
  const int64_t nblock = (int64_t)t.block_maxlen.size();
  const int64_t W = t.width;
  for (int64_t rb = 0; rb < nblock; ++rb) {
    const int64_t maxlen = t.block_maxlen[rb];
    const int64_t nchunk = t.block_first[rb + 1] - t.block_first[rb];
    for (int g = 0; g < t.rings; ++g) {
      const int64_t i = 1 + rb * t.rings + g;
      if (i > nring) continue;
      const RingInfo r = ring_info(t.nside, i);
      for (int64_t c = 0; c < nchunk; ++c) {
        const int64_t a = W * c * r.len / maxlen;
        const int64_t b = std::min(r.len, W * (c + 1) * r.len / maxlen);
        if (b <= a) continue;
        rows[(size_t)(t.block_first[rb] + c) * t.rings + g] =
            ((r.first + a) << kRowCountBits) | (b - a);
      }
    }
  }
}

// Tiles that may hold pixels within angle rho of (cx, cy, cz).
void cap_tiles(const Tiling& t, double cx, double cy, double cz, double rho,
               std::vector<std::pair<int64_t, int64_t>>& out) {
  out.clear();
  const int64_t nside = t.nside;
  const int64_t npix = 12 * nside * nside;
  const double nrm = sqrt(cx * cx + cy * cy + cz * cz);
  // Margin: a few pixel widths plus rounding slack.
  const double pix_ang = sqrt(4.0 * M_PI / (double)npix);
  rho = rho + 2.0 * pix_ang + 1e-9;
  if (!(nrm > 0.0) || rho >= M_PI) {
    out.emplace_back(0, t.ntiles - 1);
    return;
  }
  cx /= nrm;
  cy /= nrm;
  cz /= nrm;
  const double zc = std::max(-1.0, std::min(1.0, cz));
  const double thc = acos(zc);
  const double phc = atan2(cy, cx);
  const double sc = sin(thc);
  std::vector<std::pair<int64_t, int64_t>> tl;
  for (int64_t i = 1; i < 4 * nside; ++i) {
    const RingInfo r = ring_info(nside, i);
    const double th = acos(std::max(-1.0, std::min(1.0, r.z)));
    if (fabs(th - thc) > rho) continue;
    const double s = sin(th);
    double half;  // azimuth half-width of the cap on this ring
    if (thc <= rho || thc >= M_PI - rho || s * sc <= 1e-300) {
      half = M_PI;  // the cap reaches a pole, or the ring is at a pole
    } else {
      const double cd = (cos(rho) - r.z * zc) / (s * sc);
      if (cd <= -1.0) half = M_PI;
      else if (cd >= 1.0) half = 0.0;
      else half = acos(cd);
    }
    const double dphi = 2.0 * M_PI / (double)r.len;
    if (half >= M_PI - 2.0 * dphi) {
      tl.push_back(t.ring_span(i, 0, r.len - 1));
      continue;
    }
    // Pixel centres phi_j = (j + offset) dphi; keep j with |phi_j - phc| <= half.
    const double lo = (phc - half) / dphi - r.offset;
    const double hi = (phc + half) / dphi - r.offset;
    int64_t jlo = (int64_t)floor(lo) - 1;
    int64_t jhi = (int64_t)ceil(hi) + 1;
    if (jhi - jlo + 1 >= r.len) {
      tl.push_back(t.ring_span(i, 0, r.len - 1));
      continue;
    }
    // Wrap into [0, len).
    jlo = ((jlo % r.len) + r.len) % r.len;
    jhi = ((jhi % r.len) + r.len) % r.len;
    if (jlo <= jhi) {
      tl.push_back(t.ring_span(i, jlo, jhi));
    } else {
      tl.push_back(t.ring_span(i, 0, jhi));
      tl.push_back(t.ring_span(i, jlo, r.len - 1));
    }
  }
  // Merge the tile ranges.
  std::sort(tl.begin(), tl.end());
  for (auto& x : tl) {
    if (!out.empty() && x.first <= out.back().second + 1)
      out.back().second = std::max(out.back().second, x.second);
    else
      out.push_back(x);
  }
}

// Tiles of a box: all, the tiles of its cap, or those of a cap bounding the
// box (for the ray-crosses-box rule); none when the box lies entirely
// outside the slab's radii.
void box_tiles(const Tiling& t, const HostBoxGeom& g, double eta0,
               std::vector<std::pair<int64_t, int64_t>>& out) {
  out.clear();
  if (g.vis == 0) {
    out.emplace_back(0, t.ntiles - 1);
    return;
  }
  if (g.vis == 2) {
    const double c = std::max(-1.0, std::min(1.0, g.cap_cos));
    cap_tiles(t, g.cap_dir[0], g.cap_dir[1], g.cap_dir[2], acos(c), out);
    return;
  }
  double ctr[3], half = 0.0, dmin2 = 0.0, dmax2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double lo = g.origin[k], hi = g.origin[k] + g.ext[k];
    ctr[k] = 0.5 * (lo + hi);
    half += 0.25 * g.ext[k] * g.ext[k];
    const double nearest = (lo > 0.0) ? lo : (hi < 0.0 ? -hi : 0.0);
    dmin2 += nearest * nearest;
    const double far = std::max(fabs(lo), fabs(hi));
    dmax2 += far * far;
  }
  const double r_lo = eta0 - g.eta_hi, r_hi = eta0 - g.eta_lo;
  if (sqrt(dmax2) * (1.0 + 1e-12) < r_lo || sqrt(dmin2) * (1.0 - 1e-12) > r_hi) return;
  half = sqrt(half);
  const double d = sqrt(ctr[0] * ctr[0] + ctr[1] * ctr[1] + ctr[2] * ctr[2]);
  if (d <= half * (1.0 + 1e-9)) {
    out.emplace_back(0, t.ntiles - 1);
    return;
  }
  cap_tiles(t, ctr[0], ctr[1], ctr[2], asin(std::min(1.0, half / d)), out);
}

}  // namespace csmap
