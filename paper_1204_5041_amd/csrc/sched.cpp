// sched.cpp -- host-side work planning: which pixel tiles can see a box.
//
// A tile is `tile` consecutive RING pixels.  For boxes that do not see the
// whole sky the kernels test every pixel exactly; this file only has to
// produce a superset of the tiles that contain a visible pixel, so every
// quantity here carries a generous margin.
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

void push_pixels(std::vector<std::pair<int64_t, int64_t>>& px, int64_t a, int64_t b) {
  if (b >= a) px.emplace_back(a, b);
}

}  // namespace

// Tiles that may hold pixels within angle rho of (cx, cy, cz).
void cap_tiles(int64_t nside, int64_t tile, double cx, double cy, double cz, double rho,
               std::vector<std::pair<int64_t, int64_t>>& out) {
  out.clear();
  const int64_t npix = 12 * nside * nside;
  const int64_t ntiles = (npix + tile - 1) / tile;
  const double nrm = sqrt(cx * cx + cy * cy + cz * cz);
  // Margin: a few pixel widths plus rounding slack.
  const double pix_ang = sqrt(4.0 * M_PI / (double)npix);
  rho = rho + 2.0 * pix_ang + 1e-9;
  if (!(nrm > 0.0) || rho >= M_PI) {
    out.emplace_back(0, ntiles - 1);
    return;
  }
  cx /= nrm;
  cy /= nrm;
  cz /= nrm;
  const double zc = std::max(-1.0, std::min(1.0, cz));
  const double thc = acos(zc);
  const double phc = atan2(cy, cx);
  const double sc = sin(thc);
  std::vector<std::pair<int64_t, int64_t>> px;
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
      push_pixels(px, r.first, r.first + r.len - 1);
      continue;
    }
    // Pixel centres phi_j = (j + offset) dphi; keep j with |phi_j - phc| <= half.
    const double lo = (phc - half) / dphi - r.offset;
    const double hi = (phc + half) / dphi - r.offset;
    int64_t jlo = (int64_t)floor(lo) - 1;
    int64_t jhi = (int64_t)ceil(hi) + 1;
    if (jhi - jlo + 1 >= r.len) {
      push_pixels(px, r.first, r.first + r.len - 1);
      continue;
    }
    // Wrap into [0, len).
    jlo = ((jlo % r.len) + r.len) % r.len;
    jhi = ((jhi % r.len) + r.len) % r.len;
    if (jlo <= jhi) {
      push_pixels(px, r.first + jlo, r.first + jhi);
    } else {
      push_pixels(px, r.first, r.first + jhi);
      push_pixels(px, r.first + jlo, r.first + r.len - 1);
    }
  }
  // Pixel ranges -> merged tile ranges.
  std::vector<std::pair<int64_t, int64_t>> tl;
  tl.reserve(px.size());
  for (auto& p : px) tl.emplace_back(p.first / tile, p.second / tile);
  std::sort(tl.begin(), tl.end());
  for (auto& t : tl) {
    if (!out.empty() && t.first <= out.back().second + 1)
      out.back().second = std::max(out.back().second, t.second);
    else
      out.push_back(t);
  }
}

// Tiles of a box: all, the tiles of its cap, or those of a cap bounding the
// box (for the ray-crosses-box rule); none when the box lies entirely
// outside the slab's radii.
void box_tiles(int64_t nside, int64_t tile, const HostBoxGeom& g, double eta0,
               std::vector<std::pair<int64_t, int64_t>>& out) {
  out.clear();
  const int64_t npix = 12 * nside * nside;
  const int64_t ntiles = (npix + tile - 1) / tile;
  if (g.vis == 0) {
    out.emplace_back(0, ntiles - 1);
    return;
  }
  if (g.vis == 2) {
    const double c = std::max(-1.0, std::min(1.0, g.cap_cos));
    cap_tiles(nside, tile, g.cap_dir[0], g.cap_dir[1], g.cap_dir[2], acos(c), out);
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
    out.emplace_back(0, ntiles - 1);
    return;
  }
  cap_tiles(nside, tile, ctr[0], ctr[1], ctr[2], asin(std::min(1.0, half / d)), out);
}

}  // namespace csmap
