// sched.h -- host-side work planning.
#pragma once
#include <stdint.h>

#include <utility>
#include <vector>

namespace csmap {

struct HostBoxGeom {
  double origin[3], ext[3];
  double eta_lo, eta_hi;
  int vis;
  double cap_dir[3], cap_cos;
};

void cap_tiles(int64_t nside, int64_t tile, double cx, double cy, double cz, double rho,
               std::vector<std::pair<int64_t, int64_t>>& out);

void box_tiles(int64_t nside, int64_t tile, const HostBoxGeom& g, double eta0,
               std::vector<std::pair<int64_t, int64_t>>& out);

}  // namespace csmap
