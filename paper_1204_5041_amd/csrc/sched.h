// sched.h -- host-side work planning.
#pragma once
#include <stdint.h>

#include <utility>
#include <vector>

#include "tiling.h"

namespace csmap {

struct HostBoxGeom {
  double origin[3], ext[3];
  double eta_lo, eta_hi;
  int vis;
  double cap_dir[3], cap_cos;
};

// How the RING pixels are cut into the tiles that wavefronts own.
//
// Strips: tile t is the `tile_px` consecutive RING pixels starting at
// t * tile_px (the last tile is cut at the end of the map).
//
// Ring blocks: rings 1 .. 4 Nside - 1 are grouped `rings` at a time; a block
// is cut along azimuth into chunks of at most `width` pixels per ring,
// aligned so that chunk c covers the same azimuth range in every ring of the
// block (rings of a block differ in length only near the poles).  Tile =
// (block, chunk): one row of up to `width` consecutive pixels in each ring of
// the block, a compact patch of sky instead of a strip along one ring.
// Every pixel lies in exactly one row of one tile.
struct Tiling {
  int64_t nside = 0;
  int64_t tile_px = 0;       // strips: pixels per tile
  int rings = 1;             // ring blocks: rings per block (rows per tile)
  int64_t width = 64;        // ring blocks: most pixels of a row
  bool blocks = false;
  int64_t ntiles = 0;
  std::vector<int64_t> block_first;   // ring blocks: first tile of each block (+ end)
  std::vector<int64_t> block_maxlen;  // ring blocks: longest ring of each block

  // Inclusive range of tiles that hold offsets [j0, j1] of ring i (1-based).
  std::pair<int64_t, int64_t> ring_span(int64_t i, int64_t j0, int64_t j1) const;
};

void make_strips(int64_t nside, int64_t tile_px, Tiling& t);
void make_ring_blocks(int64_t nside, int rings, int64_t width, Tiling& t);

// Row table of a ring-block tiling: `rings` entries per tile, entry (t, g) =
// (first RING pixel of the row << kRowCountBits) | (pixels in the row); an
// empty row (a block past the last ring, or a short ring) is stored as 0.
void ring_block_rows(const Tiling& t, std::vector<int64_t>& rows);

// Tiles that may hold pixels within angle rho of (cx, cy, cz), as merged
// inclusive ranges (conservative: never omits a tile).
void cap_tiles(const Tiling& t, double cx, double cy, double cz, double rho,
               std::vector<std::pair<int64_t, int64_t>>& out);

void box_tiles(const Tiling& t, const HostBoxGeom& g, double eta0,
               std::vector<std::pair<int64_t, int64_t>>& out);

}  // namespace csmap
