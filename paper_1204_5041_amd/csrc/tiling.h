// tiling.h -- constants of the ring-block row table shared by the host
// planner and the kernels.
#pragma once

namespace csmap {

// Bits of a ring-block row entry taken by the pixel count; the first RING
// pixel of the row sits above them.
constexpr int kRowCountBits = 10;

}  // namespace csmap
