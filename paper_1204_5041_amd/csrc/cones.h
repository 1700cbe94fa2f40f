// cones.h -- placement of simulation boxes in healpix cones (host side).
//
// The comoving ball between two radii is cut into truncated cones subtending
// the pixels of a coarse HEALPix grid, and each cone is filled by one cubic
// simulation box, turned so that its photons travel towards the observer and
// the farthest pixel of the cone fits inside the box's far face (Sec. II.C,
// Fig. 1).
#pragma once
#include <stdint.h>

namespace csmap {

// Frame of a box placed in cone `pix` of the Nside grid, with box axis `axis`
// (0, 1 or 2) pointing out along the cone axis n (the photons, which travel
// towards -axis in the box, then travel towards the observer).  The other two
// box axes follow (e_theta + e_phi)/sqrt(2) and (e_phi - e_theta)/sqrt(2) at
// the cone centre, in cyclic order, so that the frame is right-handed and the
// pixel's diamond sits across the face diagonals.  The far face (box
// coordinate axis = side) lies in the plane n.P = r_out, centred on the
// axis: a box point x is at P = origin + rot x (rot row-major).
//
// slack = the smallest margin, in length units, of the conditions that put
// the whole truncated cone r_in <= |P| <= r_out inside the box:
//   side/2 - r_out max |e.d| over the pixel, for each transverse axis e;
//   r_in min n.d over the pixel - (r_out - side)   (the near face);
// d runs over the pixel's boundary, sampled at 257 points per edge from the
// closed form of the edges.  slack >= 0: the cone fits.
struct ConePlacement {
  double rot[9];
  double origin[3];
  double slack;
};

// Requires 1 <= nside <= 8192, 0 <= pix < 12 nside^2, axis in {0, 1, 2}.
void cone_place(int64_t nside, int64_t pix, int axis, double r_in, double r_out, double side,
                ConePlacement& out);

// Caps around the pixel centre dir that bracket the pixel: every direction
// whose cosine to dir is below cos_out lies outside the pixel, every one above
// cos_in inside (cos_in > 1 when no such cap is certain), both with a margin
// of 2% of the cap radius plus 1e-7 rad beyond the sampled boundary.
void cone_caps(int64_t nside, int64_t pix, double dir[3], double& cos_out, double& cos_in);

// Between the caps, each edge e of the pixel is bracketed by the plane
// through the origin and the edge's two end corners, with unit normal n[e]
// pointing into the pixel: hi[e] is the largest n[e].d over edge e and lo[e]
// the smallest n[e].d over the whole boundary, each moved by a margin of
// 1e-7 + (4 a_out / 256)^2 (a_out the outer cap's radius) for the sampling
// of the edges.  A direction inside the outer cap with n[e].d > hi[e] for
// every e is inside the pixel, and one with n[e].d < lo[e] for some e is
// outside it: a great-circle arc from the centre of length below pi/2 along
// which n[e].d falls to the boundary and rises again cannot exist.  When the
// centre is not strictly inside every slab or the cap is not below pi/2,
// hi = +inf and lo = -inf (the planes never decide).
struct ConeEdges {
  double n[4][3];
  double hi[4], lo[4];
};
void cone_edges(int64_t nside, int64_t pix, ConeEdges& out);

// Smallest slack over every cone of the grid (the same for every axis).
double cone_grid_slack(int64_t nside, double r_in, double r_out, double side);

}  // namespace csmap
