// Pieces of the Voronoi cell clipping (Sec. 3.2: cells are the domain box
// cut by bisector half-spaces) that the host clipper and the device one
// share, so that both take the same decisions on the same FP64 values.
// Everything here uses only +, -, *, / and comparisons, which round the
// same way on the host and on the device.
#pragma once

#ifdef __HIPCC__
#define P2M_HD __host__ __device__
#else
#define P2M_HD
#endif

namespace p2m {

// A vertex within kClipEps * |n| * scale of a clipping plane lies on it
// (scale: the largest corner norm of the box the cell started from).
constexpr double kClipEps = 1e-12;
// Face bounding spheres are inflated by this factor against rounding.
constexpr double kSealInflate = 1.0 + 1e-12;
// Cut points and corners closer than kMergeTol * scale are one point.
constexpr double kMergeTol = 1e-11;
// A face smaller than (kMinArea * scale)^2 bounds no neighbour.
constexpr double kMinArea = 1e-12;

// A key in [0, 4) that increases with the angle of (x, y) measured from
// the +x axis over [0, 2 pi): the position along the unit diamond
// |x| + |y| = 1 of the ray through (x, y).  Sorting cut points by it gives
// their angular order around the new face's centre without a library
// arctangent, whose last bit differs between implementations.  (0, 0)
// gets 0.
P2M_HD inline double diamond_angle(double x, double y)
{
    if (x == 0.0 && y == 0.0) return 0.0;
    if (y >= 0.0) return x >= 0.0 ? y / (x + y) : 1.0 + (-x) / (y - x);
    return x < 0.0 ? 2.0 + (-y) / (-x - y) : 3.0 + x / (x - y);
}

}  // namespace p2m
