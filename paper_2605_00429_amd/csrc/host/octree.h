// An adaptive octree as the convex decomposition of the domain, in place of
// the Voronoi cells of the sites (the paper notes that its scheme carries
// over to any convex decomposition with point location).  Each leaf cell is
// a box; its interception list is built as in Sec. 3.3: every triangle that
// meets the union of the balls B(u, |u - v|) over the box corners u, with v
// the mesh point closest to the box centre (Eq. (3) holds for any convex
// cell and any reference point on the mesh).  A cell is split into eight
// while its list is longer than max_list.
#pragma once

#include <cstdint>
#include <vector>

#include "bvh.h"
#include "common.h"

namespace p2m {

struct OctreeCells {
    std::vector<d3> centre;                   // leaf box centres (float32-exact)
    std::vector<std::vector<int32_t>> lists;  // leaf lists (caller triangle ids)
    // Nodes breadth first: the index of the first of 8 contiguous children
    // (child k holds x >= centre if bit 0 of k is set, y for bit 1, z for
    // bit 2), or -(leaf + 1).
    std::vector<int32_t> nodes;
    float root[4] = {0, 0, 0, 1};  // root centre xyz and half size
    int depth = 0;                 // deepest leaf
};

// The root is a cube around [lo, hi] whose half size is a power of two and
// whose centre sits on a grid of 2^-20 of it, so every split plane is exact
// in float32 and the device's descent (float32) visits the cells the host
// built.  delta inflates the ball radii.
void build_octree(const std::vector<d3>& tri, const Bvh& bvh, d3 lo, d3 hi, double delta, int max_list,
                  int max_depth, int n_threads, OctreeCells& out);

// Leaf of the point q (float32 descent, as on the device); -1 outside the root.
int32_t octree_leaf(const OctreeCells& oc, const float q[3]);

}  // namespace p2m
