// Binary bounding-volume hierarchy over the mesh triangles (FP64 boxes).
// Host uses: sphere-union vs mesh intersection (interception lists),
// closest point on the mesh (reference point of an off-surface site).  Its
// depth-first node array and leaf order are also exported to the device for
// the exact fallback of queries outside the domain box.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.h"

namespace p2m {

struct Ball {
    d3 c;
    double r;
};

class Bvh {
public:
    struct Node {
        d3 lo, hi;
        int32_t left_or_begin;  // internal: unused (left child is next node); leaf: first slot in order()
        int32_t right_or_count; // internal: right child index; leaf: -count
    };
    // tri: 3 vertices per triangle (FP64 copies of the FP32 input).  With
    // n_threads > 1 the top levels' subtrees are built on threads; the tree
    // is the same.
    void build(const std::vector<d3>& tri, int n_threads = 1);
    // Triangles (original ids) meeting the closed union of `balls`.  `stamp`
    // (size >= n triangles) and `gen` deduplicate across calls.  Stops as
    // soon as `out` holds more than `cap` entries (it is then incomplete).
    void query_union(const std::vector<Ball>& balls, std::vector<int32_t>& out,
                     std::vector<uint32_t>& stamp, uint32_t gen, size_t cap = SIZE_MAX) const;
    // Closest point of the mesh to q; returns squared distance.
    double closest(d3 q, int32_t* tri, d3* p) const;
    const std::vector<Node>& nodes() const { return nodes_; }
    const std::vector<int32_t>& order() const { return order_; }

private:
    int32_t build_rec(int32_t b, int32_t e, const std::vector<d3>& cen, std::vector<Node>& out, int par);
    static double box_d2(const Node& n, d3 q);
    const std::vector<d3>* tri_ = nullptr;
    std::vector<Node> nodes_;
    std::vector<int32_t> order_;
};

}  // namespace p2m
