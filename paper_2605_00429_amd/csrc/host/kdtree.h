// Static kd-tree over the sites (FP64), used by the host preprocessing for
// k-nearest-neighbour candidates, exact nearest-site lookups and
// "is any site closer than s to this corner" checks.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

namespace p2m {

class KdTree {
public:
    void build(const std::vector<d3>& pts);
    // k nearest points to q (excluding index `skip`), ascending distance.
    void knn(d3 q, int k, int32_t skip, std::vector<std::pair<double, int32_t>>& out) const;
    // Nearest point to q with squared distance strictly below `limit2` whose
    // index is not in `excluded` (a small sorted vector).  -1 if none.  With
    // `first`, any such point (the first the search meets) is returned.
    // With max_points >= 0 the search gives up after examining that many
    // points and returns -2 (undecided).
    int32_t nearest_below(d3 q, double limit2, const std::vector<int32_t>& excluded,
                          double* d2_out = nullptr, bool first = false, int64_t max_points = -1) const;
    // Exact nearest point (lowest index on exact ties).
    int32_t nearest(d3 q, double* d2_out = nullptr) const;
    // Every point with squared distance <= r2 (appended, unordered).
    void radius(d3 q, double r2, std::vector<int32_t>& out) const;
    // Points in tree order (a spatially coherent permutation).
    const std::vector<int32_t>& order() const { return idx_; }

private:
    struct Node {
        d3 lo, hi;
        int32_t begin, end;   // range in idx_ (leaves)
        int32_t left, right;  // children, -1 for a leaf
    };
    int32_t build_rec(int32_t b, int32_t e);
    static double box_d2(const Node& n, d3 q);
    std::vector<d3> pts_;
    std::vector<int32_t> idx_;
    std::vector<Node> nodes_;
};

}  // namespace p2m
