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
    // With n_threads > 1 the top levels' subtrees are built on threads;
    // the tree is the same.
    void build(const std::vector<d3>& pts, int n_threads = 1);
    // k nearest points to q (excluding index `skip`), ascending distance.
    void knn(d3 q, int k, int32_t skip, std::vector<std::pair<double, int32_t>>& out) const;
    // Nearest point to q with squared distance strictly below `limit2` whose
    // index is not in `excluded` (a small sorted vector).  -1 if none.  With
    // `first`, any such point (the first the search meets) is returned.
    // With max_points >= 0 the search gives up after examining that many
    // points and returns -2 (undecided).
    int32_t nearest_below(d3 q, double limit2, const std::vector<int32_t>& excluded,
                          double* d2_out = nullptr, bool first = false, int64_t max_points = -1) const;
    // nearest_below(q, limit2, excluded, nullptr, false, budget) with the
    // excluded indices given as a sorted range; the search order (nearer
    // child first) and the budget count are the same, which a device
    // version reproduces step for step.
    int32_t below(d3 q, double limit2, const int32_t* ex_begin, const int32_t* ex_end, int64_t budget = -1) const;
    // Levels of the tree (its nodes' deepest level, root = 1).  A
    // depth-first search of it holds at most depth + 1 entries.
    int depth() const { return depth_; }
    static constexpr int kBelowStack = 64;
    // Exact nearest point (lowest index on exact ties).
    int32_t nearest(d3 q, double* d2_out = nullptr) const;
    // Every point with squared distance <= r2 (appended, unordered).
    void radius(d3 q, double r2, std::vector<int32_t>& out) const;
    // Points in tree order (a spatially coherent permutation).
    const std::vector<int32_t>& order() const { return idx_; }

    // Flat copy for a device: per node lo.xyz, hi.xyz (6 doubles) and
    // begin, end, left, right (4 ints; left = -1 for a leaf); the point
    // order; the points (3 doubles each).
    void export_flat(std::vector<double>& box, std::vector<int32_t>& link, std::vector<int32_t>& order,
                     std::vector<double>& pts) const;
    int32_t n_nodes() const { return (int32_t)nodes_.size(); }
    // Distinct for every build of any tree in the process (a device copy
    // made from one build can be reused until the tree is rebuilt).
    uint64_t stamp() const { return stamp_; }

private:
    struct Node {
        d3 lo, hi;
        int32_t begin, end;   // range in idx_ (leaves)
        int32_t left, right;  // children, -1 for a leaf
    };
    int32_t build_rec(int32_t b, int32_t e, int depth, std::vector<Node>& out, int& max_depth, int par);
    static double box_d2(const Node& n, d3 q);
    std::vector<d3> pts_;
    std::vector<int32_t> idx_;
    std::vector<Node> nodes_;
    int depth_ = 0;
    uint64_t stamp_ = 0;
};

}  // namespace p2m
