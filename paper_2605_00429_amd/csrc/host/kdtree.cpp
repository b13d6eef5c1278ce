#include "kdtree.h"

#include <algorithm>
#include <atomic>
#include <limits>
#include <queue>
#include <thread>

namespace p2m {

namespace {
constexpr int kLeaf = 8;
}

void KdTree::build(const std::vector<d3>& pts, int n_threads)
{
    static std::atomic<uint64_t> next_stamp{1};
    stamp_ = next_stamp.fetch_add(1);
    pts_ = pts;
    idx_.resize(pts.size());
    for (size_t i = 0; i < pts.size(); ++i) idx_[i] = (int32_t)i;
    nodes_.clear();
    nodes_.reserve(2 * pts.size() / kLeaf + 2);
    depth_ = 0;
    int par = 0;  // levels whose left subtree goes to a thread of its own
    while (par < 6 && (1 << par) < n_threads) ++par;
    if (!pts.empty()) build_rec(0, (int32_t)pts.size(), 1, nodes_, depth_, par);
}

// Appends the subtree of idx_[b, e) to `out` in depth-first order and
// returns its root's index.  With par > 0 the two subtrees are built into
// their own arrays, the left one on a thread, and spliced in with their
// indices shifted: the same array as the sequential order gives.
int32_t KdTree::build_rec(int32_t b, int32_t e, int depth, std::vector<Node>& out, int& max_depth, int par)
{
    max_depth = std::max(max_depth, depth);
    Node n;
    n.lo = {INFINITY, INFINITY, INFINITY};
    n.hi = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = b; i < e; ++i) {
        n.lo = dmin3(n.lo, pts_[idx_[i]]);
        n.hi = dmax3(n.hi, pts_[idx_[i]]);
    }
    n.begin = b;
    n.end = e;
    n.left = n.right = -1;
    int32_t id = (int32_t)out.size();
    out.push_back(n);
    if (e - b <= kLeaf) return id;
    d3 ext = n.hi - n.lo;
    int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
    int32_t m = b + (e - b) / 2;
    std::nth_element(idx_.begin() + b, idx_.begin() + m, idx_.begin() + e,
                     [&](int32_t i, int32_t j) { return comp(pts_[i], axis) < comp(pts_[j], axis); });
    if (par <= 0) {
        int32_t l = build_rec(b, m, depth + 1, out, max_depth, 0);
        int32_t r = build_rec(m, e, depth + 1, out, max_depth, 0);
        out[id].left = l;
        out[id].right = r;
        return id;
    }
    std::vector<Node> L, R;
    int dl = 0, dr = 0;
    std::thread left([&] { build_rec(b, m, depth + 1, L, dl, par - 1); });
    build_rec(m, e, depth + 1, R, dr, par - 1);
    left.join();
    max_depth = std::max(max_depth, std::max(dl, dr));
    auto splice = [&](const std::vector<Node>& sub) {
        const int32_t shift = (int32_t)out.size();
        for (Node x : sub) {
            if (x.left >= 0) {
                x.left += shift;
                x.right += shift;
            }
            out.push_back(x);
        }
        return shift;
    };
    const int32_t l = splice(L);
    const int32_t r = splice(R);
    out[id].left = l;
    out[id].right = r;
    return id;
}

double KdTree::box_d2(const Node& n, d3 q)
{
    double dx = std::max({n.lo.x - q.x, 0.0, q.x - n.hi.x});
    double dy = std::max({n.lo.y - q.y, 0.0, q.y - n.hi.y});
    double dz = std::max({n.lo.z - q.z, 0.0, q.z - n.hi.z});
    return dx * dx + dy * dy + dz * dz;
}

void KdTree::knn(d3 q, int k, int32_t skip, std::vector<std::pair<double, int32_t>>& out) const
{
    out.clear();
    if (nodes_.empty() || k <= 0) return;
    // max-heap of the current best k
    std::priority_queue<std::pair<double, int32_t>> best;
    struct Item { double d2; int32_t node; };
    std::vector<Item> stack;
    stack.push_back({box_d2(nodes_[0], q), 0});
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        if ((int)best.size() == k && it.d2 >= best.top().first) continue;
        const Node& n = nodes_[it.node];
        if (n.left < 0) {
            for (int32_t i = n.begin; i < n.end; ++i) {
                int32_t p = idx_[i];
                if (p == skip) continue;
                double d2 = norm2(pts_[p] - q);
                if ((int)best.size() < k) best.push({d2, p});
                else if (d2 < best.top().first || (d2 == best.top().first && p < best.top().second)) {
                    best.pop();
                    best.push({d2, p});
                }
            }
            continue;
        }
        double dl = box_d2(nodes_[n.left], q), dr = box_d2(nodes_[n.right], q);
        if (dl <= dr) {
            stack.push_back({dr, n.right});
            stack.push_back({dl, n.left});
        } else {
            stack.push_back({dl, n.left});
            stack.push_back({dr, n.right});
        }
    }
    out.resize(best.size());
    for (size_t i = out.size(); i-- > 0;) {
        out[i] = best.top();
        best.pop();
    }
}

int32_t KdTree::nearest_below(d3 q, double limit2, const std::vector<int32_t>& excluded,
                              double* d2_out, bool first, int64_t max_points) const
{
    if (nodes_.empty()) return -1;
    double best = limit2;
    int32_t bi = -1;
    struct Item { double d2; int32_t node; };
    std::vector<Item> stack;
    stack.reserve(64);
    stack.push_back({box_d2(nodes_[0], q), 0});
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        if (it.d2 >= best) continue;
        const Node& n = nodes_[it.node];
        if (n.left < 0) {
            if (max_points >= 0) {
                max_points -= n.end - n.begin;
                if (max_points < 0) return -2;
            }
            for (int32_t i = n.begin; i < n.end; ++i) {
                int32_t p = idx_[i];
                double d2 = norm2(pts_[p] - q);
                if (d2 < best || (d2 == best && bi >= 0 && p < bi)) {
                    if (std::binary_search(excluded.begin(), excluded.end(), p)) continue;
                    best = d2;
                    bi = p;
                    if (first) {
                        if (d2_out) *d2_out = best;
                        return bi;
                    }
                }
            }
            continue;
        }
        double dl = box_d2(nodes_[n.left], q), dr = box_d2(nodes_[n.right], q);
        if (dl <= dr) {
            stack.push_back({dr, n.right});
            stack.push_back({dl, n.left});
        } else {
            stack.push_back({dl, n.left});
            stack.push_back({dr, n.right});
        }
    }
    if (d2_out) *d2_out = best;
    return bi;
}

int32_t KdTree::below(d3 q, double limit2, const int32_t* ex_begin, const int32_t* ex_end, int64_t budget) const
{
    if (nodes_.empty()) return -1;
    double best = limit2;
    int32_t bi = -1;
    struct Item { double d2; int32_t node; };
    // a depth-first search keeps at most one pending sibling per level
    Item st[kBelowStack];
    int top = 0;
    st[top++] = {box_d2(nodes_[0], q), 0};
    while (top > 0) {
        const Item it = st[--top];
        if (it.d2 >= best) continue;
        const Node& n = nodes_[it.node];
        if (n.left < 0) {
            if (budget >= 0) {
                budget -= n.end - n.begin;
                if (budget < 0) return -2;
            }
            for (int32_t i = n.begin; i < n.end; ++i) {
                const int32_t p = idx_[i];
                const double d2 = norm2(pts_[p] - q);
                if (d2 < best || (d2 == best && bi >= 0 && p < bi)) {
                    if (std::binary_search(ex_begin, ex_end, p)) continue;
                    best = d2;
                    bi = p;
                }
            }
            continue;
        }
        const double dl = box_d2(nodes_[n.left], q), dr = box_d2(nodes_[n.right], q);
        if (dl <= dr) {
            st[top++] = {dr, n.right};
            st[top++] = {dl, n.left};
        } else {
            st[top++] = {dl, n.left};
            st[top++] = {dr, n.right};
        }
    }
    return bi;
}

void KdTree::export_flat(std::vector<double>& box, std::vector<int32_t>& link, std::vector<int32_t>& order,
                         std::vector<double>& pts) const
{
    box.resize(6 * nodes_.size());
    link.resize(4 * nodes_.size());
    for (size_t i = 0; i < nodes_.size(); ++i) {
        const Node& n = nodes_[i];
        const double b[6] = {n.lo.x, n.lo.y, n.lo.z, n.hi.x, n.hi.y, n.hi.z};
        std::copy(b, b + 6, box.begin() + 6 * i);
        link[4 * i] = n.begin;
        link[4 * i + 1] = n.end;
        link[4 * i + 2] = n.left;
        link[4 * i + 3] = n.right;
    }
    order = idx_;
    pts.resize(3 * pts_.size());
    for (size_t i = 0; i < pts_.size(); ++i) {
        pts[3 * i] = pts_[i].x;
        pts[3 * i + 1] = pts_[i].y;
        pts[3 * i + 2] = pts_[i].z;
    }
}

int32_t KdTree::nearest(d3 q, double* d2_out) const
{
    static const std::vector<int32_t> none;
    return nearest_below(q, std::numeric_limits<double>::infinity(), none, d2_out);
}

void KdTree::radius(d3 q, double r2, std::vector<int32_t>& out) const
{
    if (nodes_.empty()) return;
    std::vector<int32_t> stack{0};
    while (!stack.empty()) {
        int32_t ni = stack.back();
        stack.pop_back();
        const Node& n = nodes_[ni];
        if (box_d2(n, q) > r2) continue;
        if (n.left < 0) {
            for (int32_t i = n.begin; i < n.end; ++i)
                if (norm2(pts_[idx_[i]] - q) <= r2) out.push_back(idx_[i]);
            continue;
        }
        stack.push_back(n.left);
        stack.push_back(n.right);
    }
}

}  // namespace p2m
