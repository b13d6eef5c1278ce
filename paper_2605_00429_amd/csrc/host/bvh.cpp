#include "bvh.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace p2m {

namespace {
constexpr int kLeafTris = 4;
}

void Bvh::build(const std::vector<d3>& tri, int n_threads)
{
    tri_ = &tri;
    const int32_t n = (int32_t)(tri.size() / 3);
    order_.resize(n);
    std::vector<d3> cen(n);
    for (int32_t i = 0; i < n; ++i) {
        order_[i] = i;
        cen[i] = (tri[3 * i] + tri[3 * i + 1] + tri[3 * i + 2]) * (1.0 / 3.0);
    }
    nodes_.clear();
    nodes_.reserve(2 * (size_t)n / kLeafTris + 2);
    int par = 0;  // levels whose left subtree goes to a thread of its own
    while (par < 6 && (1 << par) < n_threads) ++par;
    if (n > 0) build_rec(0, n, cen, nodes_, par);
}

// Appends the subtree of order_[b, e) to `out` in depth-first order (a
// node, its left subtree, its right subtree) and returns its root's index.
// With par > 0 the two subtrees are built into their own arrays, the left
// one on a thread, and spliced in with their indices shifted, which gives
// the array the sequential order gives: the ranges are disjoint and each
// split depends on its own range only.
int32_t Bvh::build_rec(int32_t b, int32_t e, const std::vector<d3>& cen, std::vector<Node>& out, int par)
{
    const std::vector<d3>& T = *tri_;
    Node nd;
    nd.lo = {INFINITY, INFINITY, INFINITY};
    nd.hi = {-INFINITY, -INFINITY, -INFINITY};
    d3 clo = nd.lo, chi = nd.hi;
    for (int32_t i = b; i < e; ++i) {
        const int32_t t = order_[i];
        for (int k = 0; k < 3; ++k) {
            nd.lo = dmin3(nd.lo, T[3 * t + k]);
            nd.hi = dmax3(nd.hi, T[3 * t + k]);
        }
        clo = dmin3(clo, cen[t]);
        chi = dmax3(chi, cen[t]);
    }
    const int32_t id = (int32_t)out.size();
    out.push_back(nd);
    if (e - b <= kLeafTris) {
        out[id].left_or_begin = b;
        out[id].right_or_count = -(e - b);
        return id;
    }
    const d3 ext = chi - clo;
    const int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
    const int32_t m = b + (e - b) / 2;
    std::nth_element(order_.begin() + b, order_.begin() + m, order_.begin() + e,
                     [&](int32_t i, int32_t j) { return comp(cen[i], axis) < comp(cen[j], axis); });
    if (par <= 0) {
        build_rec(b, m, cen, out, 0);  // left child is id + 1
        const int32_t r = build_rec(m, e, cen, out, 0);
        out[id].left_or_begin = id + 1;
        out[id].right_or_count = r;
        return id;
    }
    std::vector<Node> L, R;
    std::thread left([&] { build_rec(b, m, cen, L, par - 1); });
    build_rec(m, e, cen, R, par - 1);
    left.join();
    auto splice = [&](const std::vector<Node>& sub) {
        const int32_t shift = (int32_t)out.size();
        for (Node x : sub) {
            if (x.right_or_count >= 0) {  // internal: both links are indices
                x.left_or_begin += shift;
                x.right_or_count += shift;
            }
            out.push_back(x);
        }
        return shift;
    };
    const int32_t l = splice(L);
    const int32_t r = splice(R);
    out[id].left_or_begin = l;
    out[id].right_or_count = r;
    return id;
}

double Bvh::box_d2(const Node& n, d3 q)
{
    const double dx = std::max({n.lo.x - q.x, 0.0, q.x - n.hi.x});
    const double dy = std::max({n.lo.y - q.y, 0.0, q.y - n.hi.y});
    const double dz = std::max({n.lo.z - q.z, 0.0, q.z - n.hi.z});
    return dx * dx + dy * dy + dz * dz;
}

void Bvh::query_union(const std::vector<Ball>& balls, std::vector<int32_t>& out,
                      std::vector<uint32_t>& stamp, uint32_t gen, size_t cap) const
{
    if (nodes_.empty() || balls.empty()) return;
    const std::vector<d3>& T = *tri_;
    // Balls are handled 64 at a time; each stack entry carries the mask of
    // balls that still overlap the node, so deep nodes test few balls.
    for (size_t b0 = 0; b0 < balls.size(); b0 += 64) {
        const int nb = (int)std::min<size_t>(64, balls.size() - b0);
        const Ball* B = balls.data() + b0;
        struct Item { int32_t node; uint64_t mask; };
        Item stack[128];
        int sp = 0;
        stack[sp++] = {0, nb == 64 ? ~0ULL : ((1ULL << nb) - 1)};
        while (sp > 0) {
            const Item it = stack[--sp];
            const Node& n = nodes_[it.node];
            uint64_t m = 0;
            for (uint64_t r = it.mask; r; r &= r - 1) {
                const int k = __builtin_ctzll(r);
                if (box_d2(n, B[k].c) <= B[k].r * B[k].r) m |= 1ULL << k;
            }
            if (!m) continue;
            if (n.right_or_count < 0) {
                for (int32_t i = n.left_or_begin; i < n.left_or_begin - n.right_or_count; ++i) {
                    const int32_t t = order_[i];
                    if (stamp[t] == gen) continue;
                    const d3 a = T[3 * t], b = T[3 * t + 1], c = T[3 * t + 2];
                    const d3 lo = dmin3(a, dmin3(b, c)), hi = dmax3(a, dmax3(b, c));
                    for (uint64_t r = m; r; r &= r - 1) {
                        const Ball& bl = B[__builtin_ctzll(r)];
                        const double dx = std::max({lo.x - bl.c.x, 0.0, bl.c.x - hi.x});
                        const double dy = std::max({lo.y - bl.c.y, 0.0, bl.c.y - hi.y});
                        const double dz = std::max({lo.z - bl.c.z, 0.0, bl.c.z - hi.z});
                        const double r2 = bl.r * bl.r;
                        if (dx * dx + dy * dy + dz * dz > r2) continue;
                        d3 p;
                        if (closest_on_triangle(bl.c, a, b, c, &p) <= r2) {
                            stamp[t] = gen;
                            out.push_back(t);
                            if (out.size() > cap) return;
                            break;
                        }
                    }
                }
                continue;
            }
            stack[sp++] = {n.right_or_count, m};
            stack[sp++] = {it.node + 1, m};
        }
    }
}

double Bvh::closest(d3 q, int32_t* tri, d3* p) const
{
    const std::vector<d3>& T = *tri_;
    double best = INFINITY;
    int32_t bt = -1;
    d3 bp{0, 0, 0};
    struct Item { double d2; int32_t node; };
    Item stack[128];
    int sp = 0;
    if (nodes_.empty()) return best;
    stack[sp++] = {box_d2(nodes_[0], q), 0};
    while (sp > 0) {
        const Item it = stack[--sp];
        if (it.d2 >= best) continue;
        const Node& n = nodes_[it.node];
        if (n.right_or_count < 0) {
            for (int32_t i = n.left_or_begin; i < n.left_or_begin - n.right_or_count; ++i) {
                const int32_t t = order_[i];
                d3 pp;
                const double d2 = closest_on_triangle(q, T[3 * t], T[3 * t + 1], T[3 * t + 2], &pp);
                if (d2 < best) { best = d2; bt = t; bp = pp; }
            }
            continue;
        }
        const int32_t l = it.node + 1, r = n.right_or_count;
        const double dl = box_d2(nodes_[l], q), dr = box_d2(nodes_[r], q);
        if (dl <= dr) { stack[sp++] = {dr, r}; stack[sp++] = {dl, l}; }
        else { stack[sp++] = {dl, l}; stack[sp++] = {dr, r}; }
    }
    if (tri) *tri = bt;
    if (p) *p = bp;
    return best;
}

}  // namespace p2m
