#include "octree.h"

#include <algorithm>
#include <cmath>

namespace p2m {

namespace {

struct OCell {
    float c[3];
    float h;
    int depth;
    int32_t node;
};

}  // namespace

void build_octree(const std::vector<d3>& tri, const Bvh& bvh, d3 lo, d3 hi, double delta, int max_list,
                  int max_depth, int n_threads, OctreeCells& out)
{
    out = OctreeCells{};
    const double ext = std::max({hi.x - lo.x, hi.y - lo.y, hi.z - lo.z, 1e-30});
    const int k = (int)std::ceil(std::log2(0.5 * ext * (1.0 + 1e-9)));
    const double half = std::ldexp(1.0, k);
    const double q = std::ldexp(1.0, k - 20);
    const d3 mid = (lo + hi) * 0.5;
    out.root[0] = (float)(std::round(mid.x / q) * q);
    out.root[1] = (float)(std::round(mid.y / q) * q);
    out.root[2] = (float)(std::round(mid.z / q) * q);
    // snapping moves the centre by at most q / 2: widen by one step so the
    // cube still covers [lo, hi]
    out.root[3] = (float)(ext * 0.5 + q <= half ? half : 2.0 * half);
    max_depth = std::min(max_depth, 16);

    const int64_t nT = (int64_t)tri.size() / 3;
    struct Work {
        std::vector<Ball> balls;
        std::vector<int32_t> list;
        std::vector<uint32_t> stamp;
        uint32_t gen = 0;
    };
    std::vector<Work> work(std::max(1, n_threads));
    for (auto& w : work) w.stamp.assign(nT, 0);
    auto cell_list = [&](const OCell& cl, Work& w, size_t cap) {
        const d3 c{cl.c[0], cl.c[1], cl.c[2]};
        d3 v;
        bvh.closest(c, nullptr, &v);
        w.balls.clear();
        for (int m = 0; m < 8; ++m) {
            const d3 u{c.x + ((m & 1) ? cl.h : -(double)cl.h), c.y + ((m & 2) ? cl.h : -(double)cl.h),
                       c.z + ((m & 4) ? cl.h : -(double)cl.h)};
            w.balls.push_back({u, norm(u - v) + delta});
        }
        w.list.clear();
        if (++w.gen == 0) {
            std::fill(w.stamp.begin(), w.stamp.end(), 0);
            w.gen = 1;
        }
        bvh.query_union(w.balls, w.list, w.stamp, w.gen, cap);
    };

    std::vector<OCell> level{OCell{{out.root[0], out.root[1], out.root[2]}, out.root[3], 0, 0}};
    out.nodes.push_back(0);
    while (!level.empty()) {
        const int64_t n = (int64_t)level.size();
        std::vector<char> split(n, 0);
        std::vector<std::vector<int32_t>> full(n);
        parallel_for(n, (int)work.size(), [&](int64_t i, int tid) {
            Work& w = work[tid];
            const OCell& cl = level[i];
            const bool may_split = cl.depth < max_depth;
            cell_list(cl, w, may_split ? (size_t)max_list : SIZE_MAX);
            if (may_split && w.list.size() > (size_t)max_list) split[i] = 1;
            else full[i] = w.list;
        }, 16);
        std::vector<OCell> next;
        for (int64_t i = 0; i < n; ++i) {
            const OCell& cl = level[i];
            if (split[i]) {
                const int32_t base = (int32_t)out.nodes.size();
                out.nodes[cl.node] = base;
                const float h2 = cl.h * 0.5f;
                for (int m = 0; m < 8; ++m) {
                    out.nodes.push_back(0);
                    next.push_back(OCell{{cl.c[0] + ((m & 1) ? h2 : -h2), cl.c[1] + ((m & 2) ? h2 : -h2),
                                          cl.c[2] + ((m & 4) ? h2 : -h2)},
                                         h2, cl.depth + 1, base + m});
                }
            } else {
                const int32_t leaf = (int32_t)out.centre.size();
                out.nodes[cl.node] = -(leaf + 1);
                out.centre.push_back(d3{cl.c[0], cl.c[1], cl.c[2]});
                out.lists.push_back(std::move(full[i]));
                out.depth = std::max(out.depth, cl.depth);
            }
        }
        level.swap(next);
    }
}

int32_t octree_leaf(const OctreeCells& oc, const float q[3])
{
    float c[3] = {oc.root[0], oc.root[1], oc.root[2]};
    float h = oc.root[3];
    for (int k = 0; k < 3; ++k)
        if (!(q[k] >= c[k] - h && q[k] <= c[k] + h)) return -1;
    int32_t node = 0;
    for (;;) {
        const int32_t v = oc.nodes[node];
        if (v < 0) return -v - 1;
        int m = 0;
        h *= 0.5f;
        for (int k = 0; k < 3; ++k) {
            const bool up = q[k] >= c[k];
            m |= (int)up << k;
            c[k] = up ? c[k] + h : c[k] - h;
        }
        node = v + m;
    }
}

}  // namespace p2m
