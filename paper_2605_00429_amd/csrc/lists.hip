// Interception lists on the GPU (Sec. 3.3): for every site, the triangles
// that meet the union of its balls (the corner balls of Eq. (3), or the
// single sphere of Eq. (8)), by a traversal of the mesh BVH.
//
// The host computes the Voronoi cells and the balls; this file takes over
// the sphere-union tests.  It reproduces the host's decisions exactly: the
// same BVH, the same per-node ball masks, the same box and triangle-box
// prefilters and the same FP64 point-triangle distance, evaluated in the
// same operation order with no contraction into fused multiply-adds, so
// both paths give identical lists.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "host/build.h"
#include "host/bvh.h"

namespace p2m {
namespace {

struct GNode {
    double lo[3], hi[3];
    int32_t a;  // internal: left child (next node); leaf: first slot of the BVH order
    int32_t b;  // internal: right child; leaf: -count
};

struct G3 {
    double x, y, z;
};
__device__ __forceinline__ G3 gsub(G3 a, G3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ G3 gadd(G3 a, G3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ G3 gmul(G3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double gdot(G3 a, G3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double gmax3(double a, double b, double c)
{
    // the host takes std::max of {a, b, c}: the first of equal maxima
    double m = a;
    if (m < b) m = b;
    if (m < c) m = c;
    return m;
}

// Squared distance from q to triangle (a, b, c) by its vertex, edge and face
// regions (Ericson, Real-Time Collision Detection, Sec. 5.1.5), the
// operations in the host's order.
__device__ double tri_dist2(G3 q, G3 a, G3 b, G3 c)
{
    const G3 ab = gsub(b, a), ac = gsub(c, a), ap = gsub(q, a);
    const double d1 = gdot(ab, ap), d2 = gdot(ac, ap);
    double u = 1, v = 0, w = 0;
    if (d1 <= 0 && d2 <= 0) {
        u = 1; v = 0; w = 0;
    } else {
        const G3 bp = gsub(q, b);
        const double d3v = gdot(ab, bp), d4 = gdot(ac, bp);
        const G3 cp = gsub(q, c);
        const double d5 = gdot(ab, cp), d6 = gdot(ac, cp);
        const double vc = d1 * d4 - d3v * d2;
        const double vb = d5 * d2 - d1 * d6;
        const double va = d3v * d6 - d5 * d4;
        if (d3v >= 0 && d4 <= d3v) {
            u = 0; v = 1; w = 0;
        } else if (vc <= 0 && d1 >= 0 && d3v <= 0) {
            const double t = d1 / (d1 - d3v);
            u = 1 - t; v = t; w = 0;
        } else if (d6 >= 0 && d5 <= d6) {
            u = 0; v = 0; w = 1;
        } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
            const double t = d2 / (d2 - d6);
            u = 1 - t; v = 0; w = t;
        } else if (va <= 0 && (d4 - d3v) >= 0 && (d5 - d6) >= 0) {
            const double t = (d4 - d3v) / ((d4 - d3v) + (d5 - d6));
            u = 0; v = 1 - t; w = t;
        } else {
            const double den = va + vb + vc;
            if (den > 0 && isfinite(den)) {
                v = vb / den; w = vc / den; u = 1 - v - w;
            } else {
                // zero-area triangle: best of the three edges
                double tt[3], ee[3];
                const G3 s0[3] = {a, b, c}, s1[3] = {b, c, a};
                for (int k = 0; k < 3; ++k) {
                    const G3 e = gsub(s1[k], s0[k]);
                    const double L = gdot(e, e);
                    double t = 0.0;
                    if (L > 0) {
                        t = gdot(gsub(q, s0[k]), e) / L;
                        t = t < 0.0 ? 0.0 : (1.0 < t ? 1.0 : t);
                    }
                    tt[k] = t;
                    const G3 r = gsub(q, gadd(s0[k], gmul(e, t)));
                    ee[k] = gdot(r, r);
                }
                if (ee[0] <= ee[1] && ee[0] <= ee[2]) { u = 1 - tt[0]; v = tt[0]; w = 0; }
                else if (ee[1] <= ee[2]) { u = 0; v = 1 - tt[1]; w = tt[1]; }
                else { u = tt[2]; v = 0; w = 1 - tt[2]; }
            }
        }
    }
    const G3 p = gadd(gadd(gmul(a, u), gmul(b, v)), gmul(c, w));
    const G3 r = gsub(q, p);
    return gdot(r, r);
}

// Balls per lane: a wavefront holds up to 64 * kLaneBalls balls of one site.
constexpr int kLaneBalls = 4;
constexpr int kStack = 64;
constexpr int kWaves = 4;  // wavefronts (sites) per workgroup

// One wavefront per site, its balls spread over the lanes (ball k on lane
// k % 64).  The wavefront walks the BVH depth first as one: at each node
// every lane tests its live balls against the box (live = passed every
// ancestor's box, as in the host's per-node masks), and the node is skipped
// when no lane has one left; at a leaf, a triangle is in the list when any
// lane's live ball passes the triangle-box prefilter and the exact distance
// test.  The node and triangle loads are the same for the whole wavefront.
// The set of triangles is the host's (its order, which the layout stage
// re-sorts, is not).  Pass 1 (kFill = false) counts, and keeps the first
// kRowCap ids of each list in that site's row of `rows`; pass 2 writes the
// ids from off[site] again, for the lists longer than a row only (the
// others are copied from their rows).  A traversal that would overflow its
// stack (never for a BVH of at most 2^29 triangles) reports count -1, and
// the host builds that list itself.
static_assert(64 * kLaneBalls >= kDeviceBalls, "a wavefront must hold every ball the host sends");
constexpr int kRowCap = 256;

// kSub lanes per site (64, 32 or 16: sites with at most kSub * kLB balls
// share a wavefront, each group of lanes walking the BVH with its own
// stack; a group's steps stay uniform, and the wavefront runs until every
// group is done).  Sites are taken from sel (indices into the job's
// sites).
template <bool kFill, int kSub, int kLB>
__global__ void __launch_bounds__(64 * kWaves)
list_kernel(const GNode* __restrict__ nodes, const int32_t* __restrict__ order, const double* __restrict__ T,
            const int64_t* __restrict__ ball_off, const double* __restrict__ balls,
            const int32_t* __restrict__ sel, int64_t n_sel, int64_t* __restrict__ counts,
            const int64_t* __restrict__ off, int32_t* __restrict__ ids, int32_t* __restrict__ rows)
{
    static_assert(kSub == 64 || kSub == 32 || kSub == 16, "groups of 64, 32 or 16 lanes");
    constexpr int kPer = 64 / kSub;
    __shared__ int32_t s_node[kWaves][kPer][kStack];
    __shared__ uint8_t s_mask[kWaves][kPer][kStack][kSub];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = lane / kSub, sl = lane % kSub;
    const uint64_t group = kSub == 64 ? ~0ull : (((1ull << kSub) - 1) << (sub * kSub));
    const int64_t k_sel = ((int64_t)blockIdx.x * kWaves + wv) * kPer + sub;
    int64_t si = -1;  // this group's site, or none
    if (k_sel < n_sel) {
        si = sel[k_sel];
        // the second walk only for lists longer than a row
        if (kFill && (counts[si] < 0 || counts[si] <= kRowCap)) si = -1;
    }
    if (__ballot(si >= 0) == 0) return;  // the whole wavefront
    int nb = 0;
    int64_t b0 = 0;
    if (si >= 0) {
        b0 = ball_off[si];
        nb = (int)(ball_off[si + 1] - b0);
    }
    double bx[kLB], by[kLB], bz[kLB], r2[kLB];
    unsigned live = 0;
#pragma unroll
    for (int j = 0; j < kLB; ++j) {
        const int k = sl + kSub * j;
        bx[j] = by[j] = bz[j] = r2[j] = 0.0;
        if (si >= 0 && k < nb) {
            const double* B = balls + 4 * (b0 + k);
            bx[j] = B[0];
            by[j] = B[1];
            bz[j] = B[2];
            r2[j] = B[3] * B[3];
            live |= 1u << j;
        }
    }
    int64_t cnt = 0;
    int64_t w = (kFill && si >= 0) ? off[si] : 0;
    int sp = 0;
    if (si >= 0) {
        // every lane of the group writes the same node id, and reads back what it wrote
        s_node[wv][sub][0] = 0;
        s_mask[wv][sub][0][sl] = (uint8_t)live;
        sp = 1;
    }
    bool overflow = false;
    while (__ballot(sp > 0) != 0) {
        if (sp == 0) continue;
        --sp;
        // one group per wavefront: the node is the same in every lane
        const int32_t node = kSub == 64 ? __builtin_amdgcn_readfirstlane(s_node[wv][sub][sp]) : s_node[wv][sub][sp];
        const unsigned lm = s_mask[wv][sub][sp][sl];
        const GNode n = nodes[node];
        unsigned m = 0;
#pragma unroll
        for (int j = 0; j < kLB; ++j) {
            if (!((lm >> j) & 1u)) continue;
            const double dx = gmax3(n.lo[0] - bx[j], 0.0, bx[j] - n.hi[0]);
            const double dy = gmax3(n.lo[1] - by[j], 0.0, by[j] - n.hi[1]);
            const double dz = gmax3(n.lo[2] - bz[j], 0.0, bz[j] - n.hi[2]);
            if (dx * dx + dy * dy + dz * dz <= r2[j]) m |= 1u << j;
        }
        if ((__ballot(m != 0) & group) == 0) continue;
        if (n.b < 0) {
            for (int32_t i = n.a; i < n.a - n.b; ++i) {
                const int32_t t = order[i];
                const double* tp = T + 9 * (int64_t)t;
                const G3 a{tp[0], tp[1], tp[2]}, b{tp[3], tp[4], tp[5]}, c{tp[6], tp[7], tp[8]};
                const G3 lo{fmin(a.x, fmin(b.x, c.x)), fmin(a.y, fmin(b.y, c.y)), fmin(a.z, fmin(b.z, c.z))};
                const G3 hi{fmax(a.x, fmax(b.x, c.x)), fmax(a.y, fmax(b.y, c.y)), fmax(a.z, fmax(b.z, c.z))};
                bool hit = false;
#pragma unroll
                for (int j = 0; j < kLB; ++j) {
                    if (hit || !((m >> j) & 1u)) continue;
                    const double dx = gmax3(lo.x - bx[j], 0.0, bx[j] - hi.x);
                    const double dy = gmax3(lo.y - by[j], 0.0, by[j] - hi.y);
                    const double dz = gmax3(lo.z - bz[j], 0.0, bz[j] - hi.z);
                    if (dx * dx + dy * dy + dz * dz > r2[j]) continue;
                    hit = tri_dist2(G3{bx[j], by[j], bz[j]}, a, b, c) <= r2[j];
                }
                if ((__ballot(hit) & group) != 0) {
                    if (kFill && sl == 0) ids[w] = t;
                    if (!kFill && sl == 0 && cnt < kRowCap) rows[si * kRowCap + cnt] = t;
                    ++w;
                    ++cnt;
                }
            }
            continue;
        }
        if (sp + 2 > kStack) {
            overflow = true;
            sp = 0;
            continue;
        }
        s_node[wv][sub][sp] = n.b;
        s_mask[wv][sub][sp][sl] = (uint8_t)m;
        ++sp;
        s_node[wv][sub][sp] = node + 1;
        s_mask[wv][sub][sp][sl] = (uint8_t)m;
        ++sp;
    }
    if (!kFill && si >= 0 && sl == 0) counts[si] = overflow ? -1 : cnt;
}

// Lists that fit their row: copied to their place in the packed array.
__global__ void __launch_bounds__(64 * kWaves)
copy_rows_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ counts,
                 const int64_t* __restrict__ off, int64_t n_sites, int32_t* __restrict__ ids)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t si = (int64_t)blockIdx.x * kWaves + wv;
    if (si >= n_sites) return;
    const int64_t c = counts[si];
    if (c < 0 || c > kRowCap) return;
    for (int64_t k = lane; k < c; k += 64) ids[off[si] + k] = rows[si * kRowCap + k];
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    template <typename T>
    T* get() const { return (T*)p; }
};

void check(hipError_t e, const char* what)
{
    if (e != hipSuccess) throw Error(P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
void upload(DevBuf& b, const T* src, size_t n)
{
    check(hipMalloc(&b.p, n ? n * sizeof(T) : 16), "hipMalloc (list build)");
    if (n) check(hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (list build)");
}

}  // namespace

// Lists of job.sites on the current device, as CSR (off, ids); redo[i] is
// set for a site whose list the host must build.  The host's min / max of
// doubles (std::min / std::max on finite coordinates) equal fmin / fmax.
void gpu_build_lists(const GpuListJob& job, std::vector<int64_t>& off, std::vector<int32_t>& ids,
                     std::vector<char>& redo)
{
    const int64_t ns = (int64_t)job.sites.size();
    off.assign(ns + 1, 0);
    ids.clear();
    redo.clear();
    if (ns == 0) return;
    const std::vector<Bvh::Node>& nodes = job.bvh->nodes();
    std::vector<GNode> gn(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Bvh::Node& n = nodes[i];
        gn[i] = GNode{{n.lo.x, n.lo.y, n.lo.z}, {n.hi.x, n.hi.y, n.hi.z}, n.left_or_begin, n.right_or_count};
    }
    const std::vector<d3>& tri = *job.tri;
    std::vector<double> T(3 * tri.size());
    for (size_t i = 0; i < tri.size(); ++i) {
        T[3 * i] = tri[i].x;
        T[3 * i + 1] = tri[i].y;
        T[3 * i + 2] = tri[i].z;
    }
    DevBuf d_nodes, d_order, d_T, d_boff, d_balls, d_counts, d_off, d_ids;
    upload(d_nodes, gn.data(), gn.size());
    upload(d_order, job.bvh->order().data(), job.bvh->order().size());
    upload(d_T, T.data(), T.size());
    upload(d_boff, job.ball_off.data(), job.ball_off.size());
    upload(d_balls, job.balls.data(), job.balls.size());
    check(hipMalloc(&d_counts.p, ns * sizeof(int64_t)), "hipMalloc (list build)");
    DevBuf d_rows;
    check(hipMalloc(&d_rows.p, (size_t)ns * kRowCap * sizeof(int32_t)), "hipMalloc (list build)");
    const int block = 64 * kWaves;
    const int grid = (int)((ns + kWaves - 1) / kWaves);
    // sites by ball count: up to 16 and up to 32 balls share a wavefront
    std::vector<int32_t> sel[3];
    for (int64_t i = 0; i < ns; ++i) {
        const int64_t nb = job.ball_off[i + 1] - job.ball_off[i];
        sel[nb <= 16 ? 0 : (nb <= 32 ? 1 : 2)].push_back((int32_t)i);
    }
    DevBuf d_sel[3];
    for (int c = 0; c < 3; ++c) upload(d_sel[c], sel[c].data(), sel[c].size());
    auto launch = [&](bool fill) {
        const GNode* nd = d_nodes.get<GNode>();
        const int32_t* od = d_order.get<int32_t>();
        const double* Td = d_T.get<double>();
        const int64_t* bo = d_boff.get<int64_t>();
        const double* bl = d_balls.get<double>();
        int64_t* cn = d_counts.get<int64_t>();
        const int64_t* of = fill ? d_off.get<int64_t>() : nullptr;
        int32_t* id = fill ? d_ids.get<int32_t>() : nullptr;
        int32_t* rw = fill ? nullptr : d_rows.get<int32_t>();
        const int64_t n16 = (int64_t)sel[0].size(), n32 = (int64_t)sel[1].size(), n64 = (int64_t)sel[2].size();
        auto g = [](int64_t n, int per) { return (unsigned)((n + kWaves * per - 1) / (kWaves * per)); };
        if (fill) {
            if (n16) list_kernel<true, 16, 1><<<g(n16, 4), block>>>(nd, od, Td, bo, bl, d_sel[0].get<int32_t>(), n16, cn, of, id, rw);
            if (n32) list_kernel<true, 32, 1><<<g(n32, 2), block>>>(nd, od, Td, bo, bl, d_sel[1].get<int32_t>(), n32, cn, of, id, rw);
            if (n64) list_kernel<true, 64, kLaneBalls><<<g(n64, 1), block>>>(nd, od, Td, bo, bl, d_sel[2].get<int32_t>(), n64, cn, of, id, rw);
        } else {
            if (n16) list_kernel<false, 16, 1><<<g(n16, 4), block>>>(nd, od, Td, bo, bl, d_sel[0].get<int32_t>(), n16, cn, of, id, rw);
            if (n32) list_kernel<false, 32, 1><<<g(n32, 2), block>>>(nd, od, Td, bo, bl, d_sel[1].get<int32_t>(), n32, cn, of, id, rw);
            if (n64) list_kernel<false, 64, kLaneBalls><<<g(n64, 1), block>>>(nd, od, Td, bo, bl, d_sel[2].get<int32_t>(), n64, cn, of, id, rw);
        }
    };
    launch(false);
    check(hipGetLastError(), "list count launch");
    std::vector<int64_t> counts(ns);
    check(hipMemcpy(counts.data(), d_counts.p, ns * sizeof(int64_t), hipMemcpyDeviceToHost), "hipMemcpy (counts)");
    for (int64_t i = 0; i < ns; ++i) off[i + 1] = off[i] + (counts[i] > 0 ? counts[i] : 0);
    const int64_t total = off[ns];
    upload(d_off, off.data(), off.size());
    check(hipMalloc(&d_ids.p, total ? total * sizeof(int32_t) : 16), "hipMalloc (list build)");
    copy_rows_kernel<<<grid, block>>>(d_rows.get<int32_t>(), d_counts.get<int64_t>(), d_off.get<int64_t>(), ns,
                                      d_ids.get<int32_t>());
    check(hipGetLastError(), "list copy launch");
    bool longer = false;
    for (int64_t i = 0; i < ns && !longer; ++i) longer = counts[i] > kRowCap;
    if (longer) {
        launch(true);
        check(hipGetLastError(), "list fill launch");
    }
    ids.resize(total);
    if (total)
        check(hipMemcpy(ids.data(), d_ids.p, total * sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy (lists)");
    // a count of -1 marks a list the host must build (its range is empty)
    redo.assign(ns, 0);
    for (int64_t i = 0; i < ns; ++i) redo[i] = counts[i] < 0;
}

}  // namespace p2m
