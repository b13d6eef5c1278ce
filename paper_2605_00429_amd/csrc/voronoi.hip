// The Voronoi stage (Sec. 3.2 builds the cells the walk and the interception
// lists use) on the GPU.
//
// A cell is the domain box clipped by the bisector half-spaces of nearby
// sites; it is final once no site lies closer than its own site to any of
// its corners.  Two forms:
//
//   * corner checks alone (gpu_corner_checks): the host clips; each round
//     it hands over every corner that still needs the check, over all cells
//     in progress, and gets back, for corner x with limit r^2 (1 - slack),
//     the nearest site below the limit that is not already among the
//     cell's planes, or none, or "gave up" when a budget of examined sites
//     runs out.  One lane per check.
//   * whole cells (gpu_cells): the kNN of each site (one lane per cell),
//     then one wavefront per cell for the clipping, the corners and the
//     rounds, with the checks of each round as above.
//
// Each search runs the host's depth-first search of the site kd-tree step
// for step: the same nearer-child-first order, the same pruning against the
// best distance so far and the same count of examined sites, in FP64 with
// the host's operation order and no contraction into fused multiply-adds.
// The clipping takes the host clipper's decisions on the same values: faces
// over the lanes, the surviving polygons placed by prefix sums in face
// order, cut points gathered in that order and sorted by the same keys.
// The answers, including the budget decisions that depend on the search
// order, are therefore the host's, and so are the cells, bit for bit.  A
// cell that outgrows the fixed per-cell capacity here goes back to the host.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host/build.h"
#include "host/clip_core.h"
#include "host/kdtree.h"

namespace p2m {
namespace {

constexpr int kBlock = 256;
// Stack slots per lane: a depth-first search of a tree of depth d holds at
// most d + 1 entries; median splits into leaves of <= 8 sites keep d below
// 32 for any int32 site count.
constexpr int kMaxStack = 32;

// The site kd-tree as the device reads it: one 64-byte record per node (its
// box and its links together, so a visit is one load), and the points in
// leaf order with their ids (a leaf's points are contiguous).
struct DevNode {
    double lo[3], hi[3];
    int32_t begin, end, left, right;  // point range in leaf order; left = -1 for a leaf
};
struct DevLeafPt {
    double x, y, z;
    int32_t id, pad;
};
static_assert(sizeof(DevNode) == 64 && sizeof(DevLeafPt) == 32, "tree records");

struct KdView {
    const DevNode* node;
    const DevLeafPt* leaf;  // leaf[k]: the point at position k of the leaf order
    const double* pts;      // 3 per site, by id
};

// Squared distance from q to the node's box; the host's
// max(lo - q, 0, q - hi) per axis, summed in the same order.
__host__ __device__ __forceinline__ double box_d2(const DevNode& b, double qx, double qy, double qz)
{
    const double dx = fmax(fmax(b.lo[0] - qx, 0.0), qx - b.hi[0]);
    const double dy = fmax(fmax(b.lo[1] - qy, 0.0), qy - b.hi[1]);
    const double dz = fmax(fmax(b.lo[2] - qz, 0.0), qz - b.hi[2]);
    return dx * dx + dy * dy + dz * dz;
}

__host__ __device__ __forceinline__ bool excluded(const int32_t* ex, int64_t lo, int64_t hi, int32_t p)
{
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (ex[mid] < p) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && ex[lo] == p;
}

// One check: the search of KdTree::below, with its stack at st[k * stride]
// for k < slots.  Returns the site, -1, -2 (budget spent) or -3 (stack too
// small, which the host's depth bound rules out).
__host__ __device__ inline int32_t check_one(const KdView& kd, double qx, double qy, double qz, double best,
                                             const int32_t* excl, int64_t e0, int64_t e1, int64_t budget,
                                             int32_t* st, int stride, int slots)
{
    int32_t bi = -1;
    int top = 0;
    st[0] = 0;
    top = 1;
    while (top > 0) {
        const DevNode nd = kd.node[st[--top * stride]];
        if (box_d2(nd, qx, qy, qz) >= best) continue;
        if (nd.left < 0) {
            if (budget >= 0) {
                budget -= nd.end - nd.begin;
                if (budget < 0) return -2;
            }
            for (int32_t k = nd.begin; k < nd.end; ++k) {
                const DevLeafPt pt = kd.leaf[k];
                const int32_t p = pt.id;
                const double ax = pt.x - qx, ay = pt.y - qy, az = pt.z - qz;
                const double d2 = ax * ax + ay * ay + az * az;
                if (d2 < best || (d2 == best && bi >= 0 && p < bi)) {
                    if (excluded(excl, e0, e1, p)) continue;
                    best = d2;
                    bi = p;
                }
            }
            continue;
        }
        const double dl = box_d2(kd.node[nd.left], qx, qy, qz);
        const double dr = box_d2(kd.node[nd.right], qx, qy, qz);
        // the host pushes the farther child first and takes the nearer next;
        // a pushed node is tested against the best distance when taken
        if (top + 2 > slots) return -3;
        if (dl <= dr) {
            st[top++ * stride] = nd.right;
            st[top++ * stride] = nd.left;
        } else {
            st[top++ * stride] = nd.left;
            st[top++ * stride] = nd.right;
        }
    }
    return bi;
}

__global__ __launch_bounds__(kBlock) void corner_check_kernel(KdView kd, const double* __restrict__ q,
                                                              const double* __restrict__ limit2,
                                                              const int32_t* __restrict__ list,
                                                              const int64_t* __restrict__ excl_off,
                                                              const int32_t* __restrict__ excl, int64_t n,
                                                              int64_t budget, int stack_slots, int32_t* out)
{
    extern __shared__ int32_t stack_lds[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t l = list[i];
    // slot k of this lane's stack at stack_lds[k * blockDim.x + tid]
    out[i] = check_one(kd, q[3 * i], q[3 * i + 1], q[3 * i + 2], limit2[i], excl, excl_off[l], excl_off[l + 1],
                       budget, stack_lds + threadIdx.x, (int)blockDim.x, stack_slots);
}

// ---------------------------------------------------------------------------
// Whole cells: one wavefront (one workgroup of 64 lanes) per cell.

constexpr int kW = 64;
constexpr int kFCap = 2 * kW;   // faces of a cell (two per lane)
constexpr int kVCap = 1024;     // polygon vertices over all its faces
constexpr int kCutCap = 256;    // points on a new face before merging
constexpr int kTCap = 256;      // sites clipped by (its checks' exclusion list)
constexpr int kQCap = 1024;     // corners found final
constexpr int kKnnMax = 64;
static_assert(kQCap <= kVCap, "final corners are sorted through the spare polygon buffer");

enum : int32_t { kCellActive = 1, kCellUnresolved = 2, kCellRedo = 4, kCellOk = 8 };

struct DFace {
    int32_t id, begin, count, pad;
    double cx, cy, cz, r;  // bounding sphere of the polygon
};

struct CellHdr {
    int32_t nf, nv, buf, nt;  // faces, vertices (of buffer `buf`), sites clipped by
    int32_t nq, np, flags, pad;  // final corners, pending corners
    double dk2, scale;        // kNN radius^2, box corner norm
    double px, py, pz, pad2;  // the site
};

// Per-cell state in device memory, one fixed-size slab per cell.
struct CellMem {
    CellHdr* hdr;
    DFace* face;       // 2 * kFCap per cell: the current faces and the next
    double* vert;      // 2 * 3 * kVCap: their polygons, in face order
    double* cut;       // 3 * kCutCap: points on the new face
    int32_t* tested;   // kTCap, sorted
    double* verified;  // 3 * kQCap, sorted (x, then y, then z)
    double* pend;      // 3 * kVCap: corners pending a check; at the end, all corners
    int32_t* fout;     // kFCap: at the end, the face sites
    int32_t* np;       // per cell: checks pending while in progress, else -1
    int32_t* cnt;      // per cell at the end: corners, face sites, flags
};

struct CellLds {
    int32_t idx[kVCap];
    int32_t ilist[kVCap];
    double key[kCutCap];
    int32_t kord[kCutCap];
    uint8_t dup[kVCap];
    double bd[4];
    int32_t bi[4];
};

__device__ __forceinline__ int wave_excl(int v, int& total)
{
    const int l = (int)threadIdx.x;
    int s = v;
    for (int o = 1; o < kW; o <<= 1) {
        const int t = __shfl_up(s, o, kW);
        if (l >= o) s += t;
    }
    total = __shfl(s, kW - 1, kW);
    return s - v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = kW / 2; o > 0; o >>= 1) {
        const double t = __shfl_xor(v, o, kW);
        v = v < t ? t : v;
    }
    return v;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

__device__ __forceinline__ bool less3(double ax, double ay, double az, double bx, double by, double bz)
{
    if (ax != bx) return ax < bx;
    if (ay != by) return ay < by;
    return az < bz;
}

__device__ __forceinline__ double* cur_vert(const CellMem& M, int64_t cell, int buf)
{
    return M.vert + (cell * 2 + buf) * 3 * (int64_t)kVCap;
}

__device__ __forceinline__ DFace* cur_face(const CellMem& M, int64_t cell, int buf)
{
    return M.face + (cell * 2 + buf) * (int64_t)kFCap;
}

// A face's bounding sphere: the vertices' mean and the largest distance
// from it, inflated (the host's ClipCell::seal).
__device__ void seal_face(const double* V, DFace& f)
{
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int i = 0; i < f.count; ++i) {
        const double* v = V + 3 * (f.begin + i);
        cx = cx + v[0];
        cy = cy + v[1];
        cz = cz + v[2];
    }
    const double inv = 1.0 / f.count;
    cx = cx * inv;
    cy = cy * inv;
    cz = cz * inv;
    double r2 = 0.0;
    for (int i = 0; i < f.count; ++i) {
        const double* v = V + 3 * (f.begin + i);
        const double dx = v[0] - cx, dy = v[1] - cy, dz = v[2] - cz;
        const double d = dx * dx + dy * dy + dz * dz;
        r2 = r2 < d ? d : r2;
    }
    f.cx = cx;
    f.cy = cy;
    f.cz = cz;
    f.r = sqrt(r2) * kSealInflate;
}

__device__ double max_norm2_wave(const double* V, int nv)
{
    double m = 0.0;
    for (int i = (int)threadIdx.x; i < nv; i += kW) {
        const double* v = V + 3 * i;
        const double d = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        m = m < d ? d : m;
    }
    return wave_max(m);
}

// Signed distance of vertex i of V to the plane, the host's dot(n, v) - h.
__device__ __forceinline__ double plane_sd(const double* V, int i, double nx, double ny, double nz, double hh)
{
    const double* v = V + 3 * i;
    return nx * v[0] + ny * v[1] + nz * v[2] - hh;
}

// Clips the cell by n.x <= hh (ClipCell::clip) with every lane taking part
// and h the same in all of them.  Each lane classifies its two faces
// (untouched, touching the plane, cut); prefix sums over the faces in
// their order place the surviving polygons in the other buffer and the
// cut points in the order the host gathers them; lane 0 then builds the
// new face the way the host does.  Returns 1 if the cell changed, 0 if
// not, -1 if it would outgrow the slab (the cell is then left to the host).
__device__ int clip_wave(const CellMem& M, int64_t cell, CellHdr& h, double nx, double ny, double nz, double hh,
                         int32_t id, CellLds& L)
{
    const int l = (int)threadIdx.x;
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    if (!(nn > 0)) return 0;
    const double eps = kClipEps * nn * h.scale;
    const DFace* F = cur_face(M, cell, h.buf);
    DFace* G = cur_face(M, cell, h.buf ^ 1);
    const double* V = cur_vert(M, cell, h.buf);
    double* W = cur_vert(M, cell, h.buf ^ 1);
    double* cut = M.cut + cell * 3 * (int64_t)kCutCap;

    // 0: no face, 1: untouched, 2: touching the plane, 3: cut
    int st[2], nout[2], ncut[2];
    DFace fr[2];
    for (int k = 0; k < 2; ++k) {
        const int f = l + kW * k;
        st[k] = 0;
        nout[k] = 0;
        ncut[k] = 0;
        if (f >= h.nf) continue;
        fr[k] = F[f];
        const DFace& a = fr[k];
        // strictly inside, no vertex within eps of the plane
        if (nx * a.cx + ny * a.cy + nz * a.cz - hh + nn * a.r < -eps) {
            st[k] = 1;
            nout[k] = a.count;
            continue;
        }
        bool out = false;
        int touch = 0;
        for (int i = 0; i < a.count; ++i) {
            const double sd = plane_sd(V, a.begin + i, nx, ny, nz, hh);
            out |= sd > eps;
            touch += sd >= -eps;
        }
        if (!out) {
            st[k] = 2;
            nout[k] = a.count;
            ncut[k] = touch;
            continue;
        }
        st[k] = 3;
        int cnt = 0, cuts = 0;
        const double s0 = plane_sd(V, a.begin, nx, ny, nz, hh);
        double sa = s0;
        for (int i = 0; i < a.count; ++i) {
            const double sb = i + 1 == a.count ? s0 : plane_sd(V, a.begin + i + 1, nx, ny, nz, hh);
            if (sa <= eps) {
                ++cnt;
                cuts += sa >= -eps;
            }
            if ((sa < -eps && sb > eps) || (sa > eps && sb < -eps)) {
                ++cnt;
                ++cuts;
            }
            sa = sb;
        }
        nout[k] = cnt >= 3 ? cnt : 0;
        ncut[k] = cuts;
    }
    if (!wave_any(st[0] == 3 || st[1] == 3)) return 0;

    const int keep0 = st[0] == 1 || st[0] == 2 || nout[0] > 0;
    const int keep1 = st[1] == 1 || st[1] == 2 || nout[1] > 0;
    int tk0, tk1, tv0, tv1, tc0, tc1;
    const int pk0 = wave_excl(keep0, tk0), pv0 = wave_excl(nout[0], tv0), pc0 = wave_excl(ncut[0], tc0);
    const int pk1 = wave_excl(keep1, tk1), pv1 = wave_excl(nout[1], tv1), pc1 = wave_excl(ncut[1], tc1);
    const int nkeep = tk0 + tk1, nvert = tv0 + tv1, ncuts = tc0 + tc1;
    if (nkeep + 1 > kFCap || nvert + ncuts > kVCap || ncuts > kCutCap) return -1;

    for (int k = 0; k < 2; ++k) {
        if (st[k] == 0) continue;
        const DFace& a = fr[k];
        const int fo = k ? tk0 + pk1 : pk0;
        const int vo = k ? tv0 + pv1 : pv0;
        int co = k ? tc0 + pc1 : pc0;
        if (st[k] != 3) {
            for (int i = 0; i < a.count; ++i) {
                const double* v = V + 3 * (a.begin + i);
                double* w = W + 3 * (vo + i);
                w[0] = v[0];
                w[1] = v[1];
                w[2] = v[2];
                if (st[k] == 2 && plane_sd(V, a.begin + i, nx, ny, nz, hh) >= -eps) {
                    cut[3 * co] = v[0];
                    cut[3 * co + 1] = v[1];
                    cut[3 * co + 2] = v[2];
                    ++co;
                }
            }
            DFace g = a;
            g.begin = vo;
            G[fo] = g;
            continue;
        }
        const bool keepf = nout[k] > 0;
        int o = vo;
        const double s0 = plane_sd(V, a.begin, nx, ny, nz, hh);
        double sa = s0;
        for (int i = 0; i < a.count; ++i) {
            const int ib = i + 1 == a.count ? 0 : i + 1;
            const double sb = ib == 0 ? s0 : plane_sd(V, a.begin + ib, nx, ny, nz, hh);
            const double* va = V + 3 * (a.begin + i);
            const double* vb = V + 3 * (a.begin + ib);
            if (sa <= eps) {
                if (keepf) {
                    W[3 * o] = va[0];
                    W[3 * o + 1] = va[1];
                    W[3 * o + 2] = va[2];
                    ++o;
                }
                if (sa >= -eps) {
                    cut[3 * co] = va[0];
                    cut[3 * co + 1] = va[1];
                    cut[3 * co + 2] = va[2];
                    ++co;
                }
            }
            if ((sa < -eps && sb > eps) || (sa > eps && sb < -eps)) {
                // from the inside end to the outside end, as the host does,
                // so that both faces of the edge give the same point
                const bool a_in = sa < 0;
                const double* pin = a_in ? va : vb;
                const double* pout = a_in ? vb : va;
                const double sin_ = a_in ? sa : sb, sout = a_in ? sb : sa;
                const double t = sin_ / (sin_ - sout);
                const double x = pin[0] + (pout[0] - pin[0]) * t;
                const double y = pin[1] + (pout[1] - pin[1]) * t;
                const double z = pin[2] + (pout[2] - pin[2]) * t;
                if (keepf) {
                    W[3 * o] = x;
                    W[3 * o + 1] = y;
                    W[3 * o + 2] = z;
                    ++o;
                }
                cut[3 * co] = x;
                cut[3 * co + 1] = y;
                cut[3 * co + 2] = z;
                ++co;
            }
            sa = sb;
        }
        if (keepf) {
            DFace g{a.id, vo, nout[k], 0, 0.0, 0.0, 0.0, 0.0};
            seal_face(W, g);
            G[fo] = g;
        }
    }
    __syncthreads();

    int nf_new = nkeep, nv_new = nvert;
    if (ncuts >= 3) {
        // the new face: the cut points in angular order around their mean
        if (l == 0) {
            double cx = 0.0, cy = 0.0, cz = 0.0;
            for (int i = 0; i < ncuts; ++i) {
                cx = cx + cut[3 * i];
                cy = cy + cut[3 * i + 1];
                cz = cz + cut[3 * i + 2];
            }
            const double inv = 1.0 / ncuts;
            L.bd[0] = cx * inv;
            L.bd[1] = cy * inv;
            L.bd[2] = cz * inv;
        }
        __syncthreads();
        const double cx = L.bd[0], cy = L.bd[1], cz = L.bd[2];
        const double in = 1.0 / nn;
        const double hx = nx * in, hy = ny * in, hz = nz * in;
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (fabs(hx) < 0.57) ax = 1.0;
        else if (fabs(hy) < 0.57) ay = 1.0;
        else az = 1.0;
        double ux = hy * az - hz * ay, uy = hz * ax - hx * az, uz = hx * ay - hy * ax;
        const double ui = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
        ux = ux * ui;
        uy = uy * ui;
        uz = uz * ui;
        const double wx = hy * uz - hz * uy, wy = hz * ux - hx * uz, wz = hx * uy - hy * ux;
        for (int i = l; i < ncuts; i += kW) {
            const double rx = cut[3 * i] - cx, ry = cut[3 * i + 1] - cy, rz = cut[3 * i + 2] - cz;
            L.key[i] = diamond_angle(rx * ux + ry * uy + rz * uz, rx * wx + ry * wy + rz * wz);
        }
        __syncthreads();
        for (int i = l; i < ncuts; i += kW) {
            const double ki = L.key[i];
            int r = 0;
            for (int j = 0; j < ncuts; ++j) {
                const double kj = L.key[j];
                r += kj < ki || (kj == ki && j < i);
            }
            L.kord[r] = i;
        }
        __syncthreads();
        if (l == 0) {
            const double tol2 = (kMergeTol * h.scale) * (kMergeTol * h.scale);
            const int nb = nvert;
            int cnt = 0;
            double lx = 0.0, ly = 0.0, lz = 0.0;
            for (int r = 0; r < ncuts; ++r) {
                const int i = L.kord[r];
                const double px = cut[3 * i], py = cut[3 * i + 1], pz = cut[3 * i + 2];
                if (cnt > 0) {
                    const double dx = px - lx, dy = py - ly, dz = pz - lz;
                    if (dx * dx + dy * dy + dz * dz <= tol2) continue;
                }
                W[3 * (nb + cnt)] = px;
                W[3 * (nb + cnt) + 1] = py;
                W[3 * (nb + cnt) + 2] = pz;
                lx = px;
                ly = py;
                lz = pz;
                ++cnt;
            }
            while (cnt > 1) {
                const double* a = W + 3 * (nb + cnt - 1);
                const double* b = W + 3 * nb;
                const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
                if (dx * dx + dy * dy + dz * dz <= tol2) --cnt;
                else break;
            }
            if (cnt >= 3) {
                DFace g{id, nb, cnt, 0, 0.0, 0.0, 0.0, 0.0};
                seal_face(W, g);
                G[nkeep] = g;
                L.bi[0] = nkeep + 1;
                L.bi[1] = nb + cnt;
            } else {
                L.bi[0] = nkeep;
                L.bi[1] = nb;
            }
        }
        __syncthreads();
        nf_new = L.bi[0];
        nv_new = L.bi[1];
    }
    h.nf = nf_new;
    h.nv = nv_new;
    h.buf ^= 1;
    return 1;
}

// ClipCell::corners: the polytope's vertices sorted (x, then y, then z) and
// merged within kMergeTol * scale in that order, into dst; returns the count.
// The vertices are read from the cell's slab (cached), not copied to LDS:
// the smaller LDS footprint lets four wavefronts per SIMD run instead of
// one (C2's Voronoi stage 0.55 -> 0.48 s).
__device__ int corners_wave(const double* V, int nv, double scale, CellLds& L, double* dst)
{
    const int l = (int)threadIdx.x;
    for (int i = l; i < nv; i += kW) L.dup[i] = 0;
    __syncthreads();
    for (int i = l; i < nv; i += kW) {
        const double xi = V[3 * i], yi = V[3 * i + 1], zi = V[3 * i + 2];
        int r = 0;
        for (int j = 0; j < nv; ++j) {
            const double xj = V[3 * j], yj = V[3 * j + 1], zj = V[3 * j + 2];
            const bool eq = xj == xi && yj == yi && zj == zi;
            r += less3(xj, yj, zj, xi, yi, zi) || (eq && j < i);
        }
        L.idx[r] = i;
    }
    __syncthreads();
    if (l == 0) {
        const double tol = kMergeTol * scale;
        const double tol2 = tol * tol;
        for (int i = 0; i < nv; ++i) {
            if (L.dup[i]) continue;
            const int a = L.idx[i];
            const double ax = V[3 * a], ay = V[3 * a + 1], az = V[3 * a + 2];
            for (int j = i + 1; j < nv; ++j) {
                const int b = L.idx[j];
                const double bx = V[3 * b];
                if (!(bx - ax <= tol)) break;
                if (L.dup[j]) continue;
                const double dx = bx - ax, dy = V[3 * b + 1] - ay, dz = V[3 * b + 2] - az;
                if (dx * dx + dy * dy + dz * dz <= tol2) L.dup[j] = 1;
            }
        }
    }
    __syncthreads();
    int base = 0;
    for (int i0 = 0; i0 < nv; i0 += kW) {
        const int i = i0 + l;
        const bool keep = i < nv && !L.dup[i];
        int tot;
        const int p = wave_excl(keep, tot);
        if (keep) {
            const int a = L.idx[i];
            dst[3 * (base + p)] = V[3 * a];
            dst[3 * (base + p) + 1] = V[3 * a + 1];
            dst[3 * (base + p) + 2] = V[3 * a + 2];
        }
        base += tot;
    }
    __syncthreads();
    return base;
}

__device__ bool find_sorted(const double* Q, int n, double x, double y, double z)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (less3(Q[3 * mid], Q[3 * mid + 1], Q[3 * mid + 2], x, y, z)) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && !less3(x, y, z, Q[3 * lo], Q[3 * lo + 1], Q[3 * lo + 2]);
}

// collect_pending: of the corners C (sorted), those beyond half the kNN
// radius and not found final before, kept in order, in place.
__device__ int pending_wave(double* C, int nc, double dk2, const double* Q, int nq)
{
    int base = 0;
    for (int i0 = 0; i0 < nc; i0 += kW) {
        const int i = i0 + (int)threadIdx.x;
        bool keep = false;
        double x = 0.0, y = 0.0, z = 0.0;
        if (i < nc) {
            x = C[3 * i];
            y = C[3 * i + 1];
            z = C[3 * i + 2];
            keep = !(4.0 * (x * x + y * y + z * z) <= dk2) && !find_sorted(Q, nq, x, y, z);
        }
        int tot;
        const int p = wave_excl(keep, tot);
        // every lane has read its corner before any writes: base + p <= i
        if (keep) {
            C[3 * (base + p)] = x;
            C[3 * (base + p) + 1] = y;
            C[3 * (base + p) + 2] = z;
        }
        base += tot;
    }
    __syncthreads();
    return base;
}

__device__ void put_hdr(const CellMem& M, int64_t cell, const CellHdr& h)
{
    if (threadIdx.x == 0) {
        M.hdr[cell] = h;
        M.np[cell] = (h.flags & kCellActive) ? h.np : -1;
    }
}

// k nearest sites of each cell's site (KdTree::knn: the k smallest
// (distance^2, index) pairs the same search meets, ascending).  One lane
// per cell; the list is kept sorted in place.  n_out = -1 if the search
// stack would overflow.
__global__ __launch_bounds__(kBlock) void knn_kernel(KdView kd, const int32_t* __restrict__ sites, int64_t m, int k,
                                                     int stack_slots, double* __restrict__ out_d2,
                                                     int32_t* __restrict__ out_id, int32_t* __restrict__ n_out)
{
    extern __shared__ int32_t stack_lds[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t s = sites[i];
    const double qx = kd.pts[3 * (int64_t)s], qy = kd.pts[3 * (int64_t)s + 1], qz = kd.pts[3 * (int64_t)s + 2];
    double* bd = out_d2 + i * k;
    int32_t* bi = out_id + i * k;
    int32_t* st = stack_lds + threadIdx.x;
    const int stride = (int)blockDim.x;
    int cnt = 0, top = 1;
    st[0] = 0;
    while (top > 0) {
        const DevNode nd = kd.node[st[--top * stride]];
        const double d2n = box_d2(nd, qx, qy, qz);
        if (cnt == k && d2n >= bd[k - 1]) continue;
        if (nd.left < 0) {
            for (int32_t j = nd.begin; j < nd.end; ++j) {
                const DevLeafPt pt = kd.leaf[j];
                const int32_t p = pt.id;
                if (p == s) continue;
                const double ax = pt.x - qx, ay = pt.y - qy, az = pt.z - qz;
                const double d2 = ax * ax + ay * ay + az * az;
                int pos;
                if (cnt < k) {
                    pos = cnt++;
                } else if (d2 < bd[k - 1] || (d2 == bd[k - 1] && p < bi[k - 1])) {
                    pos = k - 1;
                } else {
                    continue;
                }
                while (pos > 0 && (d2 < bd[pos - 1] || (d2 == bd[pos - 1] && p < bi[pos - 1]))) {
                    bd[pos] = bd[pos - 1];
                    bi[pos] = bi[pos - 1];
                    --pos;
                }
                bd[pos] = d2;
                bi[pos] = p;
            }
            continue;
        }
        const double dl = box_d2(kd.node[nd.left], qx, qy, qz);
        const double dr = box_d2(kd.node[nd.right], qx, qy, qz);
        if (top + 2 > stack_slots) {
            n_out[i] = -1;
            return;
        }
        if (dl <= dr) {
            st[top++ * stride] = nd.right;
            st[top++ * stride] = nd.left;
        } else {
            st[top++ * stride] = nd.left;
            st[top++ * stride] = nd.right;
        }
    }
    n_out[i] = cnt;
}

// Corner codes of the six box faces in ClipCell::init_box's order (bit 2:
// x, bit 1: y, bit 0: z; set = the box's upper end).
__constant__ int8_t kBoxFace[6][4] = {{0, 1, 3, 2}, {4, 6, 7, 5}, {0, 4, 5, 1}, {2, 3, 7, 6}, {0, 2, 6, 4}, {1, 5, 7, 3}};

// start_cell: the box, the kNN clips, the first pending corners.
__global__ __launch_bounds__(kW) void cell_start_kernel(CellMem M, const double* __restrict__ pts,
                                                        const int32_t* __restrict__ sites, double blox, double bloy,
                                                        double bloz, double bhix, double bhiy, double bhiz,
                                                        const double* __restrict__ knn_d2,
                                                        const int32_t* __restrict__ knn_id,
                                                        const int32_t* __restrict__ knn_n, int K)
{
    __shared__ CellLds L;
    const int64_t cell = blockIdx.x;
    const int l = (int)threadIdx.x;
    const int32_t s = sites[cell];
    CellHdr h{};
    h.px = pts[3 * (int64_t)s];
    h.py = pts[3 * (int64_t)s + 1];
    h.pz = pts[3 * (int64_t)s + 2];
    DFace* F = cur_face(M, cell, 0);
    double* V = cur_vert(M, cell, 0);
    if (l == 0) {
        const double lo[3] = {blox - h.px, bloy - h.py, bloz - h.pz};
        const double hi[3] = {bhix - h.px, bhiy - h.py, bhiz - h.pz};
        for (int f = 0; f < 6; ++f) {
            for (int i = 0; i < 4; ++i) {
                const int c = kBoxFace[f][i];
                double* v = V + 3 * (4 * f + i);
                v[0] = (c & 4) ? hi[0] : lo[0];
                v[1] = (c & 2) ? hi[1] : lo[1];
                v[2] = (c & 1) ? hi[2] : lo[2];
            }
            DFace g{-1 - f, 4 * f, 4, 0, 0.0, 0.0, 0.0, 0.0};
            seal_face(V, g);
            F[f] = g;
        }
        M.tested[cell * kTCap] = s;
    }
    __syncthreads();
    h.nf = 6;
    h.nv = 24;
    h.nt = 1;
    h.scale = sqrt(max_norm2_wave(V, 24));
    const int kn = knn_n[cell];
    bool redo = kn < 0;
    bool final_r = false;
    if (!redo) {
        double r2max = max_norm2_wave(V, 24);
        for (int j = 0; j < kn; ++j) {
            const double d2 = knn_d2[cell * K + j];
            // a site at distance >= 2 * max corner radius cannot cut the cell
            if (d2 >= 4.0 * r2max) {
                final_r = true;
                break;
            }
            const int32_t e = knn_id[cell * K + j];
            const double vx = pts[3 * (int64_t)e] - h.px, vy = pts[3 * (int64_t)e + 1] - h.py,
                         vz = pts[3 * (int64_t)e + 2] - h.pz;
            const int r = clip_wave(M, cell, h, vx, vy, vz, 0.5 * (vx * vx + vy * vy + vz * vz), e, L);
            if (r < 0) {
                redo = true;
                break;
            }
            if (r > 0) r2max = max_norm2_wave(cur_vert(M, cell, h.buf), h.nv);
            if (l == 0) M.tested[cell * kTCap + h.nt] = e;
            ++h.nt;
        }
    }
    if (l == 0 && !redo) {
        int32_t* t = M.tested + cell * kTCap;
        for (int i = 1; i < h.nt; ++i) {
            const int32_t v = t[i];
            int j = i;
            for (; j > 0 && t[j - 1] > v; --j) t[j] = t[j - 1];
            t[j] = v;
        }
    }
    __syncthreads();
    if (redo) {
        h.flags = kCellRedo;
    } else if (!final_r && kn == K) {
        // sites beyond the kNN radius can only cut corners farther than half of it
        h.flags = kCellActive;
        h.dk2 = knn_d2[cell * K + K - 1];
        double* pend = M.pend + cell * 3 * (int64_t)kVCap;
        const int nc = corners_wave(cur_vert(M, cell, h.buf), h.nv, h.scale, L, pend);
        h.np = pending_wave(pend, nc, h.dk2, M.verified + cell * 3 * (int64_t)kQCap, 0);
    }
    put_hdr(M, cell, h);
}

// One round's checks: check i belongs to the a-th cell in progress with
// off[a] <= i < off[a + 1]; the corner is that cell's pending corner
// i - off[a], checked as the host's CornerChecks entry ps + x with limit
// |x|^2 keep and the cell's sites so far excluded.
__global__ __launch_bounds__(kBlock) void cell_check_kernel(KdView kd, CellMem M, const int32_t* __restrict__ act,
                                                            const int64_t* __restrict__ off, int64_t n_act,
                                                            int64_t total, double keep, int64_t budget,
                                                            int stack_slots, int32_t* __restrict__ res)
{
    extern __shared__ int32_t stack_lds[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int64_t lo = 0, hi = n_act - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int64_t cell = act[lo];
    const int64_t k = i - off[lo];
    const CellHdr& h = M.hdr[cell];
    const double* x = M.pend + cell * 3 * (int64_t)kVCap + 3 * k;
    const double lim = (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) * keep;
    res[i] = check_one(kd, h.px + x[0], h.py + x[1], h.pz + x[2], lim, M.tested + cell * kTCap, 0, h.nt, budget,
                       stack_lds + threadIdx.x, (int)blockDim.x, stack_slots);
}

// apply_round for the a-th cell in progress: its checks' results in the
// order of its pending corners.
__global__ __launch_bounds__(kW) void cell_apply_kernel(CellMem M, const double* __restrict__ pts,
                                                        const int32_t* __restrict__ act,
                                                        const int64_t* __restrict__ off,
                                                        const int32_t* __restrict__ res, int64_t budget,
                                                        int32_t max_faces)
{
    __shared__ CellLds L;
    const int64_t a = blockIdx.x;
    const int64_t cell = act[a];
    const int l = (int)threadIdx.x;
    CellHdr h = M.hdr[cell];
    const int32_t* r = res + off[a];
    double* Q = M.verified + cell * 3 * (int64_t)kQCap;
    double* Pn = M.pend + cell * 3 * (int64_t)kVCap;
    bool unres = false, redo = false;
    int nfound = 0, nver = 0;
    for (int k0 = 0; k0 < h.np; k0 += kW) {
        const int k = k0 + l;
        const bool in = k < h.np;
        const int32_t f = in ? r[k] : -1;
        const bool isf = in && f >= 0, isv = in && f != -2 && f < 0;
        unres |= in && f == -2;
        int tf, tv;
        const int pf = wave_excl(isf, tf), pv = wave_excl(isv, tv);
        if (isf) L.ilist[nfound + pf] = f;
        const int qi = h.nq + nver + pv;
        if (isv && qi < kQCap) {
            Q[3 * qi] = Pn[3 * k];
            Q[3 * qi + 1] = Pn[3 * k + 1];
            Q[3 * qi + 2] = Pn[3 * k + 2];
        }
        nfound += tf;
        nver += tv;
    }
    unres = wave_any(unres);
    redo = h.nq + nver > kQCap;
    __syncthreads();
    if (!redo && nver > 0) {
        // the final corners, sorted again (all distinct), through the
        // cell's spare polygon buffer
        h.nq += nver;
        double* Tq = cur_vert(M, cell, h.buf ^ 1);
        for (int i = l; i < h.nq; i += kW) {
            Tq[3 * i] = Q[3 * i];
            Tq[3 * i + 1] = Q[3 * i + 1];
            Tq[3 * i + 2] = Q[3 * i + 2];
        }
        __syncthreads();
        for (int i = l; i < h.nq; i += kW) {
            const double xi = Tq[3 * i], yi = Tq[3 * i + 1], zi = Tq[3 * i + 2];
            int rk = 0;
            for (int j = 0; j < h.nq; ++j) {
                const double xj = Tq[3 * j], yj = Tq[3 * j + 1], zj = Tq[3 * j + 2];
                const bool eq = xj == xi && yj == yi && zj == zi;
                rk += less3(xj, yj, zj, xi, yi, zi) || (eq && j < i);
            }
            Q[3 * rk] = xi;
            Q[3 * rk + 1] = yi;
            Q[3 * rk + 2] = zi;
        }
        __syncthreads();
    }
    if (unres) h.flags |= kCellUnresolved;
    if (!redo && nfound == 0) {
        h.flags &= ~kCellActive;
        h.np = 0;
        put_hdr(M, cell, h);
        return;
    }
    if (!redo) {
        // the sites found, sorted and distinct, clipped by in that order
        for (int i = l; i < nfound; i += kW) {
            const int32_t fi = L.ilist[i];
            int rk = 0;
            for (int j = 0; j < nfound; ++j) {
                const int32_t fj = L.ilist[j];
                rk += fj < fi || (fj == fi && j < i);
            }
            L.idx[rk] = fi;
        }
        __syncthreads();
        int nu = 0;
        for (int i0 = 0; i0 < nfound; i0 += kW) {
            const int i = i0 + l;
            const bool keep = i < nfound && (i == 0 || L.idx[i] != L.idx[i - 1]);
            int tot;
            const int p = wave_excl(keep, tot);
            if (keep) L.ilist[nu + p] = L.idx[i];
            nu += tot;
        }
        __syncthreads();
        int32_t* t = M.tested + cell * kTCap;
        for (int u = 0; u < nu; ++u) {
            const int32_t f = L.ilist[u];
            const double vx = pts[3 * (int64_t)f] - h.px, vy = pts[3 * (int64_t)f + 1] - h.py,
                         vz = pts[3 * (int64_t)f + 2] - h.pz;
            const int rr = clip_wave(M, cell, h, vx, vy, vz, 0.5 * (vx * vx + vy * vy + vz * vz), f, L);
            if (rr < 0 || h.nt >= kTCap) {
                redo = true;
                break;
            }
            if (l == 0) {
                int j = h.nt;
                for (; j > 0 && t[j - 1] > f; --j) t[j] = t[j - 1];
                t[j] = f;
            }
            ++h.nt;
            __syncthreads();
        }
    }
    if (redo) {
        h.flags = kCellRedo;
    } else if (budget >= 0 && h.nf > max_faces) {
        h.flags = (h.flags | kCellUnresolved) & ~kCellActive;
        h.np = 0;
    } else {
        const int nc = corners_wave(cur_vert(M, cell, h.buf), h.nv, h.scale, L, Pn);
        h.np = pending_wave(Pn, nc, h.dk2, Q, h.nq);
    }
    put_hdr(M, cell, h);
}

// The finished cell: its corners (into the pending area) and the sites of
// its faces of positive area (ClipCell::face_ids), sorted and distinct.
__global__ __launch_bounds__(kW) void cell_final_kernel(CellMem M)
{
    __shared__ CellLds L;
    const int64_t cell = blockIdx.x;
    const int l = (int)threadIdx.x;
    const CellHdr h = M.hdr[cell];
    int32_t* cnt = M.cnt + 3 * cell;
    if (h.flags & kCellRedo) {
        if (l == 0) {
            cnt[0] = 0;
            cnt[1] = 0;
            cnt[2] = h.flags;
        }
        return;
    }
    const double* V = cur_vert(M, cell, h.buf);
    const DFace* F = cur_face(M, cell, h.buf);
    const int nc = corners_wave(V, h.nv, h.scale, L, M.pend + cell * 3 * (int64_t)kVCap);
    const double min_area = (kMinArea * h.scale) * (kMinArea * h.scale);
    int nfo = 0;
    for (int f0 = 0; f0 < h.nf; f0 += kW) {
        const int f = f0 + l;
        bool keep = false;
        int32_t id = 0;
        if (f < h.nf) {
            const DFace a = F[f];
            const double* p0 = V + 3 * a.begin;
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int i = 1; i + 1 < a.count; ++i) {
                const double* b = V + 3 * (a.begin + i);
                const double* c = V + 3 * (a.begin + i + 1);
                const double ux = b[0] - p0[0], uy = b[1] - p0[1], uz = b[2] - p0[2];
                const double vx = c[0] - p0[0], vy = c[1] - p0[1], vz = c[2] - p0[2];
                ax = ax + (uy * vz - uz * vy);
                ay = ay + (uz * vx - ux * vz);
                az = az + (ux * vy - uy * vx);
            }
            keep = 0.5 * sqrt(ax * ax + ay * ay + az * az) > min_area;
            id = a.id;
        }
        int tot;
        const int p = wave_excl(keep, tot);
        if (keep) L.ilist[nfo + p] = id;
        nfo += tot;
    }
    __syncthreads();
    for (int i = l; i < nfo; i += kW) {
        const int32_t fi = L.ilist[i];
        int rk = 0;
        for (int j = 0; j < nfo; ++j) {
            const int32_t fj = L.ilist[j];
            rk += fj < fi || (fj == fi && j < i);
        }
        L.idx[rk] = fi;
    }
    __syncthreads();
    int32_t* fo = M.fout + cell * kFCap;
    int nu = 0;
    for (int i0 = 0; i0 < nfo; i0 += kW) {
        const int i = i0 + l;
        const bool keep = i < nfo && (i == 0 || L.idx[i] != L.idx[i - 1]);
        int tot;
        const int p = wave_excl(keep, tot);
        if (keep) fo[nu + p] = L.idx[i];
        nu += tot;
    }
    if (l == 0) {
        cnt[0] = nc;
        cnt[1] = nu;
        cnt[2] = h.flags | (h.nf >= 4 ? kCellOk : 0);
    }
}

// Packs each cell's corners and face sites at the host's offsets.
__global__ __launch_bounds__(kW) void cell_pack_kernel(CellMem M, const int64_t* __restrict__ coff,
                                                       const int64_t* __restrict__ foff, double* __restrict__ corners,
                                                       int32_t* __restrict__ faces)
{
    const int64_t cell = blockIdx.x;
    const int64_t nc = coff[cell + 1] - coff[cell], nf = foff[cell + 1] - foff[cell];
    const double* src = M.pend + cell * 3 * (int64_t)kVCap;
    for (int64_t i = threadIdx.x; i < 3 * nc; i += kW) corners[3 * coff[cell] + i] = src[i];
    for (int64_t i = threadIdx.x; i < nf; i += kW) faces[foff[cell] + i] = M.fout[cell * kFCap + i];
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
    check(hipMalloc(&b.p, n ? n * sizeof(T) : 16), "hipMalloc (corner checks)");
    if (n) check(hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (corner checks)");
}

// The device copy of the last tree checked against, per host thread: the
// rounds of one build check against the same tree many times.  It is
// replaced when a thread checks against another tree (or device), and kept
// otherwise until the thread ends (a few MB; the buffers are not freed at
// exit, when the HIP runtime may already be gone).
struct TreeCache {
    int device = -1;
    uint64_t stamp = 0;
    void* node = nullptr;
    void* leaf = nullptr;
    void* pts = nullptr;
    KdView view() const { return KdView{(const DevNode*)node, (const DevLeafPt*)leaf, (const double*)pts}; }
};
thread_local TreeCache t_tree;

void release(TreeCache& c)
{
    for (void* p : {c.node, c.leaf, c.pts})
        if (p) (void)hipFree(p);
    c = TreeCache{};
}

template <typename T>
void upload_raw(void*& dst, const std::vector<T>& v)
{
    check(hipMalloc(&dst, v.empty() ? 16 : v.size() * sizeof(T)), "hipMalloc (corner checks)");
    if (!v.empty()) check(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (corner checks)");
}

const TreeCache& device_tree(const KdTree& kd)
{
    int dev = -1;
    check(hipGetDevice(&dev), "hipGetDevice");
    if (t_tree.stamp == kd.stamp() && t_tree.device == dev) return t_tree;
    if (t_tree.device >= 0) {
        // free the old copy on the device that holds it
        const int old = t_tree.device;
        if (old != dev) check(hipSetDevice(old), "hipSetDevice");
        release(t_tree);
        if (old != dev) check(hipSetDevice(dev), "hipSetDevice");
    }
    std::vector<double> box, pts;
    std::vector<int32_t> link, order;
    kd.export_flat(box, link, order, pts);
    const size_t nn = link.size() / 4, np = order.size();
    std::vector<DevNode> node(nn);
    for (size_t i = 0; i < nn; ++i) {
        DevNode& d = node[i];
        for (int a = 0; a < 3; ++a) {
            d.lo[a] = box[6 * i + a];
            d.hi[a] = box[6 * i + 3 + a];
        }
        d.begin = link[4 * i];
        d.end = link[4 * i + 1];
        d.left = link[4 * i + 2];
        d.right = link[4 * i + 3];
    }
    std::vector<DevLeafPt> leaf(np);
    for (size_t k = 0; k < np; ++k) {
        const int32_t p = order[k];
        leaf[k] = DevLeafPt{pts[3 * (size_t)p], pts[3 * (size_t)p + 1], pts[3 * (size_t)p + 2], p, 0};
    }
    TreeCache c;
    c.device = dev;
    try {
        upload_raw(c.node, node);
        upload_raw(c.leaf, leaf);
        upload_raw(c.pts, pts);
    } catch (...) {
        release(c);
        throw;
    }
    c.stamp = kd.stamp();
    t_tree = c;
    return t_tree;
}

}  // namespace

void gpu_corner_checks(const CornerChecks& job, std::vector<int32_t>& out)
{
    const int64_t n = (int64_t)job.q.size();
    out.assign(n, -1);
    if (n == 0 || job.kd->n_nodes() == 0) return;
    const int slots = job.kd->depth() + 1;
    if (slots > kMaxStack) throw Error(P2M_ERR_INTERNAL, "site tree too deep for the device corner checks");
    const TreeCache& tc = device_tree(*job.kd);
    std::vector<double> qv(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        qv[3 * i] = job.q[i].x;
        qv[3 * i + 1] = job.q[i].y;
        qv[3 * i + 2] = job.q[i].z;
    }
    DevBuf d_q, d_lim, d_list, d_eoff, d_excl, d_out;
    upload(d_q, qv.data(), qv.size());
    upload(d_lim, job.limit2.data(), job.limit2.size());
    upload(d_list, job.list.data(), job.list.size());
    upload(d_eoff, job.excl_off.data(), job.excl_off.size());
    upload(d_excl, job.excl.data(), job.excl.size());
    check(hipMalloc(&d_out.p, n * sizeof(int32_t)), "hipMalloc (corner checks)");
    const KdView kv = tc.view();
    const int64_t grid = (n + kBlock - 1) / kBlock;
    const size_t lds = (size_t)slots * kBlock * sizeof(int32_t);
    corner_check_kernel<<<(unsigned)grid, kBlock, lds>>>(kv, d_q.get<double>(), d_lim.get<double>(),
                                                         d_list.get<int32_t>(), d_eoff.get<int64_t>(),
                                                         d_excl.get<int32_t>(), n, job.budget, slots,
                                                         d_out.get<int32_t>());
    check(hipGetLastError(), "corner check launch");
    check(hipMemcpy(out.data(), d_out.p, n * sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy (corner checks)");
    for (int64_t i = 0; i < n; ++i)
        if (out[i] == -3) throw Error(P2M_ERR_INTERNAL, "device corner check stack overflow");
}


namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace {

// Device memory of one cell in a pass (its slab and its kNN list).
size_t cell_bytes(int knn)
{
    return sizeof(CellHdr) + sizeof(DFace) * 2 * kFCap + sizeof(double) * 2 * 3 * kVCap +
           sizeof(double) * 3 * kCutCap + sizeof(int32_t) * kTCap + sizeof(double) * 3 * kQCap +
           sizeof(double) * 3 * kVCap + sizeof(int32_t) * kFCap + sizeof(int32_t) * 5 + sizeof(int64_t) * 2 +
           (sizeof(double) + sizeof(int32_t)) * (size_t)knn;
}

// Cells per device pass: as many as a quarter of the free device memory
// holds (at most 32 GiB), and at least 32,768.  Every pass ends with rounds
// that only its slowest checks fill (each round lasts as long as its
// slowest check), so fewer, larger passes finish sooner: passes of 16,384
// cells took the C2 mesh's Voronoi stage from 0.70 to 0.88 s.
int64_t pass_cells(int64_t n, int knn)
{
    size_t free_b = 0, total_b = 0;
    check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const size_t budget = std::min(free_b / 4, (size_t)32 << 30);
    const int64_t cap = std::max<int64_t>(32768, (int64_t)(budget / cell_bytes(knn)));
    return std::min(n, cap);
}

// gpu_cells for one pass.
void cells_pass(const CellJob& job, CellResult& out)
{
    const int64_t m = job.n;
    out.corner_off.assign(m + 1, 0);
    out.face_off.assign(m + 1, 0);
    out.corners.clear();
    out.faces.clear();
    out.ok.assign(m, 0);
    out.unresolved.assign(m, 0);
    out.redo.assign(m, 0);
    if (m == 0) return;
    const KdTree& kd = *job.kd;
    const int K = job.knn;
    if (K < 1 || K > kKnnMax) throw Error(P2M_ERR_INTERNAL, "device cells: kNN count out of range");
    if (kd.n_nodes() == 0) throw Error(P2M_ERR_INTERNAL, "device cells: empty site tree");
    const int slots = kd.depth() + 1;
    if (slots > kMaxStack) throw Error(P2M_ERR_INTERNAL, "site tree too deep for the device cells");
    const TreeCache& tc = device_tree(kd);
    const KdView kv = tc.view();

    // one allocation, carved into the per-cell slabs and the kNN lists
    size_t total = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = total;
        total += align256(bytes);
        return at;
    };
    const size_t o_hdr = carve(sizeof(CellHdr) * m);
    const size_t o_face = carve(sizeof(DFace) * 2 * kFCap * m);
    const size_t o_vert = carve(sizeof(double) * 2 * 3 * kVCap * m);
    const size_t o_cut = carve(sizeof(double) * 3 * kCutCap * m);
    const size_t o_tested = carve(sizeof(int32_t) * kTCap * m);
    const size_t o_ver = carve(sizeof(double) * 3 * kQCap * m);
    const size_t o_pend = carve(sizeof(double) * 3 * kVCap * m);
    const size_t o_fout = carve(sizeof(int32_t) * kFCap * m);
    const size_t o_np = carve(sizeof(int32_t) * m);
    const size_t o_cnt = carve(sizeof(int32_t) * 3 * m);
    const size_t o_kd2 = carve(sizeof(double) * K * m);
    const size_t o_kid = carve(sizeof(int32_t) * K * m);
    const size_t o_kn = carve(sizeof(int32_t) * m);
    const size_t o_sites = carve(sizeof(int32_t) * m);
    const size_t o_act = carve(sizeof(int32_t) * m);
    const size_t o_off = carve(sizeof(int64_t) * (m + 1));
    const size_t o_foff = carve(sizeof(int64_t) * (m + 1));
    DevBuf mem;
    check(hipMalloc(&mem.p, total), "hipMalloc (device cells; gpu_voronoi = 0 or 2 build the cells with less device memory)");
    char* base = (char*)mem.p;
    CellMem M;
    M.hdr = (CellHdr*)(base + o_hdr);
    M.face = (DFace*)(base + o_face);
    M.vert = (double*)(base + o_vert);
    M.cut = (double*)(base + o_cut);
    M.tested = (int32_t*)(base + o_tested);
    M.verified = (double*)(base + o_ver);
    M.pend = (double*)(base + o_pend);
    M.fout = (int32_t*)(base + o_fout);
    M.np = (int32_t*)(base + o_np);
    M.cnt = (int32_t*)(base + o_cnt);
    double* knn_d2 = (double*)(base + o_kd2);
    int32_t* knn_id = (int32_t*)(base + o_kid);
    int32_t* knn_n = (int32_t*)(base + o_kn);
    int32_t* d_sites = (int32_t*)(base + o_sites);
    int32_t* d_act = (int32_t*)(base + o_act);
    int64_t* d_off = (int64_t*)(base + o_off);
    int64_t* d_foff = (int64_t*)(base + o_foff);
    check(hipMemcpy(d_sites, job.sites, sizeof(int32_t) * m, hipMemcpyHostToDevice), "hipMemcpy (device cells)");

    const size_t stack_lds = (size_t)slots * kBlock * sizeof(int32_t);
    knn_kernel<<<(unsigned)((m + kBlock - 1) / kBlock), kBlock, stack_lds>>>(kv, d_sites, m, K, slots, knn_d2,
                                                                              knn_id, knn_n);
    check(hipGetLastError(), "kNN launch");
    cell_start_kernel<<<(unsigned)m, kW>>>(M, kv.pts, d_sites, job.blo.x, job.blo.y, job.blo.z, job.bhi.x, job.bhi.y,
                                           job.bhi.z, knn_d2, knn_id, knn_n, K);
    check(hipGetLastError(), "cell start launch");

    // rounds until no cell is in progress (the host's bound: one round per site)
    const double keep = 1.0 - job.slack;
    std::vector<int32_t> np(m), act;
    std::vector<int64_t> off;
    DevBuf d_res;
    int64_t res_cap = 0;
    const size_t n_pts = kd.order().size();
    for (size_t round = 0; round <= n_pts; ++round) {
        check(hipMemcpy(np.data(), M.np, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "hipMemcpy (device cells)");
        act.clear();
        off.assign(1, 0);
        for (int64_t i = 0; i < m; ++i)
            if (np[i] >= 0) {
                act.push_back((int32_t)i);
                off.push_back(off.back() + np[i]);
            }
        if (act.empty()) break;
        const int64_t n_act = (int64_t)act.size(), n_chk = off.back();
        check(hipMemcpy(d_act, act.data(), sizeof(int32_t) * n_act, hipMemcpyHostToDevice), "hipMemcpy (device cells)");
        check(hipMemcpy(d_off, off.data(), sizeof(int64_t) * (n_act + 1), hipMemcpyHostToDevice),
              "hipMemcpy (device cells)");
        if (n_chk > res_cap) {
            if (d_res.p) check(hipFree(d_res.p), "hipFree (device cells)");
            d_res.p = nullptr;
            res_cap = std::max<int64_t>(n_chk, 2 * res_cap);
            check(hipMalloc(&d_res.p, sizeof(int32_t) * res_cap), "hipMalloc (device cells)");
        }
        if (n_chk > 0) {
            cell_check_kernel<<<(unsigned)((n_chk + kBlock - 1) / kBlock), kBlock, stack_lds>>>(
                kv, M, d_act, d_off, n_act, n_chk, keep, job.budget, slots, d_res.get<int32_t>());
            check(hipGetLastError(), "cell check launch");
        }
        cell_apply_kernel<<<(unsigned)n_act, kW>>>(M, kv.pts, d_act, d_off, d_res.get<int32_t>(), job.budget,
                                                   job.max_faces);
        check(hipGetLastError(), "cell apply launch");
    }

    cell_final_kernel<<<(unsigned)m, kW>>>(M);
    check(hipGetLastError(), "cell final launch");
    std::vector<int32_t> cnt(3 * m);
    check(hipMemcpy(cnt.data(), M.cnt, sizeof(int32_t) * 3 * m, hipMemcpyDeviceToHost), "hipMemcpy (device cells)");
    for (int64_t i = 0; i < m; ++i) {
        const int32_t fl = cnt[3 * i + 2];
        out.redo[i] = (fl & kCellRedo) != 0;
        out.ok[i] = (fl & kCellOk) != 0;
        out.unresolved[i] = (fl & kCellUnresolved) != 0;
        out.corner_off[i + 1] = out.corner_off[i] + cnt[3 * i];
        out.face_off[i + 1] = out.face_off[i] + cnt[3 * i + 1];
    }
    const int64_t nc = out.corner_off[m], nf = out.face_off[m];
    static_assert(sizeof(d3) == 3 * sizeof(double), "d3 is three packed doubles");
    out.corners.resize(nc);
    out.faces.resize(nf);
    DevBuf d_corners, d_faces;
    check(hipMalloc(&d_corners.p, sizeof(double) * 3 * std::max<int64_t>(nc, 1)), "hipMalloc (device cells)");
    check(hipMalloc(&d_faces.p, sizeof(int32_t) * std::max<int64_t>(nf, 1)), "hipMalloc (device cells)");
    check(hipMemcpy(d_off, out.corner_off.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice),
          "hipMemcpy (device cells)");
    check(hipMemcpy(d_foff, out.face_off.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice),
          "hipMemcpy (device cells)");
    cell_pack_kernel<<<(unsigned)m, kW>>>(M, d_off, d_foff, d_corners.get<double>(), d_faces.get<int32_t>());
    check(hipGetLastError(), "cell pack launch");
    if (nc) check(hipMemcpy(out.corners.data(), d_corners.p, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost),
                  "hipMemcpy (device cells)");
    if (nf) check(hipMemcpy(out.faces.data(), d_faces.p, sizeof(int32_t) * nf, hipMemcpyDeviceToHost),
                  "hipMemcpy (device cells)");
}

}  // namespace

void gpu_cells(const CellJob& job, CellResult& out)
{
    const int64_t per = job.pass > 0 ? std::min(job.n, job.pass) : (job.n > 0 ? pass_cells(job.n, job.knn) : 1);
    if (job.n <= per) {
        cells_pass(job, out);
        return;
    }
    out.corner_off.assign(1, 0);
    out.face_off.assign(1, 0);
    out.corners.clear();
    out.faces.clear();
    out.ok.clear();
    out.unresolved.clear();
    out.redo.clear();
    for (int64_t c0 = 0; c0 < job.n; c0 += per) {
        CellJob part = job;
        part.sites = job.sites + c0;
        part.n = std::min(per, job.n - c0);
        CellResult r;
        cells_pass(part, r);
        const int64_t cb = out.corner_off.back(), fb = out.face_off.back();
        for (int64_t i = 0; i < part.n; ++i) {
            out.corner_off.push_back(cb + r.corner_off[i + 1]);
            out.face_off.push_back(fb + r.face_off[i + 1]);
        }
        out.corners.insert(out.corners.end(), r.corners.begin(), r.corners.end());
        out.faces.insert(out.faces.end(), r.faces.begin(), r.faces.end());
        out.ok.insert(out.ok.end(), r.ok.begin(), r.ok.end());
        out.unresolved.insert(out.unresolved.end(), r.unresolved.begin(), r.unresolved.end());
        out.redo.insert(out.redo.end(), r.redo.begin(), r.redo.end());
    }
}

}  // namespace p2m
