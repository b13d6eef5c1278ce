// HIP kernels of the P2M++ query stage for gfx950 (CDNA4).
//
// Query (Sec. 3.4 of the paper), one lane per point:
//   1. Cell Locate: start at the exact nearest site of the point's seed-grid
//      cell and walk the Delaunay graph, moving to the neighbour that is
//      closest to q, until no neighbour is closer.  On the Delaunay graph a
//      local minimum is the nearest site.  The bisector predicate
//      (q - s).(t - s) > |t - s|^2 / 2 is evaluated in FP64 (half rate on
//      CDNA4 vector units), which makes the located site exact up to 1e-16
//      relative, so the lists need no query-dependent inflation.
//   2. List Search: scan the site's interception list (sorted by
//      ell = |s - c| - r), skip an entry when |q - c| - r >= d_min
//      (bounding-sphere pruning), stop when ell - |q - s| >= d_min (no later
//      entry can pass), and evaluate the exact FP32 point-triangle distance
//      for the rest; keep the strict minimum (first in list order on ties).
//   Points outside the domain box take an exact branch-and-bound over the
//   triangle BVH instead (the lists are built for cells clipped to the box).
//
// Backward (not in the paper): dL/dq = g (q - p) / d and
// dL/dv_k -= g lambda_k (q - p) / d for the closest triangle's vertices
// (envelope theorem), scattered with float32 atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.h"

namespace p2m {

namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr int kWalkCap = 4096;

// Closest point of the triangle record (a, e1, e2 with Gram entries) to q.
// Returns the squared distance and the barycentric weights (v, w) of b and c.
__device__ __forceinline__ float closest_point(const float3 q, const float4 r0, const float4 r1,
                                               const float4 r2, float& v, float& w)
{
    const float apx = q.x - r0.x, apy = q.y - r0.y, apz = q.z - r0.z;
    const float d1 = r1.x * apx + r1.y * apy + r1.z * apz;  // e1 . (q - a)
    const float d2 = r2.x * apx + r2.y * apy + r2.z * apz;  // e2 . (q - a)
    const float d3 = d1 - r0.w;                             // e1 . (q - b)
    const float d4 = d2 - r1.w;                             // e2 . (q - b)
    const float d5 = d1 - r1.w;                             // e1 . (q - c)
    const float d6 = d2 - r2.w;                             // e2 . (q - c)
    const float vc = d1 * d4 - d3 * d2;
    const float vb = d5 * d2 - d1 * d6;
    const float va = d3 * d6 - d5 * d4;
    if (d1 <= 0.f && d2 <= 0.f) {
        v = 0.f; w = 0.f;
    } else if (d3 >= 0.f && d4 <= d3) {
        v = 1.f; w = 0.f;
    } else if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) {
        v = d1 / (d1 - d3); w = 0.f;
    } else if (d6 >= 0.f && d5 <= d6) {
        v = 0.f; w = 1.f;
    } else if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) {
        v = 0.f; w = d2 / (d2 - d6);
    } else if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6)); v = 1.f - w;
    } else {
        const float den = va + vb + vc;
        if (den > 0.f && den < kInf) {
            v = vb / den; w = vc / den;
        } else {
            // zero-area triangle: best of its three edges
            const float g11 = r0.w, g12 = r1.w, g22 = r2.w;
            float t0 = g11 > 0.f ? fminf(fmaxf(d1 / g11, 0.f), 1.f) : 0.f;      // a + t e1
            float t1 = g22 > 0.f ? fminf(fmaxf(d2 / g22, 0.f), 1.f) : 0.f;      // a + t e2
            const float g33 = g11 - 2.f * g12 + g22;                            // |e2 - e1|^2
            float t2 = g33 > 0.f ? fminf(fmaxf((d2 - d1 - g12 + g11) / g33, 0.f), 1.f) : 0.f;  // b + t (c - b)
            auto dist2 = [&](float vv, float ww) {
                const float rx = apx - vv * r1.x - ww * r2.x;
                const float ry = apy - vv * r1.y - ww * r2.y;
                const float rz = apz - vv * r1.z - ww * r2.z;
                return rx * rx + ry * ry + rz * rz;
            };
            const float e0 = dist2(t0, 0.f), e1 = dist2(0.f, t1), e2 = dist2(1.f - t2, t2);
            if (e0 <= e1 && e0 <= e2) { v = t0; w = 0.f; }
            else if (e1 <= e2) { v = 0.f; w = t1; }
            else { v = 1.f - t2; w = t2; }
        }
    }
    const float rx = apx - v * r1.x - w * r2.x;
    const float ry = apy - v * r1.y - w * r2.y;
    const float rz = apz - v * r1.z - w * r2.z;
    return rx * rx + ry * ry + rz * rz;
}

__device__ __forceinline__ int seed_cell(const DevMesh& m, const float3 q)
{
    const float fx = (q.x - m.gorg[0]) * m.ginv;
    const float fy = (q.y - m.gorg[1]) * m.ginv;
    const float fz = (q.z - m.gorg[2]) * m.ginv;
    const int ix = min(max((int)floorf(fx), 0), m.gdim[0] - 1);
    const int iy = min(max((int)floorf(fy), 0), m.gdim[1] - 1);
    const int iz = min(max((int)floorf(fz), 0), m.gdim[2] - 1);
    return (iz * m.gdim[1] + iy) * m.gdim[0] + ix;
}

__device__ __forceinline__ bool in_domain(const DevMesh& m, const float3 q)
{
    return q.x >= m.dlo[0] && q.x <= m.dhi[0] && q.y >= m.dlo[1] && q.y <= m.dhi[1] &&
           q.z >= m.dlo[2] && q.z <= m.dhi[2];
}

// Cell Locate: greedy walk on the Delaunay graph from the seed site.
template <bool kCtr>
__device__ __forceinline__ int locate(const DevMesh& m, const float3 q, unsigned long long& steps,
                                      unsigned long long& adj_read)
{
    int s = m.seed[seed_cell(m, q)];
    const double qx = q.x, qy = q.y, qz = q.z;
    for (int it = 0; it < kWalkCap; ++it) {
        const float4 sp = m.site_xyz[s];
        const int4 rg = m.site_rng[s];
        const double wx = qx - (double)sp.x, wy = qy - (double)sp.y, wz = qz - (double)sp.z;
        double best = 0.0;
        int nxt = -1;
        for (int k = rg.x; k < rg.y; ++k) {
            const float4 a = m.adj[k];
            const double dx = (double)a.x - (double)sp.x;
            const double dy = (double)a.y - (double)sp.y;
            const double dz = (double)a.z - (double)sp.z;
            const double val = wx * dx + wy * dy + wz * dz - 0.5 * (dx * dx + dy * dy + dz * dz);
            if (val > best) {
                best = val;
                nxt = __float_as_int(a.w);
            }
        }
        if (kCtr) {
            steps += 1;
            adj_read += (unsigned long long)(rg.y - rg.x);
        }
        if (nxt < 0) break;
        s = nxt;
    }
    return s;
}

struct Best {
    float d2;
    int slot;
    float v, w;
};

// List Search over the located site's interception list.
template <bool kCtr>
__device__ __forceinline__ Best list_search(const DevMesh& m, const float3 q, const int s,
                                            unsigned long long& list_read, unsigned long long& exact,
                                            unsigned long long& list_len)
{
    const float4 sp = m.site_xyz[s];
    const int4 rg = m.site_rng[s];
    const float wx = q.x - sp.x, wy = q.y - sp.y, wz = q.z - sp.z;
    // |q - s| rounded up so that the early-exit bound stays conservative
    const float dqs = sqrtf(wx * wx + wy * wy + wz * wz) * 1.000001f;
    Best b{kInf, -1, 0.f, 0.f};
    float dmin = kInf;
    int e = rg.z;
    for (; e < rg.w; ++e) {
        const int2 ax = m.list_aux[e];
        if (__int_as_float(ax.y) - dqs >= dmin) break;
        const float4 c = m.list_sph[e];
        const float dx = q.x - c.x, dy = q.y - c.y, dz = q.z - c.z;
        const float lim = dmin + c.w;
        if (dx * dx + dy * dy + dz * dz >= lim * lim * 1.000001f) continue;
        const float4* r = m.tri_rec + 3 * (int64_t)ax.x;
        float v, w;
        const float d2 = closest_point(q, r[0], r[1], r[2], v, w);
        if (kCtr) exact += 1;
        if (d2 < b.d2) {
            b.d2 = d2;
            b.slot = ax.x;
            b.v = v;
            b.w = w;
            dmin = sqrtf(d2);
        }
    }
    if (kCtr) {
        list_read += (unsigned long long)(e - rg.z);
        list_len += (unsigned long long)(rg.w - rg.z);
    }
    return b;
}

// Exact branch-and-bound over the triangle BVH (points outside the domain box).
__device__ Best bvh_search(const DevMesh& m, const float3 q)
{
    Best b{kInf, -1, 0.f, 0.f};
    int stack[64];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const int ni = stack[--sp];
        const float4 lo = m.bvh[2 * ni], hi = m.bvh[2 * ni + 1];
        const float bx = fmaxf(fmaxf(lo.x - q.x, q.x - hi.x), 0.f);
        const float by = fmaxf(fmaxf(lo.y - q.y, q.y - hi.y), 0.f);
        const float bz = fmaxf(fmaxf(lo.z - q.z, q.z - hi.z), 0.f);
        if (bx * bx + by * by + bz * bz > b.d2) continue;
        const int a = __float_as_int(lo.w), c = __float_as_int(hi.w);
        if (c < 0) {
            for (int slot = a; slot < a - c; ++slot) {
                const float4* r = m.tri_rec + 3 * (int64_t)slot;
                float v, w;
                const float d2 = closest_point(q, r[0], r[1], r[2], v, w);
                if (d2 < b.d2) { b.d2 = d2; b.slot = slot; b.v = v; b.w = w; }
            }
        } else if (sp + 2 <= 64) {
            stack[sp++] = c;       // right child
            stack[sp++] = ni + 1;  // left child (popped first)
        }
    }
    return b;
}

// One query end to end: locate, list search (or fallback), outputs and,
// when fused, the gradient.  Shared by the plain and the batched kernels so
// that both give bitwise identical results.
template <bool kFused, bool kCtr>
__device__ __forceinline__ void run_query(const DevMesh& m, const int64_t i, const float* __restrict__ qp,
                                          float* __restrict__ dist, int32_t* __restrict__ tri,
                                          float* __restrict__ closest, const float* __restrict__ gdist,
                                          float* __restrict__ grad_q, float* __restrict__ grad_v,
                                          unsigned long long* __restrict__ ctr)
{
    const float3 q = make_float3(qp[3 * i], qp[3 * i + 1], qp[3 * i + 2]);
    unsigned long long steps = 0, adj_read = 0, list_read = 0, exact = 0, list_len = 0, fb = 0;
    Best b{kInf, -1, 0.f, 0.f};
    const bool finite = isfinite(q.x) && isfinite(q.y) && isfinite(q.z);
    if (finite) {
        if (in_domain(m, q)) {
            const int s = locate<kCtr>(m, q, steps, adj_read);
            b = list_search<kCtr>(m, q, s, list_read, exact, list_len);
        }
        if (b.slot < 0) {
            b = bvh_search(m, q);
            fb = 1;
        }
    }
    if (kCtr) {
        atomicAdd(&ctr[CTR_WALK_STEPS], steps);
        atomicAdd(&ctr[CTR_ADJ_READ], adj_read);
        atomicAdd(&ctr[CTR_LIST_READ], list_read);
        atomicAdd(&ctr[CTR_EXACT], exact);
        atomicAdd(&ctr[CTR_FALLBACK], fb);
        atomicAdd(&ctr[CTR_LIST_LEN], list_len);
    }
    if (b.slot < 0) {
        const float nan = __int_as_float(0x7fc00000);
        dist[i] = nan;
        if (tri) tri[i] = -1;
        if (closest) {
            closest[3 * i] = nan;
            closest[3 * i + 1] = nan;
            closest[3 * i + 2] = nan;
        }
        if (kFused && grad_q) {
            grad_q[3 * i] = 0.f;
            grad_q[3 * i + 1] = 0.f;
            grad_q[3 * i + 2] = 0.f;
        }
        return;
    }
    const float4* r = m.tri_rec + 3 * (int64_t)b.slot;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    const float d = sqrtf(b.d2);
    dist[i] = d;
    if (tri) tri[i] = m.tri_user[b.slot];
    if (closest) {
        closest[3 * i] = r0.x + b.v * r1.x + b.w * r2.x;
        closest[3 * i + 1] = r0.y + b.v * r1.y + b.w * r2.y;
        closest[3 * i + 2] = r0.z + b.v * r1.z + b.w * r2.z;
    }
    if (kFused) {
        const float g = gdist[i];
        float nx = 0.f, ny = 0.f, nz = 0.f;
        if (d > 0.f) {
            // (q - p) / d from the same residual the distance came from
            const float inv = 1.f / d;
            nx = (q.x - r0.x - b.v * r1.x - b.w * r2.x) * inv;
            ny = (q.y - r0.y - b.v * r1.y - b.w * r2.y) * inv;
            nz = (q.z - r0.z - b.v * r1.z - b.w * r2.z) * inv;
        }
        if (grad_q) {
            grad_q[3 * i] = g * nx;
            grad_q[3 * i + 1] = g * ny;
            grad_q[3 * i + 2] = g * nz;
        }
        if (grad_v && d > 0.f && g != 0.f) {
            const int4 vid = m.tri_vid[b.slot];
            const float lam[3] = {1.f - b.v - b.w, b.v, b.w};
            const int ids[3] = {vid.x, vid.y, vid.z};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float s = -g * lam[k];
                if (s == 0.f) continue;
                float* dst = grad_v + 3 * (int64_t)ids[k];
                unsafeAtomicAdd(dst, s * nx);
                unsafeAtomicAdd(dst + 1, s * ny);
                unsafeAtomicAdd(dst + 2, s * nz);
            }
        }
    }
}

template <bool kFused, bool kCtr>
__global__ void __launch_bounds__(1024) fwd_kernel(const DevMesh m, const FwdArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const int64_t i = a.perm ? (int64_t)a.perm[j] : j;
    run_query<kFused, kCtr>(m, i, a.q, a.dist, a.tri, a.closest, a.grad_dist, a.grad_q, a.grad_v, a.ctr);
}

// Persistent batched kernel: each wavefront takes work items (up to `tile`
// consecutive sorted queries of one mesh) from a global counter until none
// is left, so meshes of very different sizes share one launch.
template <bool kFused>
__global__ void __launch_bounds__(1024) batch_kernel(const DevMesh* __restrict__ meshes, const BatchArgs a)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(a.counter, 1u);
        t = (unsigned)__builtin_amdgcn_readfirstlane((int)t);
        if (t >= (unsigned)a.n_items) break;
        const int mi = __builtin_amdgcn_readfirstlane(a.item_mesh[t]);
        const int64_t first = a.item_first[t];
        const int64_t count = a.q_off[mi + 1] - a.q_off[mi];
        const int64_t last = min(first + (int64_t)a.tile, count);
        const DevMesh m = meshes[mi];
        const int32_t* perm = a.perm[mi];
        float* gv = kFused ? a.grad_v[mi] : nullptr;
        const int64_t base = a.q_off[mi];
        for (int64_t j = first + lane; j < last; j += 64) {
            const int64_t i = base + (perm ? (int64_t)perm[j] : j);
            run_query<kFused, false>(m, i, a.q, a.dist, a.tri, a.closest, a.grad_dist, a.grad_q, gv, nullptr);
        }
    }
}

__global__ void __launch_bounds__(1024) bwd_kernel(const DevMesh m, const float* __restrict__ qp, int64_t n,
                                                   const int32_t* __restrict__ tri, const float* __restrict__ gd,
                                                   float* __restrict__ grad_q, float* __restrict__ grad_v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = tri[i];
    float nx = 0.f, ny = 0.f, nz = 0.f, g = 0.f, v = 0.f, w = 0.f, d = 0.f;
    int slot = -1;
    if (t >= 0 && t < m.n_tris) {
        slot = m.tri_slot[t];
        const float3 q = make_float3(qp[3 * i], qp[3 * i + 1], qp[3 * i + 2]);
        const float4* r = m.tri_rec + 3 * (int64_t)slot;
        const float4 r0 = r[0], r1 = r[1], r2 = r[2];
        d = sqrtf(closest_point(q, r0, r1, r2, v, w));
        g = gd[i];
        if (d > 0.f) {
            const float inv = 1.f / d;
            nx = (q.x - r0.x - v * r1.x - w * r2.x) * inv;
            ny = (q.y - r0.y - v * r1.y - w * r2.y) * inv;
            nz = (q.z - r0.z - v * r1.z - w * r2.z) * inv;
        }
    }
    if (grad_q) {
        grad_q[3 * i] = g * nx;
        grad_q[3 * i + 1] = g * ny;
        grad_q[3 * i + 2] = g * nz;
    }
    if (grad_v && slot >= 0 && d > 0.f && g != 0.f) {
        const int4 vid = m.tri_vid[slot];
        const float lam[3] = {1.f - v - w, v, w};
        const int ids[3] = {vid.x, vid.y, vid.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float s = -g * lam[k];
            if (s == 0.f) continue;
            float* dst = grad_v + 3 * (int64_t)ids[k];
            unsafeAtomicAdd(dst, s * nx);
            unsafeAtomicAdd(dst + 1, s * ny);
            unsafeAtomicAdd(dst + 2, s * nz);
        }
    }
}

// ---------------------------------------------------------------- reorder
// Counting sort by the Morton rank of the point's seed cell; points outside
// the domain box or non-finite go to the last bucket.

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void reorder_count_kernel(const DevMesh m, const float* __restrict__ qp, int64_t n,
                                     uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
                                     uint32_t* __restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float3 q = make_float3(qp[3 * i], qp[3 * i + 1], qp[3 * i + 2]);
    uint32_t k = (uint32_t)m.n_cells;
    if (isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && in_domain(m, q))
        k = (uint32_t)m.cell_rank[seed_cell(m, q)];
    key[i] = k;
    rank[i] = atomicAdd(&cnt[k], 1u);
}

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

// Exclusive scan of one tile in place; the tile total goes to sums[blockIdx].
__global__ void __launch_bounds__(kScanBlock) scan_tile_kernel(uint32_t* __restrict__ data, int64_t n,
                                                               uint32_t* __restrict__ sums)
{
    __shared__ uint32_t wsum[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? data[base + k] : 0u;
        tot += v[k];
    }
    // inclusive scan of per-thread totals across the wavefront
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        uint32_t s = lane < kScanBlock / 64 ? wsum[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(s, off, 64);
            if (lane >= off) s += y;
        }
        if (lane < kScanBlock / 64) wsum[lane] = s;
    }
    __syncthreads();
    uint32_t run = inc - tot + (wid > 0 ? wsum[wid - 1] : 0u);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) data[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = wsum[kScanBlock / 64 - 1];
}

__global__ void scan_add_kernel(uint32_t* __restrict__ data, int64_t n, const uint32_t* __restrict__ sums)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) data[i] += sums[i / kScanTile];
}

__global__ void reorder_scatter_kernel(int64_t n, const uint32_t* __restrict__ key,
                                       const uint32_t* __restrict__ rank, const uint32_t* __restrict__ off,
                                       int32_t* __restrict__ perm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[off[key[i]] + rank[i]] = (int32_t)i;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Exclusive scan of n uint32 in place; tmp holds scan_levels scratch.
hipError_t exclusive_scan(uint32_t* data, int64_t n, uint32_t* tmp, hipStream_t st)
{
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    scan_tile_kernel<<<(unsigned)tiles, kScanBlock, 0, st>>>(data, n, tmp);
    if (tiles > 1) {
        hipError_t e = exclusive_scan(tmp, tiles, tmp + tiles, st);
        if (e != hipSuccess) return e;
        scan_add_kernel<<<grid_for(n, 256), 256, 0, st>>>(data, n, tmp);
    }
    return hipGetLastError();
}

int64_t scan_scratch(int64_t n)
{
    int64_t total = 0;
    while (n > 1) {
        n = (n + kScanTile - 1) / kScanTile;
        total += n;
    }
    return total + 1;
}

}  // namespace

hipError_t launch_forward(const DevMesh& m, const FwdArgs& a, int block, bool fused, bool counters,
                          hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned g = grid_for(a.n, block);
    if (fused) {
        if (counters) fwd_kernel<true, true><<<g, block, 0, st>>>(m, a);
        else fwd_kernel<true, false><<<g, block, 0, st>>>(m, a);
    } else {
        if (counters) fwd_kernel<false, true><<<g, block, 0, st>>>(m, a);
        else fwd_kernel<false, false><<<g, block, 0, st>>>(m, a);
    }
    return hipGetLastError();
}

hipError_t launch_backward(const DevMesh& m, const float* q, int64_t n, const int32_t* tri,
                           const float* g, float* grad_q, float* grad_v, int block, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    bwd_kernel<<<grid_for(n, block), block, 0, st>>>(m, q, n, tri, g, grad_q, grad_v);
    return hipGetLastError();
}

size_t reorder_workspace_bytes(int64_t n, int32_t n_cells)
{
    const int64_t buckets = (int64_t)n_cells + 1;
    return sizeof(uint32_t) * (size_t)(3 * n + buckets + scan_scratch(buckets) + 64);
}

hipError_t launch_reorder(const DevMesh& m, const float* q, int64_t n, void* ws, const int32_t** perm_out,
                          hipStream_t st)
{
    const int64_t buckets = (int64_t)m.n_cells + 1;
    uint32_t* key = (uint32_t*)ws;
    uint32_t* rank = key + n;
    int32_t* perm = (int32_t*)(rank + n);
    uint32_t* cnt = (uint32_t*)(perm + n);
    uint32_t* tmp = cnt + buckets;
    fill_u32_kernel<<<grid_for(buckets, 256), 256, 0, st>>>(cnt, 0u, buckets);
    reorder_count_kernel<<<grid_for(n, 256), 256, 0, st>>>(m, q, n, key, rank, cnt);
    hipError_t e = exclusive_scan(cnt, buckets, tmp, st);
    if (e != hipSuccess) return e;
    reorder_scatter_kernel<<<grid_for(n, 256), 256, 0, st>>>(n, key, rank, cnt, perm);
    *perm_out = perm;
    return hipGetLastError();
}

hipError_t launch_batch(const DevMesh* meshes, const BatchArgs& a, int grid, int block, bool fused,
                        hipStream_t st)
{
    if (fused) batch_kernel<true><<<grid, block, 0, st>>>(meshes, a);
    else batch_kernel<false><<<grid, block, 0, st>>>(meshes, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    fill_u32_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace p2m
