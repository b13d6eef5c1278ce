// HIP kernels of the P2M++ query stage for gfx950 (CDNA4).
//
// Query (Sec. 3.4 of the paper), one lane per point:
//   1. Cell Locate: start at the exact nearest site of the point's seed-grid
//      cell and walk the Delaunay graph, moving to a neighbour closer to q
//      until none is closer.  On the Delaunay graph a local minimum is the
//      nearest site.  The bisector predicate (q - s).(t - s) > |t - s|^2 / 2
//      is decided exactly: in FP32 when its rounding bound allows, else in
//      FP64, so the lists need no query-dependent inflation.
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

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "device.h"

namespace p2m {

namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr int kWalkCap = 4096;

// Squared distance from q to the triangle (a, a + e1, a + e2), float32, as
// the search uses it to compare triangles: q is classified against the
// triangle's vertex, edge and face regions (Ericson, Real-Time Collision
// Detection, Sec. 5.1.5), all regions evaluated and resolved with selects
// so that lanes in different regions do not diverge; reciprocals use the
// 1-ulp hardware instruction.  In the face region the distance is the
// plane distance (n.(q - a))^2 / |n|^2 with n = e1 x e2: on long thin
// triangles (a fan of 512 slivers around a cap centre) the barycentric
// products cancel and the residual q - a - v e1 - w e2 keeps an in-plane
// error of up to 2e-4 of the edge length, where the plane distance stays
// within a few 1e-6.  Also returns the barycentric weights (v, w) of b and c.
__device__ __forceinline__ float closest_point(const float3 q, const float3 a, const float3 e1, const float3 e2,
                                               const float g12, float& v, float& w)
{
    const float4 r0 = make_float4(a.x, a.y, a.z, e1.x * e1.x + e1.y * e1.y + e1.z * e1.z);
    const float4 r1 = make_float4(e1.x, e1.y, e1.z, g12);
    const float4 r2 = make_float4(e2.x, e2.y, e2.z, e2.x * e2.x + e2.y * e2.y + e2.z * e2.z);
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
    const float den = va + vb + vc;
    const float e43 = d4 - d3, e56 = d5 - d6;
    // face region, then each edge / vertex region in increasing priority
    // every candidate computed, then selected: no branches (an unselected
    // reciprocal may be inf or NaN and is discarded)
    const float inv = __builtin_amdgcn_rcpf(den);
    const float t_bc = e43 * __builtin_amdgcn_rcpf(e43 + e56);
    const float t_ca = d2 * __builtin_amdgcn_rcpf(d2 - d6);
    const float t_ab = d1 * __builtin_amdgcn_rcpf(d1 - d3);
    const bool r_bc = va <= 0.f && e43 >= 0.f && e56 >= 0.f;  // edge bc
    const bool r_ca = vb <= 0.f && d2 >= 0.f && d6 <= 0.f;    // edge ca
    const bool r_c = d6 >= 0.f && d5 <= d6;                   // vertex c
    const bool r_ab = vc <= 0.f && d1 >= 0.f && d3 <= 0.f;    // edge ab
    const bool r_b = d3 >= 0.f && d4 <= d3;                   // vertex b
    const bool r_a = d1 <= 0.f && d2 <= 0.f;                  // vertex a
    float vv = vb * inv, ww = vc * inv;
    vv = r_bc ? 1.f - t_bc : vv;
    ww = r_bc ? t_bc : ww;
    vv = r_ca ? 0.f : vv;
    ww = r_ca ? t_ca : ww;
    vv = r_c ? 0.f : vv;
    ww = r_c ? 1.f : ww;
    vv = r_ab ? t_ab : vv;
    ww = r_ab ? 0.f : ww;
    vv = r_b ? 1.f : vv;
    ww = r_b ? 0.f : ww;
    vv = r_a ? 0.f : vv;
    ww = r_a ? 0.f : ww;
    const bool face = !(r_bc || r_ca || r_c || r_ab || r_b || r_a);
    const bool flat = !(den > 0.f && den < kInf);
    if (face && flat) {
        // zero-area triangle: best of its three edges (rare)
        const float g11 = r0.w, g12 = r1.w, g22 = r2.w;
        const float t0 = g11 > 0.f ? fminf(fmaxf(d1 / g11, 0.f), 1.f) : 0.f;      // a + t e1
        const float t1 = g22 > 0.f ? fminf(fmaxf(d2 / g22, 0.f), 1.f) : 0.f;      // a + t e2
        const float g33 = g11 - 2.f * g12 + g22;                                  // |e2 - e1|^2
        const float t2 = g33 > 0.f ? fminf(fmaxf((d2 - d1 - g12 + g11) / g33, 0.f), 1.f) : 0.f;
        auto dist2 = [&](float a1, float a2) {
            const float rx = apx - a1 * r1.x - a2 * r2.x;
            const float ry = apy - a1 * r1.y - a2 * r2.y;
            const float rz = apz - a1 * r1.z - a2 * r2.z;
            return rx * rx + ry * ry + rz * rz;
        };
        const float e0 = dist2(t0, 0.f), e1 = dist2(0.f, t1), e2 = dist2(1.f - t2, t2);
        if (e0 <= e1 && e0 <= e2) { vv = t0; ww = 0.f; }
        else if (e1 <= e2) { vv = 0.f; ww = t1; }
        else { vv = 1.f - t2; ww = t2; }
    }
    v = vv;
    w = ww;
    if (face && !flat) {
        // plane distance: n = e1 x e2, h = n . (q - a)
        const float nx = r1.y * r2.z - r1.z * r2.y;
        const float ny = r1.z * r2.x - r1.x * r2.z;
        const float nz = r1.x * r2.y - r1.y * r2.x;
        const float h = nx * apx + ny * apy + nz * apz;
        return h * h * __builtin_amdgcn_rcpf(nx * nx + ny * ny + nz * nz);
    }
    const float rx = apx - vv * r1.x - ww * r2.x;
    const float ry = apy - vv * r1.y - ww * r2.y;
    const float rz = apz - vv * r1.z - ww * r2.z;
    return rx * rx + ry * ry + rz * rz;
}

// Closest point of the triangle (a, b, c) to q in FP64, for the one
// triangle a query's search has chosen: the same region classification on
// the exact float32 inputs promoted to double, so that the reported
// distance, closest point and gradient direction are those of the chosen
// triangle to ~1e-15 relative, even for points within 1e-7 of the surface.
// Returns the squared distance and the barycentric weights (v, w) of b
// and c.
__device__ __forceinline__ double closest_point64(const double3 q, const double3 a, const double3 b, const double3 c,
                                               double& v, double& w)
{
    const double e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const double e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    const double apx = q.x - a.x, apy = q.y - a.y, apz = q.z - a.z;
    const double g11 = e1x * e1x + e1y * e1y + e1z * e1z;
    const double g22 = e2x * e2x + e2y * e2y + e2z * e2z;
    const double g12 = e1x * e2x + e1y * e2y + e1z * e2z;
    const double d1 = e1x * apx + e1y * apy + e1z * apz;
    const double d2 = e2x * apx + e2y * apy + e2z * apz;
    const double d3 = d1 - g11, d4 = d2 - g12, d5 = d1 - g12, d6 = d2 - g22;
    double vv, ww;
    if (d1 <= 0.0 && d2 <= 0.0) {                               // vertex a
        vv = 0.0; ww = 0.0;
    } else if (d3 >= 0.0 && d4 <= d3) {                         // vertex b
        vv = 1.0; ww = 0.0;
    } else {
        const double vc = d1 * d4 - d3 * d2;
        const double vb = d5 * d2 - d1 * d6;
        const double va = d3 * d6 - d5 * d4;
        if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {             // edge ab
            vv = d1 / (d1 - d3); ww = 0.0;
        } else if (d6 >= 0.0 && d5 <= d6) {                    // vertex c
            vv = 0.0; ww = 1.0;
        } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {       // edge ca
            vv = 0.0; ww = d2 / (d2 - d6);
        } else if (va <= 0.0 && d4 - d3 >= 0.0 && d5 - d6 >= 0.0) {  // edge bc
            const double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            vv = 1.0 - t; ww = t;
        } else {
            const double den = va + vb + vc;
            if (den > 0.0 && den < 1e308) {                     // face
                vv = vb / den; ww = vc / den;
            } else {
                // zero-area triangle: best of its three edges
                const double t0 = g11 > 0.0 ? fmin(fmax(d1 / g11, 0.0), 1.0) : 0.0;
                const double t1 = g22 > 0.0 ? fmin(fmax(d2 / g22, 0.0), 1.0) : 0.0;
                const double g33 = g11 - 2.0 * g12 + g22;
                const double t2 = g33 > 0.0 ? fmin(fmax((d2 - d1 - g12 + g11) / g33, 0.0), 1.0) : 0.0;
                auto dist2 = [&](double a1, double a2) {
                    const double rx = apx - a1 * e1x - a2 * e2x;
                    const double ry = apy - a1 * e1y - a2 * e2y;
                    const double rz = apz - a1 * e1z - a2 * e2z;
                    return rx * rx + ry * ry + rz * rz;
                };
                const double s0 = dist2(t0, 0.0), s1 = dist2(0.0, t1), s2 = dist2(1.0 - t2, t2);
                if (s0 <= s1 && s0 <= s2) { vv = t0; ww = 0.0; }
                else if (s1 <= s2) { vv = 0.0; ww = t1; }
                else { vv = 1.0 - t2; ww = t2; }
            }
        }
    }
    v = vv;
    w = ww;
    const double rx = apx - vv * e1x - ww * e2x;
    const double ry = apy - vv * e1y - ww * e2y;
    const double rz = apz - vv * e1z - ww * e2z;
    return rx * rx + ry * ry + rz * rz;
}

// The chosen triangle's exact closest point: its caller vertices from the
// vertex array (float32 inputs, exact in double), closest_point64, and the
// point p = a + v (b - a) + w (c - a), all in FP64.
struct Final {
    double d2, v, w;
    double3 p;
};

__device__ __forceinline__ Final finalize(const DevMesh& m, const float3 q, const int user)
{
    const int4 vid = gload(m.tri_vid + user);
    const float4 fa = gload(m.verts + vid.x), fb = gload(m.verts + vid.y), fc = gload(m.verts + vid.z);
    const double3 a = make_double3(fa.x, fa.y, fa.z), b = make_double3(fb.x, fb.y, fb.z),
                  c = make_double3(fc.x, fc.y, fc.z);
    Final f;
    f.d2 = closest_point64(make_double3(q.x, q.y, q.z), a, b, c, f.v, f.w);
    f.p = make_double3(a.x + f.v * (b.x - a.x) + f.w * (c.x - a.x), a.y + f.v * (b.y - a.y) + f.w * (c.y - a.y),
                       a.z + f.v * (b.z - a.z) + f.w * (c.z - a.z));
    return f;
}

// The same test on a triangle record (|e1|^2, |e2|^2 in the record are not
// used: both paths recompute them identically, so results match bitwise).
__device__ __forceinline__ float closest_point_rec(const float3 q, const float4* r, float& v, float& w)
{
    const float4 r0 = gload(r), r1 = gload(r + 1), r2 = gload(r + 2);
    return closest_point(q, make_float3(r0.x, r0.y, r0.z), make_float3(r1.x, r1.y, r1.z),
                         make_float3(r2.x, r2.y, r2.z), r1.w, v, w);
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

// FP64 value of the bisector predicate (q - s).(t - s) - |t - s|^2 / 2 for
// every neighbour t of s; the best positive one, or -1.
__device__ __noinline__ int best_neighbour_f64(const float4* __restrict__ adj, const float3 q, const float4 sp,
                                               const int4 rg)
{
    const double sx = sp.x, sy = sp.y, sz = sp.z;
    const double wx = (double)q.x - sx, wy = (double)q.y - sy, wz = (double)q.z - sz;
    double best = 0.0;
    int nxt = -1;
    for (int k = rg.x; k < rg.y; ++k) {
        const float4 a = gload(adj + k);
        const double dx = (double)a.x - sx, dy = (double)a.y - sy, dz = (double)a.z - sz;
        const double val = wx * dx + wy * dy + wz * dz - 0.5 * (dx * dx + dy * dy + dz * dz);
        if (val > best) {
            best = val;
            nxt = __float_as_int(a.w);
        }
    }
    return nxt;
}

// Cell Locate: greedy walk on the Delaunay graph from the seed site.  The
// predicate is evaluated in FP32 with a bound on its rounding error; a step
// is taken only on a certified improvement, and when no neighbour is
// certified better but one lies within the bound the site's neighbours are
// re-evaluated in FP64.  The walk therefore stops exactly where an FP64 walk
// would (a local, hence global, minimum on the Delaunay graph).  A walk
// that has not stopped after kWalkCap steps (not possible on a valid
// Delaunay graph) returns -1 and is counted: the caller then answers the
// query by the exact BVH search.
template <bool kCtr>
__device__ __forceinline__ int locate(const DevMesh& m, const float3 q, unsigned long long& steps,
                                      unsigned long long& adj_read, unsigned long long& capped,
                                      const Touch& tch, float4& sp_out, int4& rg_out)
{
    const int cell = seed_cell(m, q);
    int s = gload(m.seed + cell);
    if (kCtr && tch.seed) tch.seed[cell] = 1;
    for (int it = 0; it < kWalkCap; ++it) {
        const float4 sp = gload(m.site_rec + 2 * s);
        const int4 rg = __builtin_bit_cast(int4, gload(m.site_rec + 2 * s + 1));
        if (kCtr && tch.site) tch.site[s] = 1;
        sp_out = sp;
        rg_out = rg;
        const float wx = q.x - sp.x, wy = q.y - sp.y, wz = q.z - sp.z;
        const float wn = fabsf(wx) + fabsf(wy) + fabsf(wz);
        float best = 0.f;
        int nxt = -1;
        bool unsure = false;
        for (int k0 = rg.x; k0 < rg.y; k0 += 4) {
            float4 a[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) a[k] = gload(m.adj + (min(k0 + k, rg.y - 1)));
            if (kCtr && tch.adj)
                for (int k = 0; k < 4; ++k) tch.adj[min(k0 + k, rg.y - 1)] = 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float dx = a[k].x - sp.x, dy = a[k].y - sp.y, dz = a[k].z - sp.z;
                const float dn = fabsf(dx) + fabsf(dy) + fabsf(dz);
                const float val = wx * dx + wy * dy + wz * dz - 0.5f * (dx * dx + dy * dy + dz * dz);
                // |error| <= ~8 u (|w|_1 |d|_1 + |d|_1^2); 2^-19 leaves a 4x margin
                const float tol = 1.9073486e-6f * dn * (wn + dn);
                unsure |= fabsf(val) <= tol;
                // repeated tail entries give the same value: never a strict improvement
                if (val - tol > best) {
                    best = val - tol;
                    nxt = __float_as_int(a[k].w);
                }
            }
        }
        if (kCtr) {
            steps += 1;
            adj_read += (unsigned long long)(rg.y - rg.x);
        }
        if (nxt < 0 && unsure) nxt = best_neighbour_f64(m.adj, q, sp, rg);
        if (nxt < 0) return s;
        s = nxt;
    }
    if (kCtr) capped += 1;
    return -1;
}

// Cell Locate in the octree decomposition: descend from the root to the leaf
// box holding q (children split at the parent's centre, q >= centre taking
// the upper half, as the host built them; every split plane is exact in
// float32).  The caller has checked that q lies in the root box.
__device__ __forceinline__ int octree_locate(const DevMesh& m, const float3 q, unsigned long long& steps)
{
    float cx = m.oroot[0], cy = m.oroot[1], cz = m.oroot[2], h = m.oroot[3];
    int v = gload(m.oct);
    while (v >= 0) {
        h *= 0.5f;
        const bool ux = q.x >= cx, uy = q.y >= cy, uz = q.z >= cz;
        cx = ux ? cx + h : cx - h;
        cy = uy ? cy + h : cy - h;
        cz = uz ? cz + h : cz - h;
        v = gload(m.oct + (v + ((int)ux | ((int)uy << 1) | ((int)uz << 2))));
        steps += 1;
    }
    return -v - 1;
}

// Best triangle so far: idx >= 0 is a list entry, idx <= -2 the triangle
// slot -(idx + 2) (fallback search), -1 none.
struct Best {
    float d2;
    int idx;
    float v, w;
};

// Counts of one query for the instrumented forward.
struct QueryCounts {
    unsigned long long steps = 0, adj_read = 0, list_read = 0, exact = 0, list_len = 0, capped = 0;
};

// List Search over the located site's interception list.  Entries are
// fetched kChunk at a time (all loads issued before any is used) so that
// the scan keeps several requests in flight despite its data-dependent exit.
constexpr int kChunk = 4;

// One entry of a List Search (entry idx, bounding sphere c): false when the
// sorted exit fires.  Lists are sorted by ell = |s - c| - r, so no later
// entry can beat d_min once ell - |q - s| >= d_min (triangle inequality).
// ell is recomputed from (c, r) rather than loaded, which keeps the scan to
// one 16-byte load per entry.  The two terms are pulled apart by 1e-6
// relative, more than the float32 rounding of the differences, the sum of
// squares, the square root and the subtraction together, so the value never
// exceeds the exact ell of the same float32 values by which the lists were
// sorted.  That margin also covers the hardware square root (within 1 ulp),
// one instruction where the correctly rounded one takes about sixteen, on
// every entry scanned.  An entry past the sphere prune is tested exactly with its record
// (rec(f1, f2, f3): first vertex and ell, first edge and e1.e2, second
// edge and id).  Both scans (per lane, and per group of lanes sharing a
// site) run this one function, so they decide alike.
template <class Rec>
__device__ __forceinline__ bool scan_entry(const float3 q, const float4 sp, const float dqs, const float4 c,
                                           const int idx, float& dmin, Best& b, unsigned long long& exact,
                                           Rec rec)
{
    const float ux = sp.x - c.x, uy = sp.y - c.y, uz = sp.z - c.z;
    const float ell = __builtin_amdgcn_sqrtf(ux * ux + uy * uy + uz * uz) * (1.f - 1e-6f) - c.w * (1.f + 1e-6f);
    if (ell - dqs >= dmin) return false;
    const float dx = q.x - c.x, dy = q.y - c.y, dz = q.z - c.z;
    const float lim = dmin + c.w;
    if (dx * dx + dy * dy + dz * dz >= lim * lim * 1.000001f) return true;
    float4 f1, f2, f3;
    rec(f1, f2, f3);
    float v, w;
    const float d2 = closest_point(q, make_float3(f1.x, f1.y, f1.z), make_float3(f2.x, f2.y, f2.z),
                                   make_float3(f3.x, f3.y, f3.z), f2.w, v, w);
    exact += 1;
    if (d2 < b.d2) {
        b.d2 = d2;
        b.idx = idx;
        b.v = v;
        b.w = w;
        dmin = sqrtf(d2);
    }
    return true;
}

// Scans at most `budget` entries of the list of the site whose record is
// (sp, rg); if the list is not done by then, *resume is set to the next
// entry (else -1).  The first st_cnt entries' spheres are read from LDS
// (st + st_off, staged by stage_spheres), the rest from the sphere array;
// the two parts are scanned by separate loops so that every load has one
// address space.
template <bool kCtr>
__device__ __forceinline__ Best list_search(const DevMesh& m, const float3 q, const float4 sp, const int4 rg,
                                            const int budget, int* resume, QueryCounts& n, const Touch& tch,
                                            const float4* st = nullptr, const int st_off = 0, const int st_cnt = 0)
{
    const float wx = q.x - sp.x, wy = q.y - sp.y, wz = q.z - sp.z;
    // |q - s| rounded up so that the early-exit bound stays conservative
    const float dqs = sqrtf(wx * wx + wy * wy + wz * wz) * 1.000001f;
    Best b{kInf, -1, 0.f, 0.f};
    float dmin = kInf;
    int stop = rg.w;
    *resume = -1;
    // Tests entries e .. e + kChunk - 1 (below `end`) given their spheres;
    // false once the scan is over (stop set).
    auto scan_chunk = [&](const int e, const int end, const float4 (&c)[kChunk]) -> bool {
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (e + k >= end) return e + k < stop;
            const int64_t idx = e + k;
            auto rec = [&](float4& f1, float4& f2, float4& f3) {
                f1 = gload(m.list_rec + 3 * idx);
                f2 = gload(m.list_rec + 3 * idx + 1);
                f3 = gload(m.list_rec + 3 * idx + 2);
                if (kCtr && tch.rec) tch.rec[idx] = 1;
            };
            unsigned long long ex = 0;
            const bool go = scan_entry(q, sp, dqs, c[k], (int)idx, dmin, b, ex, rec);
            if (kCtr) n.exact += ex;
            if (!go) {
                stop = e + k;
                return false;
            }
        }
        return true;
    };
    int e = rg.z;
    // the staged part, from LDS (all kChunk loads issued before any is used)
    const int lds_end = rg.z + min(st_cnt, rg.w - rg.z);
    bool more = true;
    for (; more && e < lds_end; e += kChunk) {
        float4 c[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) c[k] = st[st_off + min(e + k, lds_end - 1) - rg.z];
        more = scan_chunk(e, lds_end, c);
    }
    // the rest, from the sphere array; an entry's record (a, e1, e2) is read
    // for an exact test only
    for (e = lds_end; more && e < stop; e += kChunk) {
        if (e - rg.z >= budget) {
            *resume = e;
            stop = e;
            break;
        }
        float4 c[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int idx = min(e + k, rg.w - 1);
            c[k] = gload(m.list_sph + idx);
            if (kCtr && tch.sph) tch.sph[idx] = 1;
        }
        more = scan_chunk(e, stop, c);
    }
    if (kCtr) {
        n.list_read += (unsigned long long)(stop - rg.z);
        n.list_len += (unsigned long long)(rg.w - rg.z);
    }
    return b;
}

// A lane scans its list alone for at most kSerialBudget entries; the lists
// of the lanes that are not done by then (the cell of a central auxiliary
// site holds nearly every triangle, and the triangle-inequality exit cannot
// fire inside it) are finished by the whole wavefront, one after the other,
// so that one lane walking thousands of entries does not hold its 63
// neighbours idle for as long.
constexpr int kSerialBudget = 512;
constexpr int kWaveChunk = 2;

// Argmin of (d2, list index) over the wavefront; ties go to the lower index.
__device__ __forceinline__ Best wave_argmin(Best b)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float d2 = __shfl_xor(b.d2, off, 64);
        const int idx = __shfl_xor(b.idx, off, 64);
        const float v = __shfl_xor(b.v, off, 64);
        const float w = __shfl_xor(b.w, off, 64);
        const bool take = d2 < b.d2 || (d2 == b.d2 && (unsigned)idx < (unsigned)b.idx);
        if (take) b = Best{d2, idx, v, w};
    }
    return b;
}

__device__ __forceinline__ float wave_min(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fminf(x, __shfl_xor(x, off, 64));
    return x;
}

// The rest of one query's List Search, from entry `from` on with the d_min
// found so far, by the whole wavefront (q and the located site s are the
// same in every lane): lane l takes entries base + l, base + 64 + l, ... of
// each chunk; d_min is shared after every chunk, and the scan stops once
// the chunk's last entry has ell - |q - s| >= d_min (the list is sorted by
// ell, so no later entry can do better).  Every lane must call it.
// Result of the wavefront's scan: the best entry and, for the instrumented
// forward, the exact tests made and entries read.
struct WaveScan {
    Best b;
    unsigned exact, read;
};

template <bool kCtr>
__device__ __noinline__ WaveScan list_search_wave(const float4* __restrict__ site_rec, const float4* __restrict__ list_sph,
                                              const float4* __restrict__ list_rec, const float3 q, const int s,
                                              const int from,
                                              const float dmin0, uint8_t* __restrict__ sph_flag,
                                              uint8_t* __restrict__ rec_flag)
{
    const int lane = threadIdx.x & 63;
    const float4 sp = gload(site_rec + 2 * s);
    const int4 rg = __builtin_bit_cast(int4, gload(site_rec + 2 * s + 1));
    const float wx = q.x - sp.x, wy = q.y - sp.y, wz = q.z - sp.z;
    const float dqs = sqrtf(wx * wx + wy * wy + wz * wz) * 1.000001f;
    Best b{kInf, -1, 0.f, 0.f};
    unsigned exact = 0;
    float dmin = dmin0;  // wave-uniform between chunks
    int end = rg.w;
    for (int base = from; base < rg.w; base += 64 * kWaveChunk) {
        float4 c[kWaveChunk], a[kWaveChunk];
#pragma unroll
        for (int k = 0; k < kWaveChunk; ++k) {
            const int idx = min(base + 64 * k + lane, rg.w - 1);
            c[k] = gload(list_sph + idx);
            a[k] = gload(list_rec + (3 * (int64_t)idx));
            if (kCtr && sph_flag) {
                sph_flag[idx] = 1;
                rec_flag[idx] = 1;
            }
        }
        float dl = fminf(dmin, sqrtf(b.d2));
#pragma unroll
        for (int k = 0; k < kWaveChunk; ++k) {
            const int e = base + 64 * k + lane;
            bool tested = false;
            if (e < rg.w && a[k].w - dqs < dl) {
                const float dx = q.x - c[k].x, dy = q.y - c[k].y, dz = q.z - c[k].z;
                const float lim = dl + c[k].w;
                if (dx * dx + dy * dy + dz * dz < lim * lim * 1.000001f) {
                    const float4 f2 = gload(list_rec + (3 * (int64_t)e + 1)), f3 = gload(list_rec + (3 * (int64_t)e + 2));
                    float v, w;
                    const float d2 = closest_point(q, make_float3(a[k].x, a[k].y, a[k].z),
                                                   make_float3(f2.x, f2.y, f2.z), make_float3(f3.x, f3.y, f3.z),
                                                   f2.w, v, w);
                    tested = true;
                    if (d2 < b.d2) {
                        b = Best{d2, e, v, w};
                        dl = fminf(dl, sqrtf(d2));
                    }
                }
            }
            if (kCtr) exact += (unsigned)__popcll(__ballot(tested));
        }
        dmin = wave_min(dl);
        // lane 63 loaded the chunk's last entry in its last slot (indices
        // past the list's end are clamped to it): its ell decides the exit
        const int last = min(base + 64 * kWaveChunk, rg.w) - 1;
        const float ell_last = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[kWaveChunk - 1].w), 63));
        if (ell_last - dqs >= dmin) {
            end = last + 1;
            break;
        }
    }
    WaveScan r;
    r.b = wave_argmin(b);
    r.exact = exact;
    r.read = (unsigned)(end - from);
    return r;
}

// Exact branch-and-bound over the triangle BVH (points outside the domain
// box, and walks stopped at the step cap).
template <bool kCtr>
__device__ __noinline__ Best bvh_search(const float4* __restrict__ bvh, const float4* __restrict__ tri_rec,
                                        const float3 q, uint8_t* __restrict__ bvh_flag, uint8_t* __restrict__ tri_flag)
{
    Best b{kInf, -1, 0.f, 0.f};
    int stack[64];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const int ni = stack[--sp];
        const float4 lo = gload(bvh + 2 * ni), hi = gload(bvh + 2 * ni + 1);
        if (kCtr && bvh_flag) bvh_flag[ni] = 1;
        const float bx = fmaxf(fmaxf(lo.x - q.x, q.x - hi.x), 0.f);
        const float by = fmaxf(fmaxf(lo.y - q.y, q.y - hi.y), 0.f);
        const float bz = fmaxf(fmaxf(lo.z - q.z, q.z - hi.z), 0.f);
        if (bx * bx + by * by + bz * bz > b.d2) continue;
        const int a = __float_as_int(lo.w), c = __float_as_int(hi.w);
        if (c < 0) {
            for (int slot = a; slot < a - c; ++slot) {
                const float4* r = tri_rec + 3 * (int64_t)slot;
                if (kCtr && tri_flag) tri_flag[slot] = 1;
                float v, w;
                const float d2 = closest_point_rec(q, r, v, w);
                if (d2 < b.d2) { b.d2 = d2; b.idx = -slot - 2; b.v = v; b.w = w; }
            }
        } else if (sp + 2 <= 64) {
            stack[sp++] = c;       // right child
            stack[sp++] = ni + 1;  // left child (popped first)
        }
    }
    return b;
}

// Vertex-gradient accumulators.  DirectAcc adds straight to global memory
// (float32 atomics).  LdsAcc first combines a workgroup's contributions in a
// hash table in LDS (points are processed in spatial order, so neighbouring
// points share vertices), then adds one global atomic per distinct vertex;
// an insertion that does not find a slot within kProbe steps goes global.
struct DirectAcc {
    float* gv;
    __device__ __forceinline__ void add(int vid, float x, float y, float z) const
    {
        __attribute__((address_space(1))) float* dst = (__attribute__((address_space(1))) float*)gv + 3 * (int64_t)vid;
        __hip_atomic_fetch_add(dst, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(dst + 1, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(dst + 2, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// An LDS pointer in LDS's own address space, so that the atomics on it are
// issued as LDS instructions rather than flat ones.
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) T* lds_ptr(T* p)
{
    return (__attribute__((address_space(3))) T*)p;
}

struct LdsAcc {
    float* gv;
    int* keys;
    float* val;         // 3 per slot
    int slots;          // power of two
    int* used = nullptr;  // if set, counts the slots taken
    static constexpr int kProbe = 32;

    __device__ __forceinline__ void init() const
    {
        for (int s = threadIdx.x; s < slots; s += blockDim.x) {
            keys[s] = -1;
            val[3 * s] = 0.f;
            val[3 * s + 1] = 0.f;
            val[3 * s + 2] = 0.f;
        }
    }
    __device__ __forceinline__ void add(int vid, float x, float y, float z) const
    {
        uint32_t h = (uint32_t)vid * 2654435761u;
        for (int p = 0; p < kProbe; ++p) {
            const int slot = (int)((h + (uint32_t)p) & (uint32_t)(slots - 1));
            int prev = -1;  // the slot's key before the exchange
            __hip_atomic_compare_exchange_strong(lds_ptr(keys) + slot, &prev, vid, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == -1 && used)
                __hip_atomic_fetch_add(lds_ptr(used), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == -1 || prev == vid) {
                __attribute__((address_space(3))) float* vs = lds_ptr(val) + 3 * slot;
                __hip_atomic_fetch_add(vs, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(vs + 1, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(vs + 2, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
        }
        DirectAcc{gv}.add(vid, x, y, z);
    }
    __device__ __forceinline__ void flush() const
    {
        for (int s = threadIdx.x; s < slots; s += blockDim.x) {
            const int k = keys[s];
            if (k >= 0) DirectAcc{gv}.add(k, val[3 * s], val[3 * s + 1], val[3 * s + 2]);
        }
    }
    // flush, and leave the table empty
    __device__ __forceinline__ void flush_clear() const
    {
        for (int s = threadIdx.x; s < slots; s += blockDim.x) {
            const int k = keys[s];
            if (k >= 0) {
                DirectAcc{gv}.add(k, val[3 * s], val[3 * s + 1], val[3 * s + 2]);
                keys[s] = -1;
                val[3 * s] = 0.f;
                val[3 * s + 1] = 0.f;
                val[3 * s + 2] = 0.f;
            }
        }
    }
};

// Adds each lane's dL/dV contributions (c: 3 values for each of the
// triangle's 3 vertices) through acc, first summed over runs of consecutive
// lanes on the same triangle (tri >= 0; -1 contributes nothing) by a
// segmented suffix sum across the wavefront, so that only the first lane of
// a run touches the accumulator: sorted points put neighbouring lanes on the
// same triangle, and their atomics on one address would serialise.  Every
// lane of the wavefront must call it.
template <class Acc>
__device__ __forceinline__ void add_vertex_grads(const DevMesh& m, const Acc& acc, const int tri, float c[9])
{
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(tri, 1, 64);
    const bool head = lane == 0 || tri < 0 || prev != tri;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? heads : (heads & ((2ull << lane) - 1ull));
    const int run = 63 - __builtin_clzll(upto);  // the run's first lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int r2 = __shfl_down(run, off, 64);
        const bool same = lane + off < 64 && r2 == run;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float o = __shfl_down(c[k], off, 64);
            if (same) c[k] += o;
        }
    }
    if (head && tri >= 0) {
        const int4 vid = gload(m.tri_vid + tri);
        const int ids[3] = {vid.x, vid.y, vid.z};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (c[3 * k] != 0.f || c[3 * k + 1] != 0.f || c[3 * k + 2] != 0.f)
                acc.add(ids[k], c[3 * k], c[3 * k + 1], c[3 * k + 2]);
    }
}

// The rest of one query after its lane's part of the list scan: lists left
// unfinished (resume >= 0) are completed by the wavefront, then fallback,
// outputs and, when fused, the gradient.  q is the point (finite tells
// whether all its coordinates are), s its located site or -1 when q is not
// finite or outside the domain box, b the scan's best so far; i is the
// output position.
//
// Every lane of the wavefront must call it (valid = false for a lane without
// a query): long lists are scanned by the whole wavefront.
template <bool kFused, bool kCtr, class Acc>
__device__ __forceinline__ void finish_query(const DevMesh& m, const bool valid, const float3 q, const bool finite,
                                             const int s, Best b, const int resume, const int64_t i,
                                             float* __restrict__ dist, int32_t* __restrict__ tri,
                                             float* __restrict__ closest, const float* __restrict__ gdist,
                                             float* __restrict__ grad_q, const Acc& acc,
                                             unsigned long long* __restrict__ ctr, QueryCounts n, const Touch tch)
{
    unsigned long long steps = n.steps, adj_read = n.adj_read, list_read = n.list_read, exact = n.exact,
                       list_len = n.list_len, fb = 0;
    // lists not done within the budget: finished by the whole wavefront
    for (uint64_t todo = __ballot(resume >= 0); todo; todo &= todo - 1) {
        const int src = __builtin_ctzll(todo);
        const float3 qs = make_float3(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.x), src)),
                                      __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.y), src)),
                                      __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.z), src)));
        const int ss = __builtin_amdgcn_readlane(s, src);
        const int from = __builtin_amdgcn_readlane(resume, src);
        const float d0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sqrtf(b.d2)), src));
        const WaveScan r = list_search_wave<kCtr>(m.site_rec, m.list_sph, m.list_rec, qs, ss, from, d0, tch.sph,
                                                  tch.rec);
        if ((int)(threadIdx.x & 63) == src) {
            // the lane's own result holds earlier entries and wins ties
            if (r.b.d2 < b.d2) b = r.b;
            list_read += r.read;
            exact += r.exact;
        }
    }
    // the fused form's gradient step below is wavefront-wide: there every
    // lane goes on
    if (!kFused && !valid) return;
    if (valid && finite && b.idx == -1) {
        b = bvh_search<kCtr>(m.bvh, m.tri_rec, q, tch.bvh, tch.tri);
        fb = 1;
    }
    if (kCtr && valid) {
        atomicAdd(&ctr[CTR_WALK_STEPS], steps);
        atomicAdd(&ctr[CTR_ADJ_READ], adj_read);
        atomicAdd(&ctr[CTR_LIST_READ], list_read);
        atomicAdd(&ctr[CTR_EXACT], exact);
        atomicAdd(&ctr[CTR_FALLBACK], fb);
        atomicAdd(&ctr[CTR_LIST_LEN], list_len);
        atomicAdd(&ctr[CTR_WALK_CAP], n.capped);
    }
    int gtri = -1;        // fused: this lane's triangle for dL/dV, or -1
    float gc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid && b.idx == -1) {
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
    } else if (valid) {
        // the winner's caller id (from its list entry, just scanned, or the
        // fallback's slot), then its exact closest point in FP64
        const int user = b.idx >= 0 ? __float_as_int(gload(m.list_rec + (3 * (int64_t)b.idx + 2)).w) : gload(m.tri_user + -b.idx - 2);
        const Final f = finalize(m, q, user);
        const double d = sqrt(f.d2);
        dist[i] = (float)d;
        if (tri) tri[i] = user;
        if (closest) {
            closest[3 * i] = (float)f.p.x;
            closest[3 * i + 1] = (float)f.p.y;
            closest[3 * i + 2] = (float)f.p.z;
        }
        if (kFused) {
            const float g = gdist[i];
            float nx = 0.f, ny = 0.f, nz = 0.f;
            if (d > 0.0) {
                const double inv = 1.0 / d;
                nx = (float)((q.x - f.p.x) * inv);
                ny = (float)((q.y - f.p.y) * inv);
                nz = (float)((q.z - f.p.z) * inv);
            }
            if (grad_q) {
                grad_q[3 * i] = g * nx;
                grad_q[3 * i + 1] = g * ny;
                grad_q[3 * i + 2] = g * nz;
            }
            if (d > 0.0 && g != 0.f) {
                const float lam[3] = {(float)(1.0 - f.v - f.w), (float)f.v, (float)f.w};
                gtri = user;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float s = -g * lam[k];
                    gc[3 * k] = s * nx;
                    gc[3 * k + 1] = s * ny;
                    gc[3 * k + 2] = s * nz;
                }
            }
        }
    }
    if (kFused && acc.gv) add_vertex_grads(m, acc, gtri, gc);
}

// Regroups a workgroup's queries by located site, so that lanes holding
// the same site become neighbours: the list scans of a wavefront then read
// the same entries, one cache line serving many lanes, instead of a few
// dozen sites' lists at once.  Each lane passes its query (q, output
// position i or -1 for none, site s or -1) and gets back the one it is to
// finish.  The key is the site's low 8 bits (queries without a site take
// 255): a workgroup's few dozen sites rarely share a key, and a shared key
// only interleaves two sites.  The ranking is stable (ballots over the key
// bits rank a wavefront's lanes, per-wavefront counts in LDS order the
// wavefronts), so the assignment is deterministic.
//
// `join` (uniform over the wavefront) says whether the wavefront takes
// part: the queries of the joining wavefronts are regrouped over the slots
// of those wavefronts only, and the others keep their own queries.  (A
// wavefront holding a list longer than one lane's scan budget stays out:
// it completes such lists one after the other, and gathering the lanes of
// a long-list site into one wavefront would queue all their scans there.)
//
// smem holds nw * 256 counts, zeroed by the caller before a barrier, then
// 5 words per thread, then nw flags.  Every thread of the workgroup must
// call it.
__device__ __forceinline__ void regroup_by_site(int* smem, const int nw, const bool join, float3& q, int64_t& i,
                                                int& s)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int* wc = smem;                             // [nw][256]: counts, then starts
    int* slot = smem + nw * 256;                // [blockDim][5]: x, y, z, i, s
    int* part = slot + 5 * (int)blockDim.x;     // [nw]: the wavefront joins
    const uint32_t d = s >= 0 ? ((uint32_t)s & 255u) : 255u;
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m1 = __ballot(bit);
        peers &= bit ? m1 : ~m1;
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(peers & below);
    if (lane == 0) part[wid] = join ? 1 : 0;
    if (join && rank == 0) wc[wid * 256 + (int)d] = __popcll(peers);
    __syncthreads();
    if (wid == 0) {
        // lane l holds keys 4l..4l+3: totals, exclusive scan, per-wavefront starts
        int t[4], tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            t[k] = 0;
            for (int w = 0; w < nw; ++w) t[k] += wc[w * 256 + 4 * lane + k];
            tot += t[k];
        }
        int inc = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        int start = inc - tot;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            for (int w = 0; w < nw; ++w) {
                const int c = wc[w * 256 + 4 * lane + k];
                wc[w * 256 + 4 * lane + k] = start;
                start += c;
            }
        }
    }
    __syncthreads();
    int me = (int)threadIdx.x;
    if (join) {
        // position pos among the joining wavefronts' 64 * (number joining)
        // slots: lane pos % 64 of the (pos / 64)-th joining wavefront
        const int pos = wc[wid * 256 + (int)d] + rank;
        int k = pos >> 6, w = 0;
        for (; w < nw; ++w) {
            if (part[w]) {
                if (k == 0) break;
                --k;
            }
        }
        me = w * 64 + (pos & 63);
    }
    slot[5 * me] = __float_as_int(q.x);
    slot[5 * me + 1] = __float_as_int(q.y);
    slot[5 * me + 2] = __float_as_int(q.z);
    slot[5 * me + 3] = (int)i;
    slot[5 * me + 4] = s;
    __syncthreads();
    const int t = (int)threadIdx.x;
    q = make_float3(__int_as_float(slot[5 * t]), __int_as_float(slot[5 * t + 1]), __int_as_float(slot[5 * t + 2]));
    i = slot[5 * t + 3];
    s = slot[5 * t + 4];
}

// LDS of regroup_by_site for a workgroup of `block` threads, in ints.
__host__ __device__ inline int regroup_lds_ints(int block) { return (block / 64) * 257 + block * 5; }

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b mod x).  Remapping block b to logical block (b mod x) * per + b / x gives
// every XCD one contiguous range of the sorted points, so each XCD's L2 sees
// one spatially coherent region instead of all of them.
__device__ __forceinline__ int64_t xcd_block(const int xcds, const int64_t per)
{
    const int64_t b = blockIdx.x;
    return (b % xcds) * per + b / xcds;
}

// LDS staging of the list spheres a wavefront is about to scan (the
// "List Search" of Sec. 3.4 reading its candidates from LDS).  After the
// regroup, lanes holding one site are neighbours; each distinct site of the
// wavefront held by at least kStageMinLanes lanes gets the first entries of
// its list copied into the wavefront's area (cap entries), its lanes
// copying entries rank, rank + lanes, ... so that each load instruction
// reads consecutive spheres.  Sites are taken in the order of their first
// lane until the area is full; a lane's st_off / st_cnt give where its
// list's first st_cnt entries are (st_cnt = 0: none staged).  Every lane of
// the wavefront must call it.
constexpr int kStageEntries = 256;  // largest area per wavefront
constexpr int kStageMinLanes = 4;
constexpr int kStageUnroll = 4;

template <bool kCtr>
__device__ __forceinline__ void stage_spheres(const DevMesh& m, float4* st, const int cap, const int s,
                                              const int4 rg, int& st_off, int& st_cnt, const Touch& tch)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    st_off = 0;
    st_cnt = 0;
    int rank = 0, lanes = 1, total = 0;
    for (uint64_t todo = __ballot(s >= 0); todo;) {
        const int lead = __builtin_ctzll(todo);
        const int ls = __builtin_amdgcn_readlane(s, lead);
        const bool mine = s == ls;
        const uint64_t grp = __ballot(mine);
        todo &= ~grp;
        const int n_lanes = __popcll(grp);
        if (n_lanes < kStageMinLanes) continue;
        const int len = __builtin_amdgcn_readlane(rg.w - rg.z, lead);
        const int cnt = min(len, cap - total);
        if (mine) {
            st_off = total;
            st_cnt = cnt;
            rank = __popcll(grp & below);
            lanes = n_lanes;
        }
        total += cnt;
    }
    for (int k0 = rank; k0 < st_cnt; k0 += lanes * kStageUnroll) {
        float4 v[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int k = min(k0 + u * lanes, st_cnt - 1);
            v[u] = gload(m.list_sph + rg.z + k);
            if (kCtr && tch.sph) tch.sph[rg.z + k] = 1;
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u)
            if (k0 + u * lanes < st_cnt) st[st_off + k0 + u * lanes] = v[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of the search kernel before the vertex-gradient table, in ints: the
// regroup's area, which the staging area (stage entries per wavefront)
// then reuses.
__host__ __device__ inline int search_lds_ints(int block, int stage)
{
    const int rg = regroup_lds_ints(block);
    const int sg = (block / 64) * stage * 4;
    return rg > sg ? rg : sg;
}

// Where one workgroup's tile of queries comes from and goes to: point j of
// the tile (thread j) is read at q[3 iq] and its outputs written at i.
struct TileIo {
    const float* q;
    float* dist;
    int32_t* tri;
    float* closest;
    const float* grad_dist;
    float* grad_q;
    unsigned long long* ctr;
    Touch touch;
    int stage;
};

// One workgroup's tile of queries through the whole search: the walk, the
// queries regrouped by located site (see regroup_by_site), optionally the
// located sites' spheres staged in LDS, the list scans and the outputs.
// smem starts with the regroup's area (nw * 256 counts, zeroed by the caller
// before a barrier, then the slots), which the staging area reuses.  Every
// thread of the workgroup must call it.
template <bool kFused, bool kCtr>
__device__ __forceinline__ void search_tile(const DevMesh& m, int* smem, const TileIo& io, const LdsAcc& acc,
                                            const bool valid, const int64_t i, const int64_t iq)
{
    const int nw = (int)(blockDim.x >> 6);
    float3 q = make_float3(0.f, 0.f, 0.f);
    if (valid) q = make_float3(gload(io.q + 3 * iq), gload(io.q + 3 * iq + 1), gload(io.q + 3 * iq + 2));
    const bool finite = valid && isfinite(q.x) && isfinite(q.y) && isfinite(q.z);
    int s = -1;
    float4 sp = make_float4(0.f, 0.f, 0.f, 0.f);
    int4 rg = make_int4(0, 0, 0, 0);
    if (finite && in_domain(m, q)) {
        unsigned long long steps = 0, adj_read = 0, capped = 0;
        if (m.oct) {
            s = octree_locate(m, q, steps);
            sp = gload(m.site_rec + 2 * s);
            rg = __builtin_bit_cast(int4, gload(m.site_rec + 2 * s + 1));
        } else {
            s = locate<kCtr>(m, q, steps, adj_read, capped, io.touch, sp, rg);
        }
        if (kCtr) {
            atomicAdd(&io.ctr[CTR_WALK_STEPS], steps);
            atomicAdd(&io.ctr[CTR_ADJ_READ], adj_read);
            atomicAdd(&io.ctr[CTR_WALK_CAP], capped);
        }
    }
    // Wavefronts holding a list longer than one lane's scan budget keep
    // their queries (see regroup_by_site); the others regroup among
    // themselves.
    int64_t i2 = valid ? i : -1;
    const bool join = __ballot(s >= 0 && rg.w - rg.z > kSerialBudget) == 0ull;
    regroup_by_site(smem, nw, join, q, i2, s);
    if (s >= 0) {
        sp = gload(m.site_rec + 2 * s);
        rg = __builtin_bit_cast(int4, gload(m.site_rec + 2 * s + 1));
    }
    const bool valid2 = i2 >= 0;
    const bool finite2 = valid2 && isfinite(q.x) && isfinite(q.y) && isfinite(q.z);
    // the located sites' spheres staged in LDS (the area reuses the
    // regroup's, once every wavefront has read its slot back)
    int st_off = 0, st_cnt = 0;
    float4* st = (float4*)smem + (threadIdx.x >> 6) * io.stage;
    if (io.stage > 0) {
        __syncthreads();
        stage_spheres<kCtr>(m, st, io.stage, s, rg, st_off, st_cnt, io.touch);
    }
    QueryCounts n;
    Best b{kInf, -1, 0.f, 0.f};
    int resume = -1;
    if (s >= 0) b = list_search<kCtr>(m, q, sp, rg, kSerialBudget, &resume, n, io.touch, st, st_off, st_cnt);
    finish_query<kFused, kCtr>(m, valid2, q, finite2, s, b, resume, valid2 ? i2 : 0, io.dist, io.tri, io.closest,
                               io.grad_dist, io.grad_q, acc, io.ctr, n, io.touch);
}

// Seven wavefronts per SIMD (at most 72 VGPRs): measured faster than the six
// the compiler picks by itself, its few spills being outside the list scan.
template <bool kFused, bool kCtr>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(7, 8))) fwd_kernel(const DevMesh m,
                                                                                             const FwdArgs a)
{
    const int64_t per = gridDim.x / a.xcds;
    const int64_t j = xcd_block(a.xcds, per) * blockDim.x + threadIdx.x;
    const bool valid = j < a.n;
    const int64_t i = valid ? (a.perm ? (int64_t)gload(a.perm + j) : j) : 0;
    // LDS: the search's area (regroup, staging), then (fused with dL/dV) the
    // table of vertex gradients, flushed once the workgroup is done.
    extern __shared__ __align__(16) int smem[];
    const int nw = (int)(blockDim.x >> 6);
    int* acc_smem = smem + search_lds_ints((int)blockDim.x, a.stage);
    const bool gv = kFused && a.grad_v;
    const LdsAcc acc{gv ? a.grad_v : nullptr, acc_smem, (float*)(acc_smem + a.acc_slots), a.acc_slots};
    for (int k = threadIdx.x; k < nw * 256; k += blockDim.x) smem[k] = 0;
    if (gv) acc.init();
    __syncthreads();
    const TileIo io{a.q, a.dist, a.tri, a.closest, a.grad_dist, a.grad_q, a.ctr, a.touch, a.stage};
    search_tile<kFused, kCtr>(m, smem, io, acc, valid, i, a.q_sorted ? j : i);
    if (gv) {
        __syncthreads();
        acc.flush();
    }
}

// Persistent batched kernel: each workgroup takes work items (up to `tile`
// consecutive sorted queries of one mesh) from a global counter until none
// is left, so meshes of very different sizes share one launch, and runs
// each item's queries through search_tile blockDim at a time (the walk, the
// regroup by site, the scans), as the plain kernel does for its one tile.
// Fused, the workgroup's LDS table of vertex gradients is flushed to the
// item's mesh after every item.
template <bool kFused>
__global__ void __launch_bounds__(1024) batch_kernel(
    const DevMesh* __restrict__ meshes, const BatchArgs a)
{
    extern __shared__ __align__(16) int smem[];
    __shared__ unsigned item_sh;
    const int nw = (int)(blockDim.x >> 6);
    int* acc_smem = smem + search_lds_ints((int)blockDim.x, a.stage);
    const bool fused_v = kFused && a.grad_v;
    if (fused_v) LdsAcc{nullptr, acc_smem, (float*)(acc_smem + a.acc_slots), a.acc_slots}.init();
    const TileIo io{a.q, a.dist, a.tri, a.closest, a.grad_dist, a.grad_q, nullptr, Touch{}, a.stage};
    for (;;) {
        __syncthreads();  // the previous item is done with LDS and item_sh
        if (threadIdx.x == 0) item_sh = atomicAdd(a.counter, 1u);
        __syncthreads();
        const unsigned t = item_sh;
        if (t >= (unsigned)a.n_items) break;
        const int mi = __builtin_amdgcn_readfirstlane(gload(a.item_mesh + t));
        const int64_t first = gload(a.item_first + t);
        const int64_t base = gload(a.q_off + mi);
        const int64_t last = min(first + (int64_t)a.tile, gload(a.q_off + mi + 1) - base);
        const DevMesh& m = meshes[mi];  // fields loaded as needed (scalar loads), not all kept live
        const int32_t* perm = a.perm[mi];
        float* gv = fused_v ? a.grad_v[mi] : nullptr;
        const LdsAcc acc{gv, acc_smem, (float*)(acc_smem + a.acc_slots), a.acc_slots};
        // workgroup-uniform trip count: every thread takes part in each tile
        for (int64_t j0 = first; j0 < last; j0 += blockDim.x) {
            if (j0 != first) __syncthreads();  // the previous tile is done with the regroup's area
            for (int k = threadIdx.x; k < nw * 256; k += blockDim.x) smem[k] = 0;
            __syncthreads();
            const int64_t j = j0 + threadIdx.x;
            const bool valid = j < last;
            const int64_t i = valid ? base + (perm ? (int64_t)gload(perm + j) : j) : 0;
            search_tile<kFused, false>(m, smem, io, acc, valid, i, i);
        }
        if (fused_v && gv) {
            __syncthreads();
            acc.flush_clear();
        }
    }
}

// The batched form without the queue: one workgroup per work item (a tile
// of blockDim queries of one mesh, items in largest-mesh-first order), the
// hardware's dispatcher handing out the workgroups as slots free up.  The
// same per-tile search as the plain kernel, with the mesh looked up per
// workgroup.
template <bool kFused>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(7, 8))) batch_tile_kernel(
    const DevMesh* __restrict__ meshes, const BatchArgs a)
{
    extern __shared__ __align__(16) int smem[];
    const int nw = (int)(blockDim.x >> 6);
    const int t = (int)blockIdx.x;
    const int mi = __builtin_amdgcn_readfirstlane(gload(a.item_mesh + t));
    const int64_t first = gload(a.item_first + t);
    const int64_t base = gload(a.q_off + mi);
    const int64_t last = min(first + (int64_t)a.tile, gload(a.q_off + mi + 1) - base);
    const DevMesh& m = meshes[mi];
    const int32_t* perm = a.perm[mi];
    float* gv = kFused && a.grad_v ? a.grad_v[mi] : nullptr;
    int* acc_smem = smem + search_lds_ints((int)blockDim.x, a.stage);
    const LdsAcc acc{gv, acc_smem, (float*)(acc_smem + a.acc_slots), a.acc_slots};
    for (int k = threadIdx.x; k < nw * 256; k += blockDim.x) smem[k] = 0;
    if (kFused && gv) acc.init();
    __syncthreads();
    const TileIo io{a.q, a.dist, a.tri, a.closest, a.grad_dist, a.grad_q, nullptr, Touch{}, a.stage};
    const int64_t j = first + threadIdx.x;
    const bool valid = j < last;
    const int64_t i = valid ? base + (perm ? (int64_t)gload(perm + j) : j) : 0;
    search_tile<kFused, false>(m, smem, io, acc, valid, i, i);
    if (kFused && gv) {
        __syncthreads();
        acc.flush();
    }
}

__global__ void __launch_bounds__(1024) bwd_kernel(const DevMesh m, const float* __restrict__ qp, int64_t n,
                                                   const int32_t* __restrict__ order,
                                                   const int32_t* __restrict__ tri, const float* __restrict__ gd,
                                                   float* __restrict__ grad_q, float* __restrict__ grad_v,
                                                   int acc_slots, int tiles)
{
    // One workgroup takes `tiles` consecutive tiles of blockDim points in
    // visiting order and keeps one LDS table of vertex gradients across
    // them (the slots' keys and values, then the count of slots taken).  It
    // is flushed to dL/dV once more than half of it is taken, and at the
    // end: consecutive tiles of sorted points share most of their vertices,
    // so a vertex reaches global memory once per run of tiles, not per tile.
    extern __shared__ int acc_smem[];
    int* used = acc_smem + 4 * acc_slots;
    const LdsAcc acc{grad_v, acc_smem, (float*)(acc_smem + acc_slots), acc_slots, used};
    if (grad_v) {
        acc.init();
        if (threadIdx.x == 0) *used = 0;
    }
    __syncthreads();
    for (int t = 0; t < tiles; ++t) {
        const int64_t j = ((int64_t)blockIdx.x * tiles + t) * blockDim.x + threadIdx.x;
        int gtri = -1;
        float gc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (j < n) {
            const int64_t i = order ? (int64_t)order[j] : j;
            const int tt = tri[i];
            float nx = 0.f, ny = 0.f, nz = 0.f, g = 0.f, d = 0.f;
            double v = 0.0, w = 0.0;
            if (tt >= 0 && tt < m.n_tris) {
                const float3 q = make_float3(qp[3 * i], qp[3 * i + 1], qp[3 * i + 2]);
                g = gd[i];
                // the triangle's exact closest point, as the forward
                // computed it for its winner
                const Final f = finalize(m, q, tt);
                const double dd = sqrt(f.d2);
                d = (float)dd;
                if (dd > 0.0) {
                    const double inv = 1.0 / dd;
                    nx = (float)((q.x - f.p.x) * inv);
                    ny = (float)((q.y - f.p.y) * inv);
                    nz = (float)((q.z - f.p.z) * inv);
                } else {
                    d = 0.f;
                }
                v = f.v;
                w = f.w;
            }
            if (grad_q) {
                grad_q[3 * i] = g * nx;
                grad_q[3 * i + 1] = g * ny;
                grad_q[3 * i + 2] = g * nz;
            }
            if (d > 0.f && g != 0.f) {
                const float lam[3] = {(float)(1.0 - v - w), (float)v, (float)w};
                gtri = tt;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float s = -g * lam[k];
                    gc[3 * k] = s * nx;
                    gc[3 * k + 1] = s * ny;
                    gc[3 * k + 2] = s * nz;
                }
            }
        }
        if (!grad_v) continue;
        add_vertex_grads(m, acc, gtri, gc);
        // every thread reads the count between two barriers, so that all
        // take the same branch
        __syncthreads();
        const int u = *used;
        __syncthreads();
        if (u > acc_slots / 2 && t + 1 < tiles) {
            acc.flush_clear();
            if (threadIdx.x == 0) *used = 0;
            __syncthreads();
        }
    }
    if (grad_v) acc.flush();
}

// ---------------------------------------------------------------- reorder
// Query sort: an LSD radix sort (8-bit digits) of the Morton code of each
// point's cell in a 2^bits-per-axis grid over the seed-grid box; points
// outside the domain box or non-finite get the largest code (last).

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x030000ff;
    x = (x | (x << 8)) & 0x0300f00f;
    x = (x | (x << 4)) & 0x030c30c3;
    x = (x | (x << 2)) & 0x09249249;
    return x;
}

// Morton code of a point's cell in the 2^bits-per-axis sort grid over the
// seed-grid box; non-finite points and points outside the domain box get
// the largest code.
__device__ __forceinline__ uint32_t point_key(const DevMesh& m, const float* __restrict__ qp, int64_t i,
                                              int bits, float sx, float sy, float sz)
{
    const float3 q = make_float3(qp[3 * i], qp[3 * i + 1], qp[3 * i + 2]);
    if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && in_domain(m, q))) return (1u << (3 * bits)) - 1u;
    const int g = (1 << bits) - 1;
    const uint32_t ix = (uint32_t)min(max((int)floorf((q.x - m.gorg[0]) * sx), 0), g);
    const uint32_t iy = (uint32_t)min(max((int)floorf((q.y - m.gorg[1]) * sy), 0), g);
    const uint32_t iz = (uint32_t)min(max((int)floorf((q.z - m.gorg[2]) * sz), 0), g);
    return spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
}

// LSD radix sort of (key, point index), 8 bits per pass.  A tile of
// kSortTile consecutive elements per workgroup: the upsweep counts digits in
// LDS; after a scan of the (digit, tile) counts the downsweep writes every
// element to its digit's range, ranked stably within the tile by wavefront
// ballots over the digit bits.  The first pass computes the keys from the
// points themselves.
constexpr int kSortBlock = 256;
constexpr int kSortIters = 16;
constexpr int kSortTile = kSortBlock * kSortIters;

template <bool kFromPoints>
__global__ void __launch_bounds__(kSortBlock) radix_upsweep(const DevMesh m, const float* __restrict__ qp,
                                                            const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                            int bits, float sx, float sy, float sz,
                                                            uint32_t* __restrict__ counts, int64_t n_tiles)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortIters; ++it) {
        const int64_t idx = base + it * kSortBlock + threadIdx.x;
        if (idx < n) {
            const uint32_t key = kFromPoints ? point_key(m, qp, idx, bits, sx, sy, sz) : keys[idx];
            atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = hist[threadIdx.x];
}

// Downsweep: the tile is ranked stably by digit into LDS, then written out
// in that order, so that consecutive threads write consecutive addresses of
// a digit's run instead of scattering one element per digit.  Wavefront w
// holds the tile's w-th quarter.  It ranks its keys by itself, 64 at a time
// (ballots over the digit bits find the lanes with the same digit, a
// running count per digit in the wavefront's own LDS row orders the
// rounds), so that only the combination of the four rows into each
// wavefront's start per digit needs the workgroup's barriers.  Tile order
// is (wavefront, round, lane) order, so the sort stays stable.  keys_out
// may be null (last pass: only the values are needed).
template <bool kFromPoints>
__global__ void __launch_bounds__(kSortBlock) radix_downsweep(
    const DevMesh m, const float* __restrict__ qp, const uint32_t* __restrict__ keys_in,
    const int32_t* __restrict__ vals_in, int64_t n, int shift, int bits, float sx, float sy, float sz,
    const uint32_t* __restrict__ offsets, int64_t n_tiles, uint32_t* __restrict__ keys_out,
    int32_t* __restrict__ vals_out, float* __restrict__ sorted_q)
{
    constexpr int kWaves = kSortBlock / 64;
    constexpr int kPerWave = kSortTile / kWaves;
    static_assert(kPerWave == 64 * kSortIters, "a wavefront ranks kSortIters rounds of 64 keys");
    __shared__ uint32_t lkey[kSortTile];
    __shared__ int32_t lval[kSortTile];
    __shared__ uint32_t wc[kWaves][256];  // per-wavefront digit counts, then starts
    __shared__ uint32_t lstart[256], gbase[256], wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = base + (int64_t)wid * kPerWave;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0u;
    gbase[tid] = offsets[(int64_t)tid * n_tiles + blockIdx.x];
    uint32_t key[kSortIters];
    int32_t val[kSortIters];
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        const int64_t idx = wbase + it * 64 + lane;
        key[it] = 0u;
        val[it] = 0;
        if (idx < n) {
            key[it] = kFromPoints ? point_key(m, qp, idx, bits, sx, sy, sz) : keys_in[idx];
            val[it] = kFromPoints ? (int32_t)idx : vals_in[idx];
        }
    }
    __syncthreads();
    // rank within the wavefront: wrank = earlier keys of this wavefront with
    // the same digit
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t wrank[kSortIters];
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        const bool valid = wbase + it * 64 + lane < n;
        const uint32_t d = (key[it] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m1 = __ballot(bit);
            peers &= bit ? m1 : ~m1;
        }
        const int leader = valid ? __builtin_ctzll(peers) : lane;
        uint32_t prev = 0u;
        // one leader per digit: this wavefront's row, distinct addresses
        if (valid && lane == leader) {
            prev = wc[wid][d];
            wc[wid][d] = prev + (uint32_t)__popcll(peers);
        }
        prev = (uint32_t)__shfl((int)prev, leader, 64);
        wrank[it] = prev + (uint32_t)__popcll(peers & below);
    }
    __syncthreads();
    // thread tid = digit: the tile's exclusive start per digit, then each
    // wavefront's start within it
    uint32_t c[kWaves], tot = 0u;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        c[w] = wc[w][tid];
        tot += c[w];
    }
    uint32_t inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t start = inc - tot;
    for (int w = 0; w < wid; ++w) start += wsum[w];
    lstart[tid] = start;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        wc[w][tid] = start;
        start += c[w];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        if (wbase + it * 64 + lane < n) {
            const uint32_t pos = wc[wid][(key[it] >> shift) & 255u] + wrank[it];
            lkey[pos] = key[it];
            lval[pos] = val[it];
        }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kSortTile, n - base);
    for (int j = tid; j < cnt; j += kSortBlock) {
        const uint32_t k = lkey[j];
        const int32_t v = lval[j];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t pos = gbase[d] + ((uint32_t)j - lstart[d]);
        if (keys_out) keys_out[pos] = k;
        vals_out[pos] = v;
        if (sorted_q) {
            sorted_q[3 * (int64_t)pos] = qp[3 * (int64_t)v];
            sorted_q[3 * (int64_t)pos + 1] = qp[3 * (int64_t)v + 1];
            sorted_q[3 * (int64_t)pos + 2] = qp[3 * (int64_t)v + 2];
        }
    }
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

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// LDS hash table for a workgroup's vertex gradients: a power of two at
// least 4x the workgroup's 3 contributions per thread.
inline int acc_slots_for(int block)
{
    int s = 1;
    while (s < 4 * block) s <<= 1;
    return s;
}

inline size_t acc_lds_bytes(int slots) { return (size_t)slots * 16; }

// Slots of a fused search's table: 256 (4 KB).  The table shares the
// workgroup with the search, and its LDS limits how many search
// wavefronts run at once: on C2's 10M points the grouped fused pass took
// 3.52 ms with 1,024 slots, 3.01 with 512 and 2.89 with 256 (128 and 64
// no better), the one-pass fused kernel 3.68 and 3.60 ms.  Contributions
// that find no free slot go straight to global memory.
inline int fused_acc_slots(int block) { return std::min(acc_slots_for(block), 256); }

// Slots of an LDS table plus its 16-byte count within 64 KB of LDS.
inline int acc_slots_capped(int want)
{
    int s = 1;
    while (s < want) s <<= 1;
    while (s > 64 && acc_lds_bytes(s) + 16 > 65536) s >>= 1;
    return s;
}

// Backward: LDS table slots per thread of the workgroup, and the number of
// rounds of resident workgroups the grid is sized for.
constexpr int kBwdSlotsPerThread = 4;
constexpr int kBwdRounds = 4;

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

// ------------------------------------------------- search grouped by site
// The search as three passes, for point sets that put many points in each
// cell: locate every point (in the visiting order), sort the points by
// located site, then scan each site's list once per group of lanes that
// share it.  In the scan pass a wavefront holds 64 consecutive points of
// the site order, so its lanes fall into a few runs of one site each.  For
// each run the wavefront loads the site's list 64 entries at a time with
// one coalesced load per lane (sphere and record) into LDS, and every lane
// of the run scans its copy there, entry by entry in list order with the
// same per-entry test (scan_entry) and budget as the per-lane scan: the
// results are the plain kernel's, bit for bit.

// Located site of each point in the visiting order: keys[j] = site (or
// n_sites when the point is not finite, outside the domain box, or its walk
// reached the step cap), pos[j] = j.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8)))
locate_kernel(const DevMesh m, const FwdArgs a, uint32_t* __restrict__ keys, int32_t* __restrict__ pos)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const int64_t i = a.perm ? (int64_t)gload(a.perm + j) : j;
    const int64_t iq = a.q_sorted ? j : i;
    const float3 q = make_float3(gload(a.q + 3 * iq), gload(a.q + 3 * iq + 1), gload(a.q + 3 * iq + 2));
    int s = -1;
    if (isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && in_domain(m, q)) {
        unsigned long long steps = 0, adj_read = 0, capped = 0;
        if (m.oct) {
            s = octree_locate(m, q, steps);
        } else {
            float4 sp;
            int4 rg;
            s = locate<false>(m, q, steps, adj_read, capped, Touch{}, sp, rg);
        }
    }
    keys[j] = s >= 0 ? (uint32_t)s : (uint32_t)m.n_sites;
    pos[j] = (int32_t)j;
}

// Entries of one shared chunk of a list in LDS: sphere, then the record.
struct ChunkEntry {
    float4 c, f1, f2, f3;
};

// Where each site's run starts and ends in the site-sorted order (runs[2k],
// runs[2k + 1]; key n_sites, the points with no site, is run n_sites).  The
// caller zeroes runs.
__global__ void run_bounds_kernel(const uint32_t* __restrict__ keys, int64_t n, int32_t* __restrict__ runs)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = keys[j];
    if (j == 0 || keys[j - 1] != k) runs[2 * (int64_t)k] = (int32_t)j;
    if (j == n - 1 || keys[j + 1] != k) runs[2 * (int64_t)k + 1] = (int32_t)(j + 1);
}

// Work items per run: one per `lanes` points (the count, to be scanned).
__global__ void run_items_kernel(const int32_t* __restrict__ runs, int64_t n_runs, int lanes,
                                 uint32_t* __restrict__ items)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_runs) return;
    items[k] = (uint32_t)((runs[2 * k + 1] - runs[2 * k] + lanes - 1) / lanes);
}

// The item list: item t = (first position, run).
__global__ void item_list_kernel(const int32_t* __restrict__ runs, const uint32_t* __restrict__ item_off,
                                 int64_t n_runs, int lanes, int2* __restrict__ item)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_runs) return;
    const int32_t b = runs[2 * k], e = runs[2 * k + 1];
    uint32_t t = item_off[k];
    for (int32_t p = b; p < e; p += lanes) item[t++] = make_int2(p, (int32_t)k);
}

// Work items of kLanes lanes (64: one per wavefront; 32: two per
// wavefront, each in its own half): up to kLanes consecutive points of one
// run, hence one site (or none: the points outside the domain box, not
// finite, or whose walk reached the step cap).  Items past the last do
// nothing.  Each item loads its site's list kLanes entries at a time into
// its own part of the LDS area.
template <bool kFused, int kLanes>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8)))
grouped_kernel(const DevMesh m, const FwdArgs a, const int32_t* __restrict__ pos, const int2* __restrict__ item,
               const uint32_t* __restrict__ n_items_p, const int32_t* __restrict__ runs)
{
    static_assert(kLanes == 64 || kLanes == 32, "items of 64 or 32 lanes");
    constexpr int kPer = 64 / kLanes;
    extern __shared__ __align__(16) int smem[];
    const int nw = (int)(blockDim.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int sub = lane / kLanes, sl = lane % kLanes;
    ChunkEntry* chunk = (ChunkEntry*)smem + (threadIdx.x >> 6) * 64 + sub * kLanes;
    int* acc_smem = smem + nw * 64 * (int)(sizeof(ChunkEntry) / sizeof(int));
    const bool gv = kFused && a.grad_v;
    const LdsAcc acc{gv ? a.grad_v : nullptr, acc_smem, (float*)(acc_smem + a.acc_slots), a.acc_slots};
    if (gv) {
        acc.init();
        __syncthreads();
    }
    const int64_t t = ((int64_t)blockIdx.x * nw + (threadIdx.x >> 6)) * kPer + sub;
    const bool live = t < (int64_t)gload(n_items_p);
    int2 it = make_int2(0, -1);
    if (live) it = gload(item + t);
    const int run = it.y;
    const int64_t j = (int64_t)it.x + sl;
    const bool valid = live && j < (int64_t)gload(runs + (2 * (int64_t)(run < 0 ? 0 : run) + 1));
    const int rs = (live && run < m.n_sites) ? run : -1;  // the item's site
    const int s = valid ? rs : -1;
    int64_t i = 0;
    float3 q = make_float3(0.f, 0.f, 0.f);
    if (valid) {
        const int64_t jj = gload(pos + j);
        i = a.perm ? (int64_t)gload(a.perm + jj) : jj;
        const int64_t iq = a.q_sorted ? jj : i;
        q = make_float3(gload(a.q + 3 * iq), gload(a.q + 3 * iq + 1), gload(a.q + 3 * iq + 2));
    }
    const bool finite = valid && isfinite(q.x) && isfinite(q.y) && isfinite(q.z);
    Best b{kInf, -1, 0.f, 0.f};
    int resume = -1;
    QueryCounts n;
    float4 sp = make_float4(0.f, 0.f, 0.f, 0.f);
    int4 rg = make_int4(0, 0, 0, 0);
    if (rs >= 0) {
        sp = gload(m.site_rec + 2 * rs);
        rg = __builtin_bit_cast(int4, gload(m.site_rec + 2 * rs + 1));
    }
    float dqs = 0.f, dmin = kInf;
    if (valid && rs >= 0) {
        const float wx = q.x - sp.x, wy = q.y - sp.y, wz = q.z - sp.z;
        // |q - s| rounded up so that the early-exit bound stays conservative
        dqs = sqrtf(wx * wx + wy * wy + wz * wz) * 1.000001f;
    }
    bool active = valid && rs >= 0 && rg.z < rg.w;
    int base = rg.z;  // the same in every lane of an item
    const uint64_t item_mask = kLanes == 64 ? ~0ull : (((1ull << kLanes) - 1ull) << (sub * kLanes));
    for (;;) {
        // the same budget as the per-lane scan: the rest of the list goes
        // to the wavefront-wide scan
        if (active && base - rg.z >= kSerialBudget) {
            resume = base;
            active = false;
        }
        const uint64_t act = __ballot(active);
        if (act == 0ull) break;
        if ((act & item_mask) != 0ull) {
            const int e = min(base + sl, rg.w - 1);
            ChunkEntry ce;
            ce.c = gload(m.list_sph + e);
            ce.f1 = gload(m.list_rec + 3 * (int64_t)e);
            ce.f2 = gload(m.list_rec + 3 * (int64_t)e + 1);
            ce.f3 = gload(m.list_rec + 3 * (int64_t)e + 2);
            chunk[sl] = ce;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (active) {
            const int cnt = min(kLanes, rg.w - base);
            for (int k0 = 0; k0 < cnt && active; k0 += kChunk) {
                // kChunk spheres read ahead, then tested in list order
                float4 cc[kChunk];
#pragma unroll
                for (int u = 0; u < kChunk; ++u) cc[u] = chunk[min(k0 + u, cnt - 1)].c;
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    if (!active || k0 + u >= cnt) break;
                    const ChunkEntry* ce = &chunk[k0 + u];
                    auto rec = [&](float4& f1, float4& f2, float4& f3) {
                        f1 = ce->f1;
                        f2 = ce->f2;
                        f3 = ce->f3;
                    };
                    if (!scan_entry(q, sp, dqs, cc[u], base + k0 + u, dmin, b, n.exact, rec)) active = false;
                }
            }
        }
        // every lane is done with the chunk before the next overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        base += kLanes;
        if (base >= rg.w) active = false;  // the list is done
    }
    finish_query<kFused, false>(m, valid, q, finite, s, b, resume, i, a.dist, a.tri, a.closest, a.grad_dist,
                                a.grad_q, acc, nullptr, n, Touch{});
    if (gv) {
        __syncthreads();
        acc.flush();
    }
}

}  // namespace

hipError_t launch_forward(const DevMesh& m, const FwdArgs& a, int block, bool fused, bool counters,
                          hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    // pad the grid to a multiple of the XCD count (see xcd_block)
    const int64_t nb = (a.n + block - 1) / block;
    const int x = a.xcds > 0 ? a.xcds : 1;
    const unsigned g = (unsigned)(((nb + x - 1) / x) * x);
    FwdArgs args = a;
    args.xcds = x;
    // staging area: up to kStageEntries spheres per wavefront, within 48 KB
    if (args.stage > 0) args.stage = std::min(kStageEntries, 49152 / (16 * (block / 64)));
    const size_t rg_bytes = 4 * (size_t)search_lds_ints(block, args.stage);
    if (fused) {
        // the table within 64 KB of LDS together with the regroup's area
        int slots = fused_acc_slots(block);
        while (slots > 64 && rg_bytes + acc_lds_bytes(slots) > 65536) slots >>= 1;
        args.acc_slots = slots;
        const size_t lds = rg_bytes + (a.grad_v ? acc_lds_bytes(slots) : 0);
        if (counters) fwd_kernel<true, true><<<g, block, lds, st>>>(m, args);
        else fwd_kernel<true, false><<<g, block, lds, st>>>(m, args);
    } else {
        if (counters) fwd_kernel<false, true><<<g, block, rg_bytes, st>>>(m, args);
        else fwd_kernel<false, false><<<g, block, rg_bytes, st>>>(m, args);
    }
    return hipGetLastError();
}

hipError_t launch_backward(const DevMesh& m, const float* q, int64_t n, const int32_t* order,
                           const int32_t* tri, const float* g, float* grad_q, float* grad_v, int block,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int slots = acc_slots_capped(kBwdSlotsPerThread * block);
    const size_t lds = grad_v ? acc_lds_bytes(slots) + 16 : 0;
    const int64_t n_tiles = (n + block - 1) / block;
    // with dL/dV, as few workgroups as fill the GPU kBwdRounds times, each
    // over consecutive tiles (fewer flushes of the table)
    int64_t tiles = 1;
    if (grad_v) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bwd_kernel, block, lds) == hipSuccess && cus > 0 &&
            per_cu > 0) {
            const int64_t slots_total = (int64_t)kBwdRounds * cus * per_cu;
            tiles = std::min<int64_t>(64, (n_tiles + slots_total - 1) / slots_total);
        }
    }
    const int64_t grid = (n_tiles + tiles - 1) / tiles;
    bwd_kernel<<<(unsigned)grid, block, lds, st>>>(m, q, n, order, tri, g, grad_q, grad_v, slots, (int)tiles);
    return hipGetLastError();
}

// Sort-grid resolution: 2^bits cells per axis, the finest grid with at most
// two cells per point (finer sorting keeps a wavefront's points on fewer
// sites; measured best on the 10M-point workload).
int sort_bits(int64_t n)
{
    int b = 2;
    while (b < 8 && (int64_t)1 << (3 * (b + 1)) <= 2 * n) ++b;
    return b;
}

size_t reorder_workspace_bytes(int64_t n, int bits)
{
    (void)bits;
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t nc = 256 * n_tiles;
    return sizeof(uint32_t) * (size_t)(4 * n + nc + scan_scratch(nc) + 64);
}

// Workspace of launch_grouped: the sort's (keys and positions, twice, and
// the digit counts), then the runs (2 per site and one more), their item
// counts and offsets (scanned with its scratch) and the item list.
// Lanes of one work item of the grouped scan: two items per wavefront
// (measured on 10M points of the 327k-triangle mesh: search 2.42 ms, against
// 2.54 ms with one 64-lane item per wavefront, whose lanes are idle more
// often when a site holds fewer than 64 points).
constexpr int kItemLanes = 32;

static size_t grouped_layout(int64_t n, int64_t n_sites, size_t* off_runs, size_t* off_cnt, size_t* off_tmp,
                             size_t* off_items)
{
    const size_t sort_bytes = (reorder_workspace_bytes(n, 0) + 255) & ~(size_t)255;
    const int64_t n_runs = n_sites + 1;
    const int64_t max_items = n / 32 + n_runs + 1;  // items of 32 or more lanes
    size_t o = sort_bytes;
    *off_runs = o;
    o += ((size_t)(2 * n_runs) * 4 + 255) & ~(size_t)255;
    *off_cnt = o;
    o += ((size_t)(n_runs + 1) * 4 + 255) & ~(size_t)255;
    *off_tmp = o;
    o += ((size_t)scan_scratch(n_runs + 1) * 4 + 255) & ~(size_t)255;
    *off_items = o;
    o += (size_t)max_items * 8;
    return o;
}

size_t grouped_workspace_bytes(int64_t n, int64_t n_sites)
{
    size_t a, b, c, d;
    return grouped_layout(n, n_sites, &a, &b, &c, &d);
}

hipError_t launch_grouped(const DevMesh& m, const FwdArgs& a, void* ws, bool fused, hipStream_t st)
{
    const int item_lanes = kItemLanes;
    if (a.n <= 0) return hipSuccess;
    const int64_t n = a.n;
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t nc = 256 * n_tiles;
    uint32_t* ka = (uint32_t*)ws;
    int32_t* va = (int32_t*)(ka + n);
    uint32_t* kb = (uint32_t*)(va + n);
    int32_t* vb = (int32_t*)(kb + n);
    uint32_t* counts = (uint32_t*)(vb + n);
    uint32_t* tmp = counts + nc;
    size_t o_runs, o_cnt, o_tmp, o_items;
    grouped_layout(n, m.n_sites, &o_runs, &o_cnt, &o_tmp, &o_items);
    int32_t* runs = (int32_t*)((char*)ws + o_runs);
    uint32_t* cnt = (uint32_t*)((char*)ws + o_cnt);
    uint32_t* stmp = (uint32_t*)((char*)ws + o_tmp);
    int2* items = (int2*)((char*)ws + o_items);
    const int64_t n_runs = (int64_t)m.n_sites + 1;
    locate_kernel<<<grid_for(n, 256), 256, 0, st>>>(m, a, ka, va);
    // sort by site (keys up to n_sites), 8 bits per pass, stable: within a
    // site the points keep their visiting order
    int key_bits = 1;
    while (key_bits < 31 && ((int64_t)1 << key_bits) <= (int64_t)m.n_sites) ++key_bits;
    uint32_t *kin = ka, *kout = kb;
    int32_t *vin = va, *vout = vb;
    for (int shift = 0; shift < key_bits; shift += 8) {
        radix_upsweep<false><<<(unsigned)n_tiles, kSortBlock, 0, st>>>(m, a.q, kin, n, shift, 0, 0.f, 0.f, 0.f,
                                                                       counts, n_tiles);
        hipError_t e = exclusive_scan(counts, nc, tmp, st);
        if (e != hipSuccess) return e;
        radix_downsweep<false><<<(unsigned)n_tiles, kSortBlock, 0, st>>>(m, a.q, kin, vin, n, shift, 0, 0.f, 0.f,
                                                                         0.f, counts, n_tiles, kout, vout, nullptr);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // the runs of each site and the work items (a site's run in pieces of
    // at most item_lanes points; the item count stays on the device)
    fill_u32_kernel<<<grid_for(2 * n_runs, 256), 256, 0, st>>>((uint32_t*)runs, 0u, 2 * n_runs);
    run_bounds_kernel<<<grid_for(n, 256), 256, 0, st>>>(kin, n, runs);
    fill_u32_kernel<<<1, 1, 0, st>>>(cnt + n_runs, 0u, 1);
    run_items_kernel<<<grid_for(n_runs, 256), 256, 0, st>>>(runs, n_runs, item_lanes, cnt);
    hipError_t e = exclusive_scan(cnt, n_runs + 1, stmp, st);
    if (e != hipSuccess) return e;
    item_list_kernel<<<grid_for(n_runs, 256), 256, 0, st>>>(runs, cnt, n_runs, item_lanes, items);
    FwdArgs args = a;
    const int block = 256;
    const int nw = block / 64;
    const size_t chunk_bytes = (size_t)nw * 64 * sizeof(ChunkEntry);
    size_t lds = chunk_bytes;
    if (fused && a.grad_v) {
        int slots = fused_acc_slots(block);
        while (slots > 64 && chunk_bytes + acc_lds_bytes(slots) > 65536) slots >>= 1;
        args.acc_slots = slots;
        lds += acc_lds_bytes(slots);
    }
    // waves for every item: n / lanes full ones and at most one partial per run
    const int64_t max_items = n / item_lanes + n_runs + 1;
    const int64_t per_wave = 64 / item_lanes;
    const unsigned grid = (unsigned)(((max_items + per_wave - 1) / per_wave + nw - 1) / nw);
    if (fused) grouped_kernel<true, kItemLanes><<<grid, block, lds, st>>>(m, args, vin, items, cnt + n_runs, runs);
    else grouped_kernel<false, kItemLanes><<<grid, block, lds, st>>>(m, args, vin, items, cnt + n_runs, runs);
    return hipGetLastError();
}

const int32_t* reorder_perm_location(void* ws, int64_t n, int bits)
{
    if (bits <= 0) bits = sort_bits(n);
    const int passes = (3 * bits + 7) / 8;
    // passes alternate between (ka, va) and (kb, vb); see launch_reorder
    uint32_t* ka = (uint32_t*)ws;
    return (passes % 2 == 1) ? (const int32_t*)(ka + n) : (const int32_t*)(ka + 3 * n);
}

hipError_t launch_reorder(const DevMesh& m, const float* q, int64_t n, int bits, void* ws,
                          const int32_t** perm_out, hipStream_t st, float* sorted_q)
{
    if (bits <= 0) bits = sort_bits(n);
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t nc = 256 * n_tiles;
    uint32_t* ka = (uint32_t*)ws;
    int32_t* va = (int32_t*)(ka + n);
    uint32_t* kb = (uint32_t*)(va + n);
    int32_t* vb = (int32_t*)(kb + n);
    uint32_t* counts = (uint32_t*)(vb + n);
    uint32_t* tmp = counts + nc;
    // the sort grid spans the seed-grid box
    const float G = (float)(1 << bits);
    const float cell = 1.0f / m.ginv;
    const float sx = G / (m.gdim[0] * cell), sy = G / (m.gdim[1] * cell), sz = G / (m.gdim[2] * cell);
    const int key_bits = 3 * bits;
    const unsigned grid = (unsigned)n_tiles;
    uint32_t *kin = nullptr, *kout = ka;
    int32_t *vin = nullptr, *vout = va;
    for (int shift = 0; shift < key_bits; shift += 8) {
        const bool last = shift + 8 >= key_bits;
        float* sq = last ? sorted_q : nullptr;
        uint32_t* ko = last ? nullptr : kout;
        if (shift == 0) {
            radix_upsweep<true><<<grid, kSortBlock, 0, st>>>(m, q, nullptr, n, shift, bits, sx, sy, sz, counts, n_tiles);
        } else {
            radix_upsweep<false><<<grid, kSortBlock, 0, st>>>(m, q, kin, n, shift, bits, sx, sy, sz, counts, n_tiles);
        }
        hipError_t e = exclusive_scan(counts, nc, tmp, st);
        if (e != hipSuccess) return e;
        if (shift == 0) {
            radix_downsweep<true><<<grid, kSortBlock, 0, st>>>(m, q, nullptr, nullptr, n, shift, bits, sx, sy, sz,
                                                               counts, n_tiles, ko, vout, sq);
        } else {
            radix_downsweep<false><<<grid, kSortBlock, 0, st>>>(m, q, kin, vin, n, shift, bits, sx, sy, sz, counts,
                                                                n_tiles, ko, vout, sq);
        }
        kin = kout;
        vin = vout;
        kout = (kout == ka) ? kb : ka;
        vout = (vout == va) ? vb : va;
    }
    *perm_out = vin;
    return hipGetLastError();
}

hipError_t launch_batch(const DevMesh* meshes, const BatchArgs& a, int grid, int block, bool fused, int stage,
                        hipStream_t st)
{
    BatchArgs args = a;
    // grid <= 0: one workgroup per work item (a.tile == block), no queue
    const bool direct = grid <= 0;
    if (direct && a.tile != block) return hipErrorInvalidValue;
    // as launch_forward: the staging area within 48 KB, the fused table
    // within 64 KB of LDS together with the search's area
    args.stage = stage > 0 ? std::min(kStageEntries, 49152 / (16 * (block / 64))) : 0;
    const size_t rg_bytes = 4 * (size_t)search_lds_ints(block, args.stage);
    if (fused) {
        int slots = fused_acc_slots(block);
        while (slots > 64 && rg_bytes + acc_lds_bytes(slots) > 65536) slots >>= 1;
        args.acc_slots = slots;
        const size_t lds = rg_bytes + (a.grad_v ? acc_lds_bytes(slots) : 0);
        if (direct) batch_tile_kernel<true><<<(unsigned)a.n_items, block, lds, st>>>(meshes, args);
        else batch_kernel<true><<<grid, block, lds, st>>>(meshes, args);
    } else {
        if (direct) batch_tile_kernel<false><<<(unsigned)a.n_items, block, rg_bytes, st>>>(meshes, args);
        else batch_kernel<false><<<grid, block, rg_bytes, st>>>(meshes, args);
    }
    return hipGetLastError();
}

// Reduction of a point set's distances (the mesh-to-mesh measures built on
// the point query): the largest distance with the lowest index among equal
// ones, the sums of d and d^2 in FP64, and the number of non-NaN distances.
// Stage 1 leaves 5 doubles per block; stage 2 (one block) folds them.
constexpr int kRedBlock = 256;

struct RedVal {
    double mx, idx, sum, sum2, cnt;
};

__device__ __forceinline__ RedVal red_combine(RedVal a, const RedVal& b)
{
    if (b.mx > a.mx || (b.mx == a.mx && b.idx >= 0 && (a.idx < 0 || b.idx < a.idx))) {
        a.mx = b.mx;
        a.idx = b.idx;
    }
    a.sum += b.sum;
    a.sum2 += b.sum2;
    a.cnt += b.cnt;
    return a;
}

__device__ __forceinline__ RedVal red_block(RedVal v)
{
    __shared__ double sh[5][kRedBlock];
    sh[0][threadIdx.x] = v.mx;
    sh[1][threadIdx.x] = v.idx;
    sh[2][threadIdx.x] = v.sum;
    sh[3][threadIdx.x] = v.sum2;
    sh[4][threadIdx.x] = v.cnt;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const RedVal o{sh[0][threadIdx.x + w], sh[1][threadIdx.x + w], sh[2][threadIdx.x + w],
                           sh[3][threadIdx.x + w], sh[4][threadIdx.x + w]};
            RedVal m{sh[0][threadIdx.x], sh[1][threadIdx.x], sh[2][threadIdx.x], sh[3][threadIdx.x],
                     sh[4][threadIdx.x]};
            m = red_combine(m, o);
            sh[0][threadIdx.x] = m.mx;
            sh[1][threadIdx.x] = m.idx;
            sh[2][threadIdx.x] = m.sum;
            sh[3][threadIdx.x] = m.sum2;
            sh[4][threadIdx.x] = m.cnt;
        }
        __syncthreads();
    }
    return RedVal{sh[0][0], sh[1][0], sh[2][0], sh[3][0], sh[4][0]};
}

__global__ void __launch_bounds__(kRedBlock) reduce_dist_kernel(const float* __restrict__ d, int64_t n,
                                                                 double* __restrict__ part)
{
    RedVal v{-1.0, -1.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedBlock) {
        const float x = d[i];
        if (x != x) continue;  // NaN: a non-finite point
        const double xd = (double)x;
        if (xd > v.mx) {       // indices grow along a thread's stride: the first wins
            v.mx = xd;
            v.idx = (double)i;
        }
        v.sum += xd;
        v.sum2 += xd * xd;
        v.cnt += 1.0;
    }
    const RedVal r = red_block(v);
    if (threadIdx.x == 0) {
        double* o = part + 5 * (int64_t)blockIdx.x;
        o[0] = r.mx;
        o[1] = r.idx;
        o[2] = r.sum;
        o[3] = r.sum2;
        o[4] = r.cnt;
    }
}

__global__ void __launch_bounds__(kRedBlock) reduce_final_kernel(const double* __restrict__ part, int nb,
                                                                  double* __restrict__ out)
{
    RedVal v{-1.0, -1.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedBlock)
        v = red_combine(v, RedVal{part[5 * b], part[5 * b + 1], part[5 * b + 2], part[5 * b + 3], part[5 * b + 4]});
    const RedVal r = red_block(v);
    if (threadIdx.x == 0) {
        out[0] = r.mx;
        out[1] = r.idx;
        out[2] = r.sum;
        out[3] = r.sum2;
        out[4] = r.cnt;
    }
}

int reduce_blocks(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + kRedBlock - 1) / kRedBlock));
}

hipError_t launch_reduce_dist(const float* d, int64_t n, double* part, double* out, hipStream_t st)
{
    const int nb = reduce_blocks(n);
    reduce_dist_kernel<<<nb, kRedBlock, 0, st>>>(d, n, part);
    reduce_final_kernel<<<1, kRedBlock, 0, st>>>(part, nb, out);
    return hipGetLastError();
}

// The six values of p2m_mesh_distance from the two one-sided reductions
// (max, argmax, sum, sum of squares, count): one-sided Hausdorff A to B and
// B to A, the symmetric one, the Chamfer sums of means of d and of d^2 (a
// side without points contributes 0), and the number of points counted.
__global__ void mesh_distance_combine_kernel(const double* __restrict__ ab, const double* __restrict__ ba,
                                             double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    const double hab = ab[0], hba = ba[0];
    out[0] = hab;
    out[1] = hba;
    out[2] = hab > hba ? hab : hba;
    const double na = ab[4], nb = ba[4];
    out[3] = (na > 0.0 ? ab[2] / na : 0.0) + (nb > 0.0 ? ba[2] / nb : 0.0);
    out[4] = (na > 0.0 ? ab[3] / na : 0.0) + (nb > 0.0 ? ba[3] / nb : 0.0);
    out[5] = na + nb;
}

hipError_t launch_mesh_distance_combine(const double* ab, const double* ba, double* out, hipStream_t st)
{
    mesh_distance_combine_kernel<<<1, 64, 0, st>>>(ab, ba, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    fill_u32_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace p2m
