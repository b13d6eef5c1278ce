// Host-side helpers for the P2M++ preprocessing: FP64 vector math, the
// library's own point-triangle distance, and a small parallel-for.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

namespace p2m {

struct d3 {
    double x, y, z;
};
inline d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline d3 operator*(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline d3 cross(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm2(d3 a) { return dot(a, a); }
inline double norm(d3 a) { return std::sqrt(dot(a, a)); }
inline d3 dmin3(d3 a, d3 b) { return {std::min(a.x, b.x), std::min(a.y, b.y), std::min(a.z, b.z)}; }
inline d3 dmax3(d3 a, d3 b) { return {std::max(a.x, b.x), std::max(a.y, b.y), std::max(a.z, b.z)}; }
inline double comp(d3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// Error carrying a library status code (see p2m.h) and a message.
struct Error : std::runtime_error {
    int32_t code;
    Error(int32_t c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Closest point on triangle (a, b, c) to q by classifying q against the
// triangle's vertex, edge and face regions (Ericson, Real-Time Collision
// Detection, Sec. 5.1.5).  Returns the squared distance; writes the closest
// point and its barycentric weights for (a, b, c).
inline double closest_on_triangle(d3 q, d3 a, d3 b, d3 c, d3* p_out, double* bary = nullptr)
{
    d3 ab = b - a, ac = c - a, ap = q - a;
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    double u = 1, v = 0, w = 0;  // weights of a, b, c
    if (d1 <= 0 && d2 <= 0) {
        u = 1; v = 0; w = 0;
    } else {
        d3 bp = q - b;
        double d3v = dot(ab, bp), d4 = dot(ac, bp);
        d3 cp = q - c;
        double d5 = dot(ab, cp), d6 = dot(ac, cp);
        double vc = d1 * d4 - d3v * d2;
        double vb = d5 * d2 - d1 * d6;
        double va = d3v * d6 - d5 * d4;
        if (d3v >= 0 && d4 <= d3v) {
            u = 0; v = 1; w = 0;
        } else if (vc <= 0 && d1 >= 0 && d3v <= 0) {
            double t = d1 / (d1 - d3v);
            u = 1 - t; v = t; w = 0;
        } else if (d6 >= 0 && d5 <= d6) {
            u = 0; v = 0; w = 1;
        } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
            double t = d2 / (d2 - d6);
            u = 1 - t; v = 0; w = t;
        } else if (va <= 0 && (d4 - d3v) >= 0 && (d5 - d6) >= 0) {
            double t = (d4 - d3v) / ((d4 - d3v) + (d5 - d6));
            u = 0; v = 1 - t; w = t;
        } else {
            double den = va + vb + vc;
            if (den > 0 && std::isfinite(den)) {
                v = vb / den; w = vc / den; u = 1 - v - w;
            } else {
                // Degenerate (zero-area) triangle: best of the three edges.
                auto seg = [&](d3 s0, d3 s1, double& t) {
                    d3 e = s1 - s0;
                    double L = norm2(e);
                    t = L > 0 ? std::clamp(dot(q - s0, e) / L, 0.0, 1.0) : 0.0;
                    return norm2(q - (s0 + e * t));
                };
                double t0, t1, t2;
                double e0 = seg(a, b, t0), e1 = seg(b, c, t1), e2 = seg(c, a, t2);
                if (e0 <= e1 && e0 <= e2) { u = 1 - t0; v = t0; w = 0; }
                else if (e1 <= e2) { u = 0; v = 1 - t1; w = t1; }
                else { u = t2; v = 0; w = 1 - t2; }
            }
        }
    }
    d3 p = a * u + b * v + c * w;
    if (p_out) *p_out = p;
    if (bary) { bary[0] = u; bary[1] = v; bary[2] = w; }
    return norm2(q - p);
}

// Run fn(i, thread_id) for i in [0, n) on n_threads threads, dynamic chunks.
inline void parallel_for(int64_t n, int n_threads, const std::function<void(int64_t, int)>& fn,
                         int64_t chunk = 64)
{
    if (n <= 0) return;
    if (n_threads <= 1 || n <= chunk) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> pool;
    std::exception_ptr err = nullptr;
    std::atomic<bool> failed{false};
    for (int t = 0; t < n_threads; ++t) {
        pool.emplace_back([&, t] {
            try {
                for (;;) {
                    int64_t b = next.fetch_add(chunk);
                    if (b >= n || failed.load()) break;
                    int64_t e = std::min(n, b + chunk);
                    for (int64_t i = b; i < e; ++i) fn(i, t);
                }
            } catch (...) {
                if (!failed.exchange(true)) err = std::current_exception();
            }
        });
    }
    for (auto& th : pool) th.join();
    if (err) std::rethrow_exception(err);
}

inline int resolve_threads(int requested)
{
    if (requested > 0) return requested;
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)hc : 1;
}

}  // namespace p2m
