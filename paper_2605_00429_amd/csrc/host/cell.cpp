#include "cell.h"

#include "clip_core.h"

#include <algorithm>
#include <cmath>

namespace p2m {

void ClipCell::seal(Face& f) const
{
    d3 c{0, 0, 0};
    for (int32_t i = 0; i < f.count; ++i) c = c + v_[f.begin + i];
    c = c * (1.0 / f.count);
    double r2 = 0;
    for (int32_t i = 0; i < f.count; ++i) r2 = std::max(r2, norm2(v_[f.begin + i] - c));
    f.c = c;
    f.r = std::sqrt(r2) * kSealInflate;
}

void ClipCell::compact()
{
    tmp_.clear();
    for (Face& f : faces_) {
        const int32_t nb = (int32_t)tmp_.size();
        for (int32_t i = 0; i < f.count; ++i) tmp_.push_back(v_[f.begin + i]);
        f.begin = nb;
    }
    v_.swap(tmp_);
}

void ClipCell::init_box(d3 lo, d3 hi)
{
    faces_.clear();
    v_.clear();
    auto add = [&](int32_t id, std::initializer_list<d3> pts) {
        Face f{id, (int32_t)v_.size(), (int32_t)pts.size(), {0, 0, 0}, 0};
        for (const d3& p : pts) v_.push_back(p);
        seal(f);
        faces_.push_back(f);
    };
    add(-1, {{lo.x, lo.y, lo.z}, {lo.x, lo.y, hi.z}, {lo.x, hi.y, hi.z}, {lo.x, hi.y, lo.z}});
    add(-2, {{hi.x, lo.y, lo.z}, {hi.x, hi.y, lo.z}, {hi.x, hi.y, hi.z}, {hi.x, lo.y, hi.z}});
    add(-3, {{lo.x, lo.y, lo.z}, {hi.x, lo.y, lo.z}, {hi.x, lo.y, hi.z}, {lo.x, lo.y, hi.z}});
    add(-4, {{lo.x, hi.y, lo.z}, {lo.x, hi.y, hi.z}, {hi.x, hi.y, hi.z}, {hi.x, hi.y, lo.z}});
    add(-5, {{lo.x, lo.y, lo.z}, {lo.x, hi.y, lo.z}, {hi.x, hi.y, lo.z}, {hi.x, lo.y, lo.z}});
    add(-6, {{lo.x, lo.y, hi.z}, {hi.x, lo.y, hi.z}, {hi.x, hi.y, hi.z}, {lo.x, hi.y, hi.z}});
    live_ = v_.size();
    scale_ = std::sqrt(max_norm2());
}

double ClipCell::max_norm2() const
{
    double m = 0;
    for (const Face& f : faces_)
        for (int32_t i = 0; i < f.count; ++i) m = std::max(m, norm2(v_[f.begin + i]));
    return m;
}

bool ClipCell::clip(d3 n, double h, int32_t id)
{
    const double nn = norm(n);
    if (!(nn > 0)) return false;
    const double eps = kClipEps * nn * scale_;
    cut_.clear();
    bool changed = false;
    for (size_t fi = 0; fi < faces_.size();) {
        Face& f = faces_[fi];
        // strictly inside, no vertex within eps of the plane: untouched
        if (dot(n, f.c) - h + nn * f.r < -eps) {
            ++fi;
            continue;
        }
        sd_.resize(f.count);
        bool out = false;
        for (int32_t i = 0; i < f.count; ++i) {
            sd_[i] = dot(n, v_[f.begin + i]) - h;
            out |= sd_[i] > eps;
        }
        if (!out) {
            // vertices on the plane belong to the new face
            for (int32_t i = 0; i < f.count; ++i)
                if (sd_[i] >= -eps) cut_.push_back(v_[f.begin + i]);
            ++fi;
            continue;
        }
        changed = true;
        const int32_t nb = (int32_t)v_.size();
        for (int32_t i = 0; i < f.count; ++i) {
            const int32_t ia = i, ib = (i + 1) % f.count;
            const double sa = sd_[ia], sb = sd_[ib];
            const d3 va = v_[f.begin + ia], vb = v_[f.begin + ib];
            if (sa <= eps) {
                v_.push_back(va);
                if (sa >= -eps) cut_.push_back(va);
            }
            if ((sa < -eps && sb > eps) || (sa > eps && sb < -eps)) {
                // Interpolate from the inside end to the outside end so that
                // both faces sharing this edge produce the same point.
                const bool a_in = sa < 0;
                const d3 pin = a_in ? va : vb;
                const d3 pout = a_in ? vb : va;
                const double sin_ = a_in ? sa : sb, sout = a_in ? sb : sa;
                const double t = sin_ / (sin_ - sout);
                const d3 x = pin + (pout - pin) * t;
                v_.push_back(x);
                cut_.push_back(x);
            }
        }
        const int32_t cnt = (int32_t)v_.size() - nb;
        live_ -= (size_t)f.count;
        if (cnt >= 3) {
            f.begin = nb;
            f.count = cnt;
            seal(f);
            live_ += (size_t)cnt;
            ++fi;
        } else {
            // dropped; the faces after it keep their order
            v_.resize(nb);
            faces_.erase(faces_.begin() + (std::ptrdiff_t)fi);
        }
    }
    if (!changed) return false;

    // The new face: the cut points ordered by angle around their centroid
    // (by diamond_angle, ties by the order the faces gave them).
    if (cut_.size() >= 3) {
        d3 c{0, 0, 0};
        for (const d3& p : cut_) c = c + p;
        c = c * (1.0 / cut_.size());
        const d3 nh = n * (1.0 / nn);
        d3 ax = std::fabs(nh.x) < 0.57 ? d3{1, 0, 0} : (std::fabs(nh.y) < 0.57 ? d3{0, 1, 0} : d3{0, 0, 1});
        d3 u = cross(nh, ax);
        u = u * (1.0 / norm(u));
        const d3 w = cross(nh, u);
        std::vector<std::pair<double, int32_t>> ang(cut_.size());
        for (size_t i = 0; i < cut_.size(); ++i) {
            const d3 r = cut_[i] - c;
            ang[i] = {diamond_angle(dot(r, u), dot(r, w)), (int32_t)i};
        }
        std::sort(ang.begin(), ang.end());
        const double tol2 = (kMergeTol * scale_) * (kMergeTol * scale_);
        const int32_t nb = (int32_t)v_.size();
        for (const auto& e : ang) {
            const d3& p = cut_[e.second];
            if ((int32_t)v_.size() > nb && norm2(p - v_.back()) <= tol2) continue;
            v_.push_back(p);
        }
        while ((int32_t)v_.size() - nb > 1 && norm2(v_.back() - v_[nb]) <= tol2) v_.pop_back();
        const int32_t cnt = (int32_t)v_.size() - nb;
        if (cnt >= 3) {
            Face f{id, nb, cnt, {0, 0, 0}, 0};
            seal(f);
            faces_.push_back(f);
            live_ += (size_t)cnt;
        } else {
            v_.resize(nb);
        }
    }
    if (v_.size() > 2 * live_ + 1024) compact();
    return true;
}

void ClipCell::corners(std::vector<d3>& out) const
{
    out.clear();
    for (const Face& f : faces_) out.insert(out.end(), v_.begin() + f.begin, v_.begin() + f.begin + f.count);
    std::sort(out.begin(), out.end(), [](const d3& a, const d3& b) {
        if (a.x != b.x) return a.x < b.x;
        if (a.y != b.y) return a.y < b.y;
        return a.z < b.z;
    });
    const double tol = kMergeTol * scale_;
    const double tol2 = tol * tol;
    std::vector<char> dup(out.size(), 0);
    for (size_t i = 0; i < out.size(); ++i) {
        if (dup[i]) continue;
        for (size_t j = i + 1; j < out.size() && out[j].x - out[i].x <= tol; ++j)
            if (!dup[j] && norm2(out[j] - out[i]) <= tol2) dup[j] = 1;
    }
    size_t k = 0;
    for (size_t i = 0; i < out.size(); ++i)
        if (!dup[i]) out[k++] = out[i];
    out.resize(k);
}

void ClipCell::face_ids(std::vector<int32_t>& out) const
{
    out.clear();
    const double min_area = (kMinArea * scale_) * (kMinArea * scale_);
    for (const Face& f : faces_) {
        d3 a{0, 0, 0};
        const d3& p0 = v_[f.begin];
        for (int32_t i = 1; i + 1 < f.count; ++i)
            a = a + cross(v_[f.begin + i] - p0, v_[f.begin + i + 1] - p0);
        if (0.5 * norm(a) > min_area) out.push_back(f.id);
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
}

}  // namespace p2m
