// P2M++ preprocessing (Sec. 3.2 and 3.3 of the paper), host side.
//
//  1. Sites: the referenced mesh vertices (one site per distinct position).
//  2. Voronoi cells: each site's cell inside the domain box, by clipping the
//     box with bisector half-spaces (kNN candidates first, then exact
//     "is a site closer than s to this corner" checks until every corner
//     is final).  The planes that bound a face are the site's Delaunay
//     neighbours, used by the locate walk.
//  3. Ring-based augmentation (Sec. 3.2): a uniform grid of scale tau counts
//     Voronoi vertices; a dense grid cell gets a central site at the
//     cluster's centroid plus sites on an enclosing sphere; sites that come
//     too close to an accepted one are dropped (the overlap rule), and so is
//     any auxiliary site whose cell would reach the domain box.
//  4. Interception lists (Sec. 3.3): for an on-surface site v, every
//     triangle meeting the union of the balls B(u, |u - v|) over the cell
//     corners u (the Vertex Sphere Union theorem, Eq. (3)); for an auxiliary
//     site s, reference point proj(s, M), either the single conservative
//     sphere of Eq. (8) or the same corner-ball union about proj(s, M).
//     Radii are inflated by delta so that rounding never loses a triangle.
//  5. Per-triangle bounding spheres (Sec. 3.4, pruning) and, per list entry,
//     ell = |s - c| - r, by which each list is sorted so that the query can
//     stop once ell - |q - s| >= d_min (triangle inequality).
//  6. Device layout: triangles in BVH leaf order, sites in Morton order,
//     seed grid of exact nearest sites for the locate walk's start.
#include "build.h"

#include <chrono>
#include <cstring>
#include <limits>
#include <numeric>
#include <unordered_map>

#include "bvh.h"
#include "cell.h"
#include "kdtree.h"
#include "octree.h"

namespace p2m {

namespace {

using clk = std::chrono::steady_clock;
double secs_since(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }

float round_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}

float round_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

float ibits(int32_t i)
{
    float f;
    std::memcpy(&f, &i, 4);
    return f;
}

uint64_t spread21(uint64_t x)
{
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

uint64_t morton_of(d3 p, d3 lo, double inv)
{
    auto q = [&](double v, double l) {
        double t = (v - l) * inv;
        t = std::min(std::max(t, 0.0), 2097151.0);
        return (uint64_t)t;
    };
    return spread21(q(p.x, lo.x)) | (spread21(q(p.y, lo.y)) << 1) | (spread21(q(p.z, lo.z)) << 2);
}

// Smallest sphere containing triangle (a, b, c): centre of the longest edge
// for a right or obtuse (or degenerate) triangle, else the circumcentre.
d3 min_sphere_center(d3 a, d3 b, d3 c)
{
    const double ab = norm2(b - a), bc = norm2(c - b), ca = norm2(a - c);
    if (ab >= bc + ca) return (a + b) * 0.5;
    if (bc >= ab + ca) return (b + c) * 0.5;
    if (ca >= ab + bc) return (c + a) * 0.5;
    const d3 e1 = b - a, e2 = c - a, n = cross(e1, e2);
    const double n2 = norm2(n);
    if (!(n2 > 0)) return (a + b) * 0.5;
    return a + cross(e2 * norm2(e1) - e1 * norm2(e2), n) * (1.0 / (2.0 * n2));
}

bool d3_less(const d3& a, const d3& b)
{
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
}

// Per-thread scratch of the list stage.
struct CellWork {
    std::vector<d3> corners;
    std::vector<int32_t> faces;
    std::vector<Ball> balls;
    std::vector<int32_t> list;
    std::vector<uint32_t> stamp;
    uint32_t gen = 0;
};

// The host implementation of CheckFn.
void host_corner_checks(const CornerChecks& job, int nth, std::vector<int32_t>& out)
{
    out.assign(job.q.size(), -1);
    parallel_for((int64_t)job.q.size(), nth, [&](int64_t i, int) {
        const int32_t l = job.list[i];
        const int32_t* ex = job.excl.data();
        out[i] = job.kd->below(job.q[i], job.limit2[i], ex + job.excl_off[l], ex + job.excl_off[l + 1], job.budget);
    }, 64);
}

constexpr int kKnn = 24;
// Sites one corner check of the first (density) pass may examine; ordinary
// checks examine a few dozen.
constexpr int64_t kPass1Budget = 4096;
// A budgeted cell that has gained more faces than this stops refining and
// counts as unresolved.  Before the auxiliary sites exist, the cell of a
// vertex on a rotational axis (the centre of a cylinder's cap) is cut by
// nearly every vertex of the wall, and clipping tens of thousands of faces
// one plane at a time is quadratic; such cells are built again, exactly,
// once the auxiliary sites cut them off.
constexpr int32_t kPass1MaxFaces = 4096;
// Float32 input positions break exact co-sphericity at the 1e-7 level; a
// violation smaller than this is rounding noise of a degenerate corner.
constexpr double kCornerSlack = 1e-6;
// Sites whose cells are in progress at once (bounds the memory of the
// clipped polytopes kept between check rounds).
constexpr int64_t kCellChunk = 32768;
// Sites whose cells one device call builds.
constexpr int64_t kDeviceCellChunk = int64_t(1) << 20;

// One cell under construction: the clipped polytope, the sites tried so far
// (sorted; the exclusion list of its checks), the corners found final, and
// the corners checked in the current round.
struct CellState {
    ClipCell cell;
    std::vector<int32_t> tested;
    std::vector<d3> verified, pending;
    double dK2 = 0;
    int64_t first = 0;  // index of its first check in the round's batch
    bool active = false, unresolved = false;
};

// Squared distance below which a site is closer to corner x (relative to
// the site) than the site itself, by more than the slack: a site closer
// than s by less than kCornerSlack (relative, in squared distance) is
// skipped, so that the cell stays a superset of the exact one; the walk's
// stop region and the lists are both built from this computed cell.
inline double corner_limit(d3 x) { return norm2(x) * (1.0 - kCornerSlack); }

// Corners of the current polytope that still need a check: beyond half of
// the kNN radius (closer ones cannot be cut by a site outside the kNN) and
// not verified before.  Verified corners stay valid: clipping only removes
// corners and adds new ones (bitwise copies survive).
void collect_pending(CellState& c, std::vector<d3>& corners)
{
    c.pending.clear();
    c.cell.corners(corners);
    for (const d3& x : corners) {
        if (4.0 * norm2(x) <= c.dK2) continue;
        if (std::binary_search(c.verified.begin(), c.verified.end(), x, d3_less)) continue;
        c.pending.push_back(x);
    }
}

// Applies one round's results to a cell (results in the order of
// c.pending): a check that gave up marks the cell unresolved, a site found
// is clipped by, a corner with no closer site is final.  The cell stays in
// progress, with its new corners pending, when some site was found.
template <class Res>
void apply_round(CellState& c, const Res& res, const std::vector<d3>& P, d3 ps, bool budgeted,
                 std::vector<int32_t>& found, std::vector<d3>& corners)
{
    found.clear();
    for (size_t k = 0; k < c.pending.size(); ++k) {
        const int32_t f = res(k);
        if (f == -2) c.unresolved = true;
        else if (f >= 0) found.push_back(f);
        else c.verified.push_back(c.pending[k]);
    }
    std::sort(c.verified.begin(), c.verified.end(), d3_less);
    if (found.empty()) {
        c.active = false;
        c.pending.clear();
        return;
    }
    std::sort(found.begin(), found.end());
    found.erase(std::unique(found.begin(), found.end()), found.end());
    for (int32_t f : found) {
        const d3 nv = P[f] - ps;
        c.cell.clip(nv, 0.5 * norm2(nv), f);
        c.tested.insert(std::upper_bound(c.tested.begin(), c.tested.end(), f), f);
    }
    if (budgeted && c.cell.n_faces() > kPass1MaxFaces) {
        c.unresolved = true;
        c.active = false;
        c.pending.clear();
        return;
    }
    collect_pending(c, corners);
}

// Cells still in progress below this count finish on the host: such a tail
// (cells near a rotational axis that gain neighbours a few at a time) needs
// many rounds of a few checks each, where a device round trip per round
// costs more than the checks.
constexpr int64_t kHostTail = 256;

// Per-thread scratch of the Voronoi stage.
struct CellScratch {
    std::vector<std::pair<double, int32_t>> knn;
    std::vector<d3> corners;
    std::vector<int32_t> found;
    std::vector<int32_t> res;
};

// Step 1 of a cell: the box clipped by the bisectors of the site's kNN in
// order of distance, stopping once the next site is beyond twice the
// farthest corner; the cell stays in progress, with the corners that a site
// outside the kNN could still cut pending, unless that stop came first.
void start_cell(CellState& c, int32_t s, const std::vector<d3>& P, const KdTree& kd, d3 blo, d3 bhi,
                CellScratch& w)
{
    const d3 ps = P[s];
    c.cell.init_box(blo - ps, bhi - ps);
    kd.knn(ps, kKnn, s, w.knn);
    c.tested.push_back(s);
    double r2max = c.cell.max_norm2();
    bool final_by_radius = false;
    for (const auto& e : w.knn) {
        // a site at distance >= 2 * max corner radius cannot cut the cell
        if (e.first >= 4.0 * r2max) {
            final_by_radius = true;
            break;
        }
        const d3 nv = P[e.second] - ps;
        if (c.cell.clip(nv, 0.5 * norm2(nv), e.second)) r2max = c.cell.max_norm2();
        c.tested.push_back(e.second);
    }
    std::sort(c.tested.begin(), c.tested.end());
    // sites beyond the kNN radius can only cut corners farther than half of it
    c.active = !final_by_radius && (int)w.knn.size() == kKnn;
    if (c.active) {
        c.dK2 = w.knn.back().first;
        collect_pending(c, w.corners);
    }
}

// The remaining rounds of one cell, its checks answered by KdTree::below
// (the answers a batch of CornerChecks gives).
void finish_cell(CellState& c, int32_t s, const std::vector<d3>& P, const KdTree& kd, int64_t budget,
                 size_t round, CellScratch& w)
{
    const d3 ps = P[s];
    for (size_t r = round; c.active && r <= P.size(); ++r) {
        w.res.resize(c.pending.size());
        for (size_t k = 0; k < c.pending.size(); ++k)
            w.res[k] = kd.below(ps + c.pending[k], corner_limit(c.pending[k]), c.tested.data(),
                                c.tested.data() + c.tested.size(), budget);
        apply_round(c, [&](size_t k) { return w.res[k]; }, P, ps, budget >= 0, w.found, w.corners);
    }
}

using CellDone = std::function<void(int64_t, int, const std::vector<d3>&, const std::vector<int32_t>&, bool, bool)>;

void cell_done(CellState& c, int64_t i, int tid, CellScratch& w, const CellDone& done)
{
    std::vector<int32_t> faces;
    c.cell.corners(w.corners);
    c.cell.face_ids(faces);
    done(i, tid, w.corners, faces, !c.cell.empty(), c.unresolved);
    c = CellState();
}

// Voronoi cells of the sites in `sites` (indices into P) clipped to the box
// [blo, bhi], by rounds:
//   1. each cell clips the box by the bisectors of its kNN (start_cell);
//   2. every corner that a site outside the kNN could still cut is checked
//      (CornerChecks: the nearest site closer to it than the cell's own, or
//      none); the checks of all cells in progress go out as one batch;
//   3. each cell clips by the sites its checks found and collects its new
//      corners; cells with nothing found are final.  Rounds repeat until
//      no cell is in progress; the last few cells run their remaining
//      rounds on the host (KdTree::below gives the same answers).
// A cell's steps depend on that cell alone, so batching changes nothing:
// with `cells`, a device builds each chunk of cells whole, the same way,
// and the host builds only the cells it hands back.
// With budget >= 0 each check examines at most that many sites, and a cell
// stops refining past kPass1MaxFaces faces; a check that gives up, or that
// cap, leaves the cell a superset and marks it unresolved.  That
// happens at corners that nearly all sites are almost equidistant from
// (the centre of a sphere tessellation, the axis of a cylinder).  done(i,
// tid, corners, faces, ok, unresolved) receives sites[i]'s cell inside a
// parallel loop.
void compute_cells(const std::vector<int32_t>& sites, const std::vector<d3>& P, const KdTree& kd, d3 blo, d3 bhi,
                   int64_t budget, int nth, const CheckFn& check, bool host_tail, const CellFn* cells, int64_t pass,
                   p2m_stats& stats, const CellDone& done)
{
    std::vector<CellScratch> scr(nth);
    const int64_t n = (int64_t)sites.size();
    if (kd.depth() + 1 > KdTree::kBelowStack) throw Error(P2M_ERR_INTERNAL, "site tree too deep");
    // the device keeps its cells in its own memory, so its chunks are
    // larger (the host keeps only their corners and face sites)
    const int64_t step = cells ? kDeviceCellChunk : kCellChunk;
    for (int64_t c0 = 0; c0 < n; c0 += step) {
        const int64_t m = std::min(step, n - c0);
        if (cells) {
            CellJob job;
            job.kd = &kd;
            job.sites = sites.data() + c0;
            job.n = m;
            job.blo = blo;
            job.bhi = bhi;
            job.budget = budget;
            job.max_faces = kPass1MaxFaces;
            job.knn = kKnn;
            job.slack = kCornerSlack;
            job.pass = pass;
            CellResult r;
            (*cells)(job, r);
            const int64_t n_redo = std::count(r.redo.begin(), r.redo.end(), (char)1);
            stats.n_cells_device += m - n_redo;
            stats.n_cells_host += n_redo;
            parallel_for(m, nth, [&](int64_t i, int tid) {
                if (r.redo[i]) {
                    CellState c;
                    start_cell(c, sites[c0 + i], P, kd, blo, bhi, scr[tid]);
                    finish_cell(c, sites[c0 + i], P, kd, budget, 0, scr[tid]);
                    cell_done(c, c0 + i, tid, scr[tid], done);
                    return;
                }
                const std::vector<d3> corners(r.corners.begin() + r.corner_off[i],
                                              r.corners.begin() + r.corner_off[i + 1]);
                const std::vector<int32_t> faces(r.faces.begin() + r.face_off[i], r.faces.begin() + r.face_off[i + 1]);
                done(c0 + i, tid, corners, faces, r.ok[i] != 0, r.unresolved[i] != 0);
            }, 4);
            continue;
        }
        stats.n_cells_host += m;
        std::vector<CellState> st(m);
        parallel_for(m, nth, [&](int64_t i, int tid) {
            start_cell(st[i], sites[c0 + i], P, kd, blo, bhi, scr[tid]);
        }, 16);
        std::vector<int64_t> act;
        for (int64_t i = 0; i < m; ++i)
            if (st[i].active) act.push_back(i);
        for (size_t round = 0; !act.empty() && round <= P.size(); ++round) {
            if (host_tail && (int64_t)act.size() <= kHostTail) {
                // the tail: each cell runs its remaining rounds by itself
                parallel_for((int64_t)act.size(), nth, [&](int64_t j, int tid) {
                    finish_cell(st[act[j]], sites[c0 + act[j]], P, kd, budget, round, scr[tid]);
                }, 1);
                act.clear();
                break;
            }
            // one batch of checks over every cell in progress
            CornerChecks job;
            job.kd = &kd;
            job.budget = budget;
            job.excl_off.push_back(0);
            for (int64_t i : act) {
                CellState& c = st[i];
                c.first = (int64_t)job.q.size();
                const int32_t list = (int32_t)job.excl_off.size() - 1;
                const d3 ps = P[sites[c0 + i]];
                for (const d3& x : c.pending) {
                    job.q.push_back(ps + x);
                    job.limit2.push_back(corner_limit(x));
                    job.list.push_back(list);
                }
                job.excl.insert(job.excl.end(), c.tested.begin(), c.tested.end());
                job.excl_off.push_back((int64_t)job.excl.size());
            }
            std::vector<int32_t> res;
            check(job, res);
            parallel_for((int64_t)act.size(), nth, [&](int64_t j, int tid) {
                CellState& c = st[act[j]];
                CellScratch& w = scr[tid];
                const int64_t first = c.first;
                apply_round(c, [&](size_t k) { return res[first + (int64_t)k]; }, P, P[sites[c0 + act[j]]],
                            budget >= 0, w.found, w.corners);
            }, 16);
            std::vector<int64_t> next;
            for (int64_t i : act)
                if (st[i].active) next.push_back(i);
            act.swap(next);
        }
        parallel_for(m, nth, [&](int64_t i, int tid) { cell_done(st[i], c0 + i, tid, scr[tid], done); }, 16);
    }
}

// Eigenvectors of a symmetric 3x3 matrix (xx, xy, xz, yy, yz, zz) by
// cyclic Jacobi rotations; returns the eigenvalues in w and the vectors as
// the columns of v.
void sym3_eigen(const double c[6], double w[3], double v[3][3])
{
    double a[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double on = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-30 * on || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = 0.5 * std::atan2(2.0 * a[p][q], a[q][q] - a[p][p]);
                const double cs = std::cos(th), sn = std::sin(th);
                for (int k = 0; k < 3; ++k) {  // columns p, q
                    const double kp = a[k][p], kq = a[k][q];
                    a[k][p] = cs * kp - sn * kq;
                    a[k][q] = sn * kp + cs * kq;
                }
                for (int k = 0; k < 3; ++k) {  // rows p, q
                    const double pk = a[p][k], qk = a[q][k];
                    a[p][k] = cs * pk - sn * qk;
                    a[q][k] = sn * pk + cs * qk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double kp = v[k][p], kq = v[k][q];
                    v[k][p] = cs * kp - sn * kq;
                    v[k][q] = sn * kp + cs * kq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) w[i] = a[i][i];
}

// A cluster of Voronoi vertices is read as a line (the axis of a cylinder,
// a cone or a latitude-ring stack, or locally the core circle of a torus)
// when its covariance has one eigenvalue at least four times the next;
// then *axis is that eigenvector.
bool elongated_axis(const double cov[6], d3& axis)
{
    double w[3], v[3][3];
    sym3_eigen(cov, w, v);
    int i0 = 0;
    for (int i = 1; i < 3; ++i)
        if (w[i] > w[i0]) i0 = i;
    double second = -INFINITY;
    for (int i = 0; i < 3; ++i)
        if (i != i0) second = std::max(second, w[i]);
    if (!(w[i0] > 0.0) || w[i0] < 4.0 * std::max(second, 0.0)) return false;
    axis = d3{v[0][i0], v[1][i0], v[2][i0]};
    const double n = norm(axis);
    if (!(n > 0)) return false;
    axis = axis * (1.0 / n);
    return true;
}

// Auxiliary sites of one dense cluster at pc, whose distance to the mesh is
// d_wall: layers at radii d_wall / 2, d_wall / 4, ... (at least tau, at
// most `layers` of them; one layer at d_wall / 2 when that is below tau).
// A line cluster (axis given) gets rings in the plane through pc normal to
// the axis, a point cluster spherical shells, each with sites about tau
// apart (rings at least min_ring sites).  Vertex cells that reached the
// cluster end at the outermost layer, where each ring site's cell spans a
// small angle about the cluster, so that no cell near the cluster keeps a
// corner from which the whole surrounding wall is almost equidistant.
template <class Emit>
void ring_layer_sites(d3 pc, const d3* axis, double d_wall, double tau, int layers, int min_ring, Emit emit)
{
    double rho = 0.5 * d_wall;
    if (!(rho > 0)) return;
    d3 u{1, 0, 0}, v{0, 1, 0};
    if (axis) {
        const d3 a = *axis;
        const d3 e = std::fabs(a.x) < 0.6 ? d3{1, 0, 0} : (std::fabs(a.y) < 0.6 ? d3{0, 1, 0} : d3{0, 0, 1});
        u = cross(a, e);
        u = u * (1.0 / norm(u));
        v = cross(a, u);
    }
    for (int k = 0; k < layers; ++k) {
        if (k > 0 && rho < tau) break;
        if (axis) {
            const int m = std::max(min_ring, (int)std::ceil(2.0 * M_PI * rho / tau));
            const double sep = 0.5 * std::min(tau, 2.0 * M_PI * rho / m);
            const double off = (k % 2) ? 0.5 : 0.0;
            for (int j = 0; j < m; ++j) {
                const double ph = 2.0 * M_PI * (j + off) / m;
                emit(pc + (u * std::cos(ph) + v * std::sin(ph)) * rho, sep);
            }
        } else {
            const int m = std::max(12, (int)std::ceil(4.0 * M_PI * rho * rho / (tau * tau)));
            const double sep = 0.5 * std::min(tau, rho * std::sqrt(4.0 * M_PI / m));
            for (int j = 0; j < m; ++j) {
                // golden-spiral directions
                const double z = 1.0 - 2.0 * (j + 0.5) / m;
                const double r = std::sqrt(std::max(0.0, 1.0 - z * z));
                const double ph = j * 2.399963229728653 + 0.5 * k;
                emit(pc + d3{r * std::cos(ph), r * std::sin(ph), z} * rho, sep);
            }
        }
        rho *= 0.5;
    }
}

void check_mesh(const p2m_mesh_desc& m)
{
    if (m.n_vertices < 0 || m.n_triangles < 0) throw Error(P2M_ERR_INVALID_ARG, "negative mesh size");
    if (m.n_triangles == 0) throw Error(P2M_ERR_BAD_MESH, "mesh has no triangles");
    if (!m.vertices || !m.triangles) throw Error(P2M_ERR_INVALID_ARG, "null mesh array");
    if (m.n_vertices > std::numeric_limits<int32_t>::max() || m.n_triangles > (int64_t(1) << 29))
        throw Error(P2M_ERR_OOM, "mesh too large for 32-bit indices");
    for (int64_t i = 0; i < 3 * m.n_triangles; ++i) {
        const int32_t v = m.triangles[i];
        if (v < 0 || v >= m.n_vertices)
            throw Error(P2M_ERR_BAD_MESH, "triangle " + std::to_string(i / 3) + " has vertex index " +
                                              std::to_string(v) + " out of range");
    }
}

}  // namespace

void build_host(const p2m_mesh_desc& mesh, const p2m_build_opts& o, HostStructure& H, const GpuListFn* gpu,
                const CheckFn* gpu_checks, const CellFn* gpu_cells)
{
    const auto t_start = clk::now();
    check_mesh(mesh);
    if (!(o.domain_scale >= 1.0f) || !(o.tau_scale > 0) || o.ring_sites < 0 || o.ring_layers < 0 ||
        !(o.list_inflation_rel >= 0) || !(o.seed_cell_scale > 0) || o.seed_max_cells < 1 ||
        o.decomposition < 0 || o.decomposition > 1 || o.octree_max_list < 1 || o.octree_max_depth < 0 ||
        o.octree_max_depth > 16 || o.gpu_voronoi < 0 || o.gpu_voronoi > 2 || o.gpu_cell_pass < 0)
        throw Error(P2M_ERR_INVALID_ARG, "invalid build option");
    const int nth = resolve_threads(o.n_threads);
    const int64_t nV = mesh.n_vertices, nT = mesh.n_triangles;
    H.n_vertices = nV;
    H.n_triangles = nT;

    // ---- sites: distinct positions of referenced vertices
    std::vector<char> used(nV, 0);
    for (int64_t i = 0; i < 3 * nT; ++i) used[mesh.triangles[i]] = 1;
    std::vector<int32_t> ref;
    for (int64_t v = 0; v < nV; ++v)
        if (used[v]) {
            const float* p = mesh.vertices + 3 * v;
            if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]))
                throw Error(P2M_ERR_BAD_MESH, "vertex " + std::to_string(v) + " is not finite");
            ref.push_back((int32_t)v);
        }
    std::sort(ref.begin(), ref.end(), [&](int32_t a, int32_t b) {
        const float* p = mesh.vertices + 3 * (int64_t)a;
        const float* q = mesh.vertices + 3 * (int64_t)b;
        if (p[0] != q[0]) return p[0] < q[0];
        if (p[1] != q[1]) return p[1] < q[1];
        if (p[2] != q[2]) return p[2] < q[2];
        return a < b;
    });
    std::vector<d3> P;
    H.site_of_vertex.assign(nV, -1);
    std::vector<int32_t> site_vertex;  // a representative vertex per vertex site
    for (size_t i = 0; i < ref.size(); ++i) {
        const float* p = mesh.vertices + 3 * (int64_t)ref[i];
        if (i == 0 || std::memcmp(p, mesh.vertices + 3 * (int64_t)ref[i - 1], 12) != 0) {
            P.push_back({p[0], p[1], p[2]});
            site_vertex.push_back(ref[i]);
        }
        H.site_of_vertex[ref[i]] = (int32_t)P.size() - 1;
    }
    const int32_t nVS = (int32_t)P.size();

    // ---- triangles (FP64 copies), boxes, edge length
    std::vector<d3> T(3 * nT);
    for (int64_t i = 0; i < 3 * nT; ++i) {
        const float* p = mesh.vertices + 3 * (int64_t)mesh.triangles[i];
        T[i] = {p[0], p[1], p[2]};
    }
    d3 mlo{INFINITY, INFINITY, INFINITY}, mhi{-INFINITY, -INFINITY, -INFINITY};
    for (const d3& p : P) {
        mlo = dmin3(mlo, p);
        mhi = dmax3(mhi, p);
    }
    double diag = norm(mhi - mlo);
    if (!(diag > 0)) diag = 1.0;
    H.diag = diag;
    double edge_sum = 0;
    for (int64_t t = 0; t < nT; ++t)
        edge_sum += norm(T[3 * t + 1] - T[3 * t]) + norm(T[3 * t + 2] - T[3 * t + 1]) + norm(T[3 * t] - T[3 * t + 2]);
    double mean_edge = edge_sum / (3.0 * nT);
    if (!(mean_edge > 0)) mean_edge = diag * 1e-3;
    const d3 mc = (mlo + mhi) * 0.5;
    auto padded_box = [&](double scale, d3& lo, d3& hi) {
        d3 h = (mhi - mlo) * (0.5 * scale);
        const double floor_h = 0.05 * diag * scale;
        h = {std::max(h.x, floor_h), std::max(h.y, floor_h), std::max(h.z, floor_h)};
        lo = mc - h;
        hi = mc + h;
    };
    d3 blo, bhi;
    padded_box(o.domain_scale, blo, bhi);
    for (int k = 0; k < 3; ++k) {
        H.dlo[k] = round_up(comp(blo, k));    // query box slightly inside the clip box
        H.dhi[k] = round_down(comp(bhi, k));
    }
    const double delta = (double)o.list_inflation_rel * diag;

    auto t0 = clk::now();
    Bvh bvh;
    bvh.build(T, nth);
    KdTree kd;
    kd.build(P, nth);
    std::vector<CellWork> work(nth);
    for (auto& w : work) w.stamp.assign(nT, 0);
    const CheckFn checks = gpu_checks ? *gpu_checks
                                      : CheckFn([nth](const CornerChecks& job, std::vector<int32_t>& out) {
                                            host_corner_checks(job, nth, out);
                                        });

    const bool octree = o.decomposition == 1;
    std::vector<char> is_aux(P.size(), 0);
    std::vector<std::vector<int32_t>> nbr, lists;
    int32_t nS = 0;
    int64_t n_dense = 0;
    OctreeCells oc;
    if (octree) {
        // ---- octree decomposition: leaves are the cells, no Voronoi stage
        d3 olo, ohi;
        padded_box(1.25, olo, ohi);
        build_octree(T, bvh, olo, ohi, delta, o.octree_max_list, o.octree_max_depth, nth, oc);
        P = oc.centre;
        nS = (int32_t)P.size();
        nbr.assign(nS, {});
        lists.swap(oc.lists);
        is_aux.assign(nS, 1);
        std::fill(H.site_of_vertex.begin(), H.site_of_vertex.end(), -1);
        // queries outside the root cube take the BVH fallback
        for (int k = 0; k < 3; ++k) {
            H.dlo[k] = oc.root[k] - oc.root[3];
            H.dhi[k] = oc.root[k] + oc.root[3];
        }
        H.stats.t_lists_s = secs_since(t0);
    } else {
    // ---- pass 1 and ring-based augmentation (Sec. 3.2)
    // Cells (corners relative to the site, bounding-plane ids) of every site.
    std::vector<std::vector<d3>> cell_corners(P.size());
    std::vector<std::vector<int32_t>> cell_faces(P.size());
    std::vector<char> cell_ok(P.size(), 0), cell_done(P.size(), 0), unresolved(P.size(), 0);
    double t_vor1 = 0;
    if (o.augment && nVS >= 5) {
        const double tau = o.tau_scale * mean_edge;
        struct Acc {
            int64_t n = 0;       // distinct sites with a Voronoi vertex in this grid cell
            int64_t nc = 0;      // Voronoi-vertex occurrences
            d3 s{0, 0, 0};
            double s2 = 0;
            double m[6] = {0, 0, 0, 0, 0, 0};  // second moments xx, xy, xz, yy, yz, zz
        };
        std::vector<std::unordered_map<uint64_t, Acc>> maps(nth);
        const double tolb = 1e-9 * norm(bhi - blo);
        const d3 glo = mlo - d3{tau, tau, tau};
        auto key_of = [&](d3 u) {
            const uint64_t ix = (uint64_t)((u.x - glo.x) / tau);
            const uint64_t iy = (uint64_t)((u.y - glo.y) / tau);
            const uint64_t iz = (uint64_t)((u.z - glo.z) / tau);
            return ix | (iy << 21) | (iz << 42);
        };
        const double gmax = 2097150.0 * tau;
        // Voronoi vertices of each cell that can seed a cluster, keyed by
        // their grid cell (sorted by key within the site)
        std::vector<std::vector<std::pair<uint64_t, d3>>> site_keys(nVS);
        std::vector<int32_t> vsites(nVS);
        std::iota(vsites.begin(), vsites.end(), 0);
        compute_cells(vsites, P, kd, blo, bhi, kPass1Budget, nth, checks, gpu_checks != nullptr, gpu_cells, o.gpu_cell_pass, H.stats,
                      [&](int64_t s, int, const std::vector<d3>& corners, const std::vector<int32_t>& faces, bool ok,
                          bool unres) {
            cell_corners[s] = corners;
            cell_faces[s] = faces;
            cell_ok[s] = ok;
            unresolved[s] = unres;
            const d3 ps = P[s];
            auto& kc = site_keys[s];
            for (const d3& x : corners) {
                const d3 u = ps + x;
                // finite Voronoi vertices only (not on the domain box)
                if (u.x <= blo.x + tolb || u.y <= blo.y + tolb || u.z <= blo.z + tolb ||
                    u.x >= bhi.x - tolb || u.y >= bhi.y - tolb || u.z >= bhi.z - tolb)
                    continue;
                // only clusters inside the mesh box can get auxiliary sites
                if (u.x < mlo.x || u.y < mlo.y || u.z < mlo.z || u.x > mhi.x || u.y > mhi.y || u.z > mhi.z)
                    continue;
                if (u.x - glo.x > gmax || u.y - glo.y > gmax || u.z - glo.z > gmax) continue;
                kc.push_back({key_of(u), u});
            }
            std::stable_sort(kc.begin(), kc.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        });
        // Per grid cell: distinct sites, vertex count and moments, summed in
        // site order (so that the sums do not depend on the thread count or
        // scheduling): the keys are split into buckets by value, each bucket
        // gathered in site order and summed by one thread.
        const int nb = std::max(1, nth) * 4;
        std::vector<std::vector<std::pair<uint64_t, d3>>> buckets(nb);
        std::vector<std::vector<int32_t>> bucket_site(nb);
        for (int32_t s = 0; s < nVS; ++s) {
            for (const auto& kv : site_keys[s]) {
                const int b = (int)((kv.first * 0x9E3779B97F4A7C15ull) >> 58) % nb;
                buckets[b].push_back(kv);
                bucket_site[b].push_back(s);
            }
            std::vector<std::pair<uint64_t, d3>>().swap(site_keys[s]);
        }
        parallel_for(nb, nth, [&](int64_t b, int tid) {
            auto& e = buckets[b];
            auto& es = bucket_site[b];
            std::vector<int64_t> ord(e.size());
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](int64_t i, int64_t j) { return e[i].first < e[j].first; });
            auto& mp = maps[tid];
            for (size_t k = 0; k < ord.size(); ++k) {
                const int64_t i = ord[k];
                Acc& a = mp[e[i].first];
                if (k == 0 || e[i].first != e[ord[k - 1]].first || es[i] != es[ord[k - 1]]) a.n++;
                a.nc++;
                const d3 u = e[i].second;
                a.s = a.s + u;
                a.s2 += norm2(u);
                a.m[0] += u.x * u.x;
                a.m[1] += u.x * u.y;
                a.m[2] += u.x * u.z;
                a.m[3] += u.y * u.y;
                a.m[4] += u.y * u.z;
                a.m[5] += u.z * u.z;
            }
        }, 1);
        // each key lives in one bucket, so merging the per-thread maps only
        // moves entries
        for (int t = 1; t < nth; ++t)
            for (auto& kv : maps[t]) maps[0][kv.first] = kv.second;
        t_vor1 = secs_since(t0);
        // Reference density: grid cells that hold mesh vertices (the
        // sampling density near the surface the paper scales tau by).
        std::unordered_map<uint64_t, char> site_cells;
        for (int32_t s = 0; s < nVS; ++s) site_cells[key_of(P[s])] = 1;
        std::vector<std::pair<uint64_t, Acc>> cells(maps[0].begin(), maps[0].end());
        maps.clear();
        std::sort(cells.begin(), cells.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        // every grid cell holding a mesh vertex counts, with 0 when no
        // Voronoi vertex falls in it (a cylinder's cells are radial wedges
        // with no vertex near the surface)
        std::vector<int64_t> counts;
        for (auto& c : cells)
            if (site_cells.count(c.first)) counts.push_back(c.second.n);
        counts.resize(site_cells.size(), 0);
        int64_t median = 0;
        if (!counts.empty()) {
            std::nth_element(counts.begin(), counts.begin() + counts.size() / 2, counts.end());
            median = counts[counts.size() / 2];
        }
        const double thr = std::max((double)o.dense_min_sites, (double)o.dense_rel * (double)median);
        // icosahedron directions for the enclosing sphere
        std::vector<d3> dirs;
        {
            const double g = (1.0 + std::sqrt(5.0)) / 2.0;
            const double ico[12][3] = {{-1, g, 0}, {1, g, 0}, {-1, -g, 0}, {1, -g, 0}, {0, -1, g}, {0, 1, g},
                                       {0, -1, -g}, {0, 1, -g}, {g, 0, -1}, {g, 0, 1}, {-g, 0, -1}, {-g, 0, 1}};
            const int nr = std::min(o.ring_sites, 12);
            for (int i = 0; i < nr; ++i) {
                d3 d{ico[i][0], ico[i][1], ico[i][2]};
                dirs.push_back(d * (1.0 / norm(d)));
            }
            // more than 12: golden-spiral directions
            for (int i = 12; i < o.ring_sites; ++i) {
                const double z = 1.0 - 2.0 * (i - 12 + 0.5) / (o.ring_sites - 12);
                const double r = std::sqrt(std::max(0.0, 1.0 - z * z));
                const double ph = i * 2.399963229728653;
                dirs.push_back({r * std::cos(ph), r * std::sin(ph), z});
            }
        }
        struct Cand {
            d3 p;
            double sep;
        };
        std::vector<Cand> centrals, rings;
        for (auto& c : cells) {
            if ((double)c.second.n < thr) continue;
            ++n_dense;
            const Acc& a = c.second;
            const d3 pc = a.s * (1.0 / a.nc);
            centrals.push_back({pc, 0.5 * tau});
            if (o.ring_layers <= 0) {
                // one enclosing sphere of ring_sites sites
                const double rms = std::sqrt(std::max(0.0, a.s2 / a.nc - norm2(pc)));
                const double rho = std::min(std::max(3.0 * rms, tau), 3.0 * tau);
                for (const d3& d : dirs) rings.push_back({pc + d * rho, 0.5 * rho});
                continue;
            }
            // Layered rings (see ring_layer_sites): the cluster's shape from
            // the covariance of its Voronoi vertices, the free radius from the
            // distance to the mesh.
            double cov[6];
            const double inv_n = 1.0 / (double)a.nc;
            const double mm[6] = {pc.x * pc.x, pc.x * pc.y, pc.x * pc.z, pc.y * pc.y, pc.y * pc.z, pc.z * pc.z};
            for (int k = 0; k < 6; ++k) cov[k] = a.m[k] * inv_n - mm[k];
            d3 axis;
            const bool line = elongated_axis(cov, axis);
            int32_t ct;
            d3 cp;
            const double d_wall = std::sqrt(bvh.closest(pc, &ct, &cp));
            ring_layer_sites(pc, line ? &axis : nullptr, d_wall, tau, o.ring_layers, std::max(o.ring_sites, 8),
                             [&](d3 p, double sep) { rings.push_back({p, sep}); });
        }
        // accept centrals first, then ring sites; the overlap rule drops a
        // candidate within its separation radius of an accepted one
        std::vector<d3> acc;
        const double cell_h = 0.25 * tau;
        std::unordered_map<uint64_t, std::vector<int32_t>> grid;
        auto gkey = [&](d3 p, int dx, int dy, int dz) {
            const int64_t ix = (int64_t)std::floor((p.x - glo.x) / cell_h) + dx;
            const int64_t iy = (int64_t)std::floor((p.y - glo.y) / cell_h) + dy;
            const int64_t iz = (int64_t)std::floor((p.z - glo.z) / cell_h) + dz;
            return (uint64_t)(ix & 0x1fffff) | ((uint64_t)(iy & 0x1fffff) << 21) | ((uint64_t)(iz & 0x1fffff) << 42);
        };
        const double min_site_sep = 1e-3 * mean_edge;
        auto try_accept = [&](const Cand& c) {
            if (c.p.x <= mlo.x || c.p.y <= mlo.y || c.p.z <= mlo.z || c.p.x >= mhi.x || c.p.y >= mhi.y || c.p.z >= mhi.z)
                return;
            const int reach = (int)std::ceil(c.sep / cell_h);
            for (int dx = -reach; dx <= reach; ++dx)
                for (int dy = -reach; dy <= reach; ++dy)
                    for (int dz = -reach; dz <= reach; ++dz) {
                        auto it = grid.find(gkey(c.p, dx, dy, dz));
                        if (it == grid.end()) continue;
                        for (int32_t j : it->second)
                            if (norm2(acc[j] - c.p) < c.sep * c.sep) return;
                    }
            double d2;
            kd.nearest(c.p, &d2);
            if (d2 < min_site_sep * min_site_sep) return;
            // round to float32 now: sites are stored and compared in float32 positions
            const d3 pf{(float)c.p.x, (float)c.p.y, (float)c.p.z};
            grid[gkey(pf, 0, 0, 0)].push_back((int32_t)acc.size());
            acc.push_back(pf);
        };
        for (const Cand& c : centrals) try_accept(c);
        for (const Cand& c : rings) try_accept(c);
        if (!acc.empty()) {
            // drop auxiliary sites whose cells reach the domain box (an
            // unbounded cell would get a list of the whole mesh)
            std::vector<d3> aux = acc;
            // Only cells next to a dropped site change when it goes, so each
            // iteration after the first rebuilds just those.
            std::vector<char> need(aux.size(), 1);
            std::vector<std::vector<int32_t>> anb(aux.size());  // aux neighbours (aux indices)
            for (int iter = 0; iter < 6 && !aux.empty(); ++iter) {
                std::vector<d3> PP = P;
                PP.insert(PP.end(), aux.begin(), aux.end());
                KdTree kd2;
                kd2.build(PP, nth);
                std::vector<char> drop(aux.size(), 0);
                std::vector<int32_t> asites;
                for (size_t i = 0; i < aux.size(); ++i)
                    if (need[i]) asites.push_back(nVS + (int32_t)i);
                compute_cells(asites, PP, kd2, blo, bhi, -1, nth, checks, gpu_checks != nullptr, gpu_cells, o.gpu_cell_pass, H.stats,
                              [&](int64_t j, int, const std::vector<d3>&, const std::vector<int32_t>& faces, bool ok,
                                  bool) {
                    const int32_t i = asites[j] - nVS;
                    if (faces.empty() || faces.front() < 0 || !ok) drop[i] = 1;
                    anb[i].clear();
                    for (int32_t f : faces)
                        if (f >= nVS) anb[i].push_back(f - nVS);
                });
                std::vector<int32_t> newid(aux.size(), -1);
                std::vector<d3> keep;
                for (size_t i = 0; i < aux.size(); ++i)
                    if (!drop[i]) {
                        newid[i] = (int32_t)keep.size();
                        keep.push_back(aux[i]);
                    }
                const bool stable = keep.size() == aux.size();
                std::vector<char> need2(keep.size(), 0);
                for (size_t i = 0; i < aux.size(); ++i) {
                    if (!drop[i]) continue;
                    for (int32_t f : anb[i])
                        if (newid[f] >= 0) need2[newid[f]] = 1;
                }
                for (size_t i = 0; i < aux.size(); ++i) {
                    if (drop[i]) continue;
                    for (int32_t f : anb[i])
                        if (drop[f]) need2[newid[i]] = 1;
                }
                std::vector<std::vector<int32_t>> anb2(keep.size());
                for (size_t i = 0; i < aux.size(); ++i) {
                    if (drop[i]) continue;
                    for (int32_t f : anb[i])
                        if (newid[f] >= 0) anb2[newid[i]].push_back(newid[f]);
                }
                aux.swap(keep);
                need.swap(need2);
                anb.swap(anb2);
                if (stable) break;
            }
            // Vertex cells reused from pass 1 unless an auxiliary site is
            // closer than the site to one of their corners.
            KdTree kda;
            kda.build(aux, nth);
            static const std::vector<int32_t> none;
            parallel_for(nVS, nth, [&](int64_t s, int) {
                if (unresolved[s]) { cell_done[s] = 0; return; }
                bool hit = false;
                for (const d3& x : cell_corners[s])
                    if (!aux.empty() && kda.nearest_below(P[s] + x, norm2(x), none) >= 0) { hit = true; break; }
                cell_done[s] = !hit;
            }, 256);
            P.insert(P.end(), aux.begin(), aux.end());
            is_aux.assign(P.size(), 0);
            for (size_t i = nVS; i < P.size(); ++i) is_aux[i] = 1;
            kd.build(P, nth);
        } else {
            for (int32_t s = 0; s < nVS; ++s) cell_done[s] = !unresolved[s];
        }
    }
    H.stats.t_optimize_s = secs_since(t0) - t_vor1;
    if (!o.augment || nVS < 5) std::fill(cell_done.begin(), cell_done.end(), 0);
    nS = (int32_t)P.size();
    if ((int64_t)nS > std::numeric_limits<int32_t>::max() / 2) throw Error(P2M_ERR_OOM, "too many sites");

    // ---- pass 2: remaining cells, then neighbours and interception lists
    t0 = clk::now();
    cell_corners.resize(nS);
    cell_faces.resize(nS);
    cell_ok.resize(nS, 0);
    cell_done.resize(nS, 0);
    {
        std::vector<int32_t> todo;
        for (int32_t s = 0; s < nS; ++s)
            if (!cell_done[s]) todo.push_back(s);
        compute_cells(todo, P, kd, blo, bhi, -1, nth, checks, gpu_checks != nullptr, gpu_cells, o.gpu_cell_pass, H.stats,
                      [&](int64_t i, int, const std::vector<d3>& corners, const std::vector<int32_t>& faces, bool ok,
                          bool) {
            const int32_t s = todo[i];
            cell_corners[s] = corners;
            cell_faces[s] = faces;
            cell_ok[s] = ok;
        });
    }
    H.stats.t_voronoi_s = t_vor1 + secs_since(t0);
    t0 = clk::now();
    nbr.assign(nS, {});
    lists.assign(nS, {});
    std::vector<char> bad(nS, 0);
    std::vector<std::vector<Ball>> dev_balls(gpu ? nS : 0);
    auto host_list = [&](CellWork& w, const std::vector<Ball>& balls, std::vector<int32_t>& out) {
        w.list.clear();
        if (++w.gen == 0) {
            std::fill(w.stamp.begin(), w.stamp.end(), 0);
            w.gen = 1;
        }
        bvh.query_union(balls, w.list, w.stamp, w.gen);
        out = w.list;
    };
    parallel_for(nS, nth, [&](int64_t s, int tid) {
        CellWork& w = work[tid];
        if (!cell_ok[s]) { bad[s] = 1; return; }
        w.corners.swap(cell_corners[s]);
        std::vector<d3>().swap(cell_corners[s]);
        auto& nb = nbr[s];
        for (int32_t f : cell_faces[s])
            if (f >= 0) nb.push_back(f);
        std::vector<int32_t>().swap(cell_faces[s]);
        const d3 ps = P[s];
        d3 v = ps;  // reference point on the mesh
        if (is_aux[s]) bvh.closest(ps, nullptr, &v);
        w.balls.clear();
        if (is_aux[s] && o.aux_list_mode == 0) {
            // Eq. (8): one sphere about s containing every corner ball
            double r = 0;
            for (const d3& x : w.corners) r = std::max(r, norm(x) + norm(ps + x - v));
            w.balls.push_back({ps, r + delta});
        } else {
            for (const d3& x : w.corners) {
                const d3 u = ps + x;
                w.balls.push_back({u, norm(u - v) + delta});
            }
            // drop balls contained in another ball
            std::sort(w.balls.begin(), w.balls.end(), [](const Ball& a, const Ball& b) { return a.r > b.r; });
            size_t k = 0;
            for (size_t i = 0; i < w.balls.size(); ++i) {
                bool inside = false;
                for (size_t j = 0; j < k && !inside; ++j)
                    inside = norm(w.balls[i].c - w.balls[j].c) + w.balls[i].r <= w.balls[j].r;
                if (!inside) w.balls[k++] = w.balls[i];
            }
            w.balls.resize(k);
        }
        if (gpu && !w.balls.empty() && w.balls.size() <= (size_t)kDeviceBalls) {
            dev_balls[s] = w.balls;  // tested on the device below
            return;
        }
        host_list(w, w.balls, lists[s]);
        if (lists[s].empty()) bad[s] = 2;
    }, 16);
    if (gpu) {
        GpuListJob job;
        job.tri = &T;
        job.bvh = &bvh;
        job.ball_off.push_back(0);
        for (int32_t s = 0; s < nS; ++s) {
            if (dev_balls[s].empty()) continue;
            job.sites.push_back(s);
            job.ball_off.push_back(job.ball_off.back() + (int64_t)dev_balls[s].size());
        }
        job.balls.resize(4 * (size_t)job.ball_off.back());
        parallel_for((int64_t)job.sites.size(), nth, [&](int64_t i, int) {
            double* out = job.balls.data() + 4 * job.ball_off[i];
            for (const Ball& b : dev_balls[job.sites[i]]) {
                out[0] = b.c.x;
                out[1] = b.c.y;
                out[2] = b.c.z;
                out[3] = b.r;
                out += 4;
            }
        }, 1024);
        std::vector<int64_t> off;
        std::vector<int32_t> ids;
        std::vector<char> redo;
        (*gpu)(job, off, ids, redo);
        parallel_for((int64_t)job.sites.size(), nth, [&](int64_t i, int tid) {
            const int32_t s = job.sites[i];
            if (redo[i]) host_list(work[tid], dev_balls[s], lists[s]);
            else lists[s].assign(ids.begin() + off[i], ids.begin() + off[i + 1]);
            std::vector<Ball>().swap(dev_balls[s]);
            if (lists[s].empty()) bad[s] = 2;
        }, 256);
    }
    for (int32_t s = 0; s < nS; ++s)
        if (bad[s]) throw Error(P2M_ERR_INTERNAL, std::string(bad[s] == 1 ? "empty Voronoi cell" : "empty interception list") +
                                                      " at site " + std::to_string(s));
    H.stats.t_lists_s = secs_since(t0);
    }  // Voronoi decomposition
    const int32_t n_vertex_sites = octree ? 0 : nVS;

    // ---- layout
    t0 = clk::now();
    // triangle slots: BVH leaf order
    const std::vector<int32_t>& torder = bvh.order();
    std::vector<int32_t> slot_of(nT);
    for (int64_t i = 0; i < nT; ++i) slot_of[torder[i]] = (int32_t)i;
    // bounding spheres (user order)
    std::vector<float> sph(4 * nT);
    parallel_for(nT, nth, [&](int64_t t, int) {
        const d3 a = T[3 * t], b = T[3 * t + 1], c = T[3 * t + 2];
        const d3 cc = min_sphere_center(a, b, c);
        const float cx = (float)cc.x, cy = (float)cc.y, cz = (float)cc.z;
        const d3 cf{cx, cy, cz};
        const double r = std::max({norm(a - cf), norm(b - cf), norm(c - cf)});
        sph[4 * t] = cx;
        sph[4 * t + 1] = cy;
        sph[4 * t + 2] = cz;
        sph[4 * t + 3] = round_up(r * (1.0 + 1e-6));
    }, 4096);
    // site order: Morton code of position
    std::vector<int32_t> sorder(nS);
    std::iota(sorder.begin(), sorder.end(), 0);
    {
        const double ext = std::max({mhi.x - mlo.x, mhi.y - mlo.y, mhi.z - mlo.z, 1e-30});
        const double inv = 2097151.0 / ext;
        std::vector<uint64_t> key(nS);
        parallel_for(nS, nth, [&](int64_t s, int) { key[s] = morton_of(P[s], mlo, inv); }, 4096);
        std::stable_sort(sorder.begin(), sorder.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    }
    std::vector<int32_t> new_id(nS);
    for (int32_t i = 0; i < nS; ++i) new_id[sorder[i]] = i;

    // triangle records in slot order
    H.tri_rec.resize(12 * (size_t)nT);
    H.tri_user.resize(nT);
    H.tri_vid.resize(4 * (size_t)nT);
    parallel_for(nT, nth, [&](int64_t i, int) {
        const int32_t t = torder[i];
        const d3 a = T[3 * t], b = T[3 * t + 1], c = T[3 * t + 2];
        const float e1x = (float)(b.x - a.x), e1y = (float)(b.y - a.y), e1z = (float)(b.z - a.z);
        const float e2x = (float)(c.x - a.x), e2y = (float)(c.y - a.y), e2z = (float)(c.z - a.z);
        const double g11 = (double)e1x * e1x + (double)e1y * e1y + (double)e1z * e1z;
        const double g12 = (double)e1x * e2x + (double)e1y * e2y + (double)e1z * e2z;
        const double g22 = (double)e2x * e2x + (double)e2y * e2y + (double)e2z * e2z;
        float* r = &H.tri_rec[12 * i];
        r[0] = (float)a.x; r[1] = (float)a.y; r[2] = (float)a.z; r[3] = (float)g11;
        r[4] = e1x; r[5] = e1y; r[6] = e1z; r[7] = (float)g12;
        r[8] = e2x; r[9] = e2y; r[10] = e2z; r[11] = (float)g22;
        H.tri_user[i] = t;
        H.tri_vid[4 * (size_t)t] = mesh.triangles[3 * t];
        H.tri_vid[4 * (size_t)t + 1] = mesh.triangles[3 * t + 1];
        H.tri_vid[4 * (size_t)t + 2] = mesh.triangles[3 * t + 2];
        H.tri_vid[4 * (size_t)t + 3] = 0;
    }, 4096);
    H.n_sites = nS;
    H.n_aux = nS - n_vertex_sites;
    H.site_rec.assign(nS, SiteRec{});
    H.site_is_aux.assign(nS, 0);
    int64_t adj_nnz = 0, list_nnz = 0, adj_max = 0, list_max = 0;
    for (int32_t s = 0; s < nS; ++s) {
        adj_nnz += (int64_t)nbr[s].size();
        list_nnz += (int64_t)lists[s].size();
        adj_max = std::max<int64_t>(adj_max, nbr[s].size());
        list_max = std::max<int64_t>(list_max, lists[s].size());
    }
    if (adj_nnz > std::numeric_limits<int32_t>::max() || list_nnz > std::numeric_limits<int32_t>::max())
        throw Error(P2M_ERR_OOM, "interception lists exceed 2^31 entries");
    H.adj.resize(4 * (size_t)adj_nnz);
    H.list_rec.resize((size_t)list_nnz);
    std::vector<int64_t> adj_off(nS + 1, 0), list_off(nS + 1, 0);
    for (int32_t i = 0; i < nS; ++i) {
        const int32_t s = sorder[i];
        adj_off[i + 1] = adj_off[i] + (int64_t)nbr[s].size();
        list_off[i + 1] = list_off[i] + (int64_t)lists[s].size();
    }
    // per-thread scratch for the neighbours and the list entries of a site
    std::vector<std::vector<int32_t>> nb_scr(nth);
    std::vector<std::vector<std::pair<float, int32_t>>> ent_scr(nth);
    parallel_for(nS, nth, [&](int64_t i, int tid) {
        const int32_t s = sorder[i];
        const float sx = (float)P[s].x, sy = (float)P[s].y, sz = (float)P[s].z;
        SiteRec& sr = H.site_rec[i];
        sr.x = sx;
        sr.y = sy;
        sr.z = sz;
        sr.pad = 0.f;
        sr.adj_begin = (int32_t)adj_off[i];
        sr.adj_end = (int32_t)adj_off[i + 1];
        sr.list_begin = (int32_t)list_off[i];
        sr.list_end = (int32_t)list_off[i + 1];
        H.site_is_aux[i] = is_aux[s];
        std::vector<int32_t>& nb = nb_scr[tid];
        nb.resize(nbr[s].size());
        for (size_t k = 0; k < nb.size(); ++k) nb[k] = new_id[nbr[s][k]];
        std::sort(nb.begin(), nb.end());
        for (size_t k = 0; k < nb.size(); ++k) {
            const int64_t e = adj_off[i] + (int64_t)k;
            const int32_t t = sorder[nb[k]];
            H.adj[4 * e] = (float)P[t].x;
            H.adj[4 * e + 1] = (float)P[t].y;
            H.adj[4 * e + 2] = (float)P[t].z;
            H.adj[4 * e + 3] = ibits(nb[k]);
        }
        // list entries sorted by ell = |s - c| - r (rounded down)
        const d3 sf{sx, sy, sz};
        std::vector<std::pair<float, int32_t>>& ent = ent_scr[tid];
        ent.resize(lists[s].size());
        for (size_t k = 0; k < ent.size(); ++k) {
            const int32_t t = lists[s][k];
            const d3 c{sph[4 * t], sph[4 * t + 1], sph[4 * t + 2]};
            ent[k] = {round_down(norm(sf - c) - (double)sph[4 * t + 3]), slot_of[t]};
        }
        std::sort(ent.begin(), ent.end());
        for (size_t k = 0; k < ent.size(); ++k) {
            const int64_t e = list_off[i] + (int64_t)k;
            const int32_t slot = ent[k].second;
            const int32_t t = torder[slot];
            const float* tr = &H.tri_rec[12 * (size_t)slot];
            ListRec& L = H.list_rec[e];
            L.cx = sph[4 * t];
            L.cy = sph[4 * t + 1];
            L.cz = sph[4 * t + 2];
            L.r = sph[4 * t + 3];
            L.ax = tr[0];
            L.ay = tr[1];
            L.az = tr[2];
            L.ell = ent[k].first;
            L.e1x = tr[4];
            L.e1y = tr[5];
            L.e1z = tr[6];
            L.g12 = tr[7];
            L.e2x = tr[8];
            L.e2y = tr[9];
            L.e2z = tr[10];
            L.tri = t;
        }
    }, 256);
    for (int64_t v = 0; v < nV; ++v)
        if (H.site_of_vertex[v] >= 0) H.site_of_vertex[v] = new_id[H.site_of_vertex[v]];

    // fallback BVH nodes
    const auto& nodes = bvh.nodes();
    H.bvh.resize(8 * nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
        const auto& n = nodes[i];
        float* r = &H.bvh[8 * i];
        r[0] = round_down(n.lo.x); r[1] = round_down(n.lo.y); r[2] = round_down(n.lo.z);
        r[3] = ibits(n.left_or_begin);
        r[4] = round_up(n.hi.x); r[5] = round_up(n.hi.y); r[6] = round_up(n.hi.z);
        r[7] = ibits(n.right_or_count);
    }
    if (octree) {
        // leaf ids in the final site order; no seed grid (the descent starts at the root)
        H.oct = oc.nodes;
        for (int32_t& v : H.oct)
            if (v < 0) v = -(new_id[-v - 1] + 1);
        for (int k = 0; k < 4; ++k) H.oroot[k] = oc.root[k];
        H.gcell = 1.0f;
        for (int k = 0; k < 3; ++k) {
            H.gdim[k] = 1;
            H.gorg[k] = 0.0f;
        }
        H.seed.assign(1, 0);
    }
    // seed grid over the mesh box x1.25: exact nearest site of each cell centre
    if (!octree) {
        d3 glo, ghi;
        padded_box(1.25, glo, ghi);
        double cell = o.seed_cell_scale * mean_edge;
        const d3 ext = ghi - glo;
        auto dims = [&](double c, int64_t* g) {
            g[0] = std::max<int64_t>(1, (int64_t)std::ceil(ext.x / c));
            g[1] = std::max<int64_t>(1, (int64_t)std::ceil(ext.y / c));
            g[2] = std::max<int64_t>(1, (int64_t)std::ceil(ext.z / c));
            return g[0] * g[1] * g[2];
        };
        int64_t g[3];
        int64_t ncell = dims(cell, g);
        while (ncell > o.seed_max_cells || g[0] > 2048 || g[1] > 2048 || g[2] > 2048) {
            cell *= std::max(1.01, std::cbrt((double)ncell / (double)o.seed_max_cells));
            ncell = dims(cell, g);
        }
        H.gcell = (float)cell;
        for (int k = 0; k < 3; ++k) {
            H.gdim[k] = (int32_t)g[k];
            H.gorg[k] = (float)comp(glo, k);
        }
        H.seed.resize(ncell);
        const double gc = (double)H.gcell;
        auto centre = [&](int64_t idx) {
            const int64_t ix = idx % g[0], iy = (idx / g[0]) % g[1], iz = idx / (g[0] * g[1]);
            return d3{H.gorg[0] + (ix + 0.5) * gc, H.gorg[1] + (iy + 0.5) * gc, H.gorg[2] + (iz + 0.5) * gc};
        };
        if (gpu_checks) {
            // the nearest site is the corner check with no limit and nothing
            // excluded (the same search as KdTree::nearest), in slices
            const int64_t slice = int64_t(1) << 22;
            for (int64_t b = 0; b < ncell; b += slice) {
                const int64_t m = std::min(slice, ncell - b);
                CornerChecks job;
                job.kd = &kd;
                job.q.resize(m);
                parallel_for(m, nth, [&](int64_t i, int) { job.q[i] = centre(b + i); }, 4096);
                job.limit2.assign(m, INFINITY);
                job.list.assign(m, 0);
                job.excl_off.assign(2, 0);
                std::vector<int32_t> res;
                (*gpu_checks)(job, res);
                for (int64_t i = 0; i < m; ++i) {
                    if (res[i] < 0) throw Error(P2M_ERR_INTERNAL, "device nearest-site search found no site");
                    H.seed[b + i] = new_id[res[i]];
                }
            }
        } else {
            parallel_for(ncell, nth, [&](int64_t idx, int) { H.seed[idx] = new_id[kd.nearest(centre(idx))]; }, 1024);
        }
    }
    H.stats.t_layout_s = secs_since(t0);

    H.stats.n_vertices = nV;
    H.stats.n_triangles = nT;
    H.stats.n_sites = nS;
    H.stats.n_vertex_sites = n_vertex_sites;
    H.stats.n_aux_sites = nS - n_vertex_sites;
    H.stats.n_dense_cells = n_dense;
    H.stats.adj_nnz = adj_nnz;
    H.stats.adj_max = adj_max;
    H.stats.adj_avg = (double)adj_nnz / nS;
    H.stats.list_nnz = list_nnz;
    H.stats.list_max = list_max;
    H.stats.list_avg = (double)list_nnz / nS;
    for (int k = 0; k < 3; ++k) H.stats.seed_dims[k] = H.gdim[k];
    H.stats.diag = diag;
    H.stats.t_total_s = secs_since(t_start);
}

}  // namespace p2m
