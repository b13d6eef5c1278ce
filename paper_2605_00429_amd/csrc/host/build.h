// Host preprocessing of P2M++: from a triangle mesh to the flat arrays the
// query kernels read (sites, Delaunay adjacency, interception lists,
// triangle records, seed grid, fallback BVH).
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

#include "common.h"
#include "p2m.h"

namespace p2m {

// One site: position and the ranges of its adjacency and list entries.
struct SiteRec {
    float x, y, z, pad;
    int32_t adj_begin, adj_end, list_begin, list_end;
};

// One interception-list entry (64 B): the triangle's bounding sphere, its
// record for the exact test (a, e1, e2 and e1.e2; |e1|^2 and |e2|^2 are
// recomputed), ell = |s - c| - r rounded down, and the caller's triangle id.
struct ListRec {
    float cx, cy, cz, r;
    float ax, ay, az, ell;
    float e1x, e1y, e1z, g12;
    float e2x, e2y, e2z;
    int32_t tri;
};

struct HostStructure {
    int64_t n_vertices = 0, n_triangles = 0;
    double diag = 0;  // mesh AABB diagonal

    // Sites in device order.
    int32_t n_sites = 0, n_aux = 0;
    std::vector<SiteRec> site_rec;
    std::vector<uint8_t> site_is_aux;
    // Adjacency entries: neighbour x, y, z and its site id (int bits).
    std::vector<float> adj;
    // Interception-list entries, each site's list sorted by ell (released
    // after upload; list_tri keeps their caller triangle ids).
    std::vector<ListRec> list_rec;
    std::vector<int32_t> list_tri;
    // Triangles in slot order (BVH leaf order): v0, |e1|^2 | e1, e1.e2 | e2, |e2|^2.
    std::vector<float> tri_rec;
    std::vector<int32_t> tri_user;  // slot -> caller's triangle id
    std::vector<int32_t> tri_vid;   // caller triangle id -> caller's vertex ids a, b, c, 0
    // Seed grid: exact nearest site of every cell centre.
    std::vector<int32_t> seed;
    int32_t gdim[3] = {0, 0, 0};
    float gorg[3] = {0, 0, 0};
    float gcell = 1;
    // Domain box: queries inside use the site lists, outside the BVH.
    float dlo[3] = {0, 0, 0}, dhi[3] = {0, 0, 0};
    // Fallback BVH nodes: lo xyz, a | hi xyz, b (see Bvh::Node; leaf ranges in slots).
    std::vector<float> bvh;
    // Octree decomposition only (empty otherwise): nodes breadth first, a
    // node holding the first of its 8 children or -(site + 1) for a leaf;
    // root centre xyz and half size.
    std::vector<int32_t> oct;
    float oroot[4] = {0, 0, 0, 0};
    // Host-side views for inspection.
    std::vector<int32_t> site_of_vertex;  // caller vertex -> site id or -1

    p2m_stats stats{};
};

class Bvh;

// The sphere-union tests of the list stage, handed to a device: for each
// site in `sites`, its balls (4 doubles each: centre, radius) in
// balls[4 * ball_off[i] .. 4 * ball_off[i + 1]), at most kDeviceBalls per site.
constexpr int kDeviceBalls = 256;
struct GpuListJob {
    const std::vector<d3>* tri = nullptr;  // 3 vertices per triangle (FP64)
    const Bvh* bvh = nullptr;
    std::vector<int32_t> sites;
    std::vector<int64_t> ball_off;
    std::vector<double> balls;
};
// Fills CSR lists (off, ids) for job.sites; redo[i] asks the host to build
// site i's list itself.  Throws p2m::Error.
using GpuListFn = std::function<void(const GpuListJob&, std::vector<int64_t>& off, std::vector<int32_t>& ids,
                                     std::vector<char>& redo)>;

class KdTree;

// A batch of corner checks of the Voronoi stage against the sites of one
// kd-tree: for check i, KdTree::below(q[i], limit2[i], exclusion list
// list[i], budget), where exclusion list j is the sorted run
// excl[excl_off[j] .. excl_off[j + 1]).
struct CornerChecks {
    const KdTree* kd = nullptr;
    std::vector<d3> q;
    std::vector<double> limit2;
    std::vector<int32_t> list;
    std::vector<int64_t> excl_off;
    std::vector<int32_t> excl;
    int64_t budget = -1;
};
// Fills out[i] with check i's result (site index, -1 or -2).  Throws
// p2m::Error.
using CheckFn = std::function<void(const CornerChecks&, std::vector<int32_t>& out)>;

// A chunk of Voronoi cells for a device (Sec. 3.2): the cell of point
// sites[i] of the tree, clipped to the box [blo, bhi], built the way the
// host builds it: the box clipped by the bisectors of the knn nearest
// sites (stopping at twice the farthest corner), then rounds of corner
// checks (KdTree::below with limit |x|^2 (1 - slack)) and clips until no
// corner beyond half the knn radius is cut.  With budget >= 0 each check
// examines at most that many sites and a cell with more than max_faces
// faces stops, unresolved.
struct CellJob {
    const KdTree* kd = nullptr;
    const int32_t* sites = nullptr;
    int64_t n = 0;
    d3 blo{0, 0, 0}, bhi{0, 0, 0};
    int64_t budget = -1;
    int32_t max_faces = 0;
    int32_t knn = 0;
    double slack = 0;
    int64_t pass = 0;  // cells per device pass; 0 = as device memory allows
};
// Per cell i: its distinct corners relative to the site (sorted as
// ClipCell::corners gives them) in corners[corner_off[i] .. corner_off[i+1]),
// the sites of its faces of positive area (sorted) in
// faces[face_off[i] .. face_off[i+1]), whether it is a polytope (ok) and
// whether a check or the face cap gave up (unresolved).  redo[i] asks the
// host to build cell i itself (it outgrew the device's per-cell capacity);
// its other entries are then empty.
struct CellResult {
    std::vector<int64_t> corner_off, face_off;
    std::vector<d3> corners;
    std::vector<int32_t> faces;
    std::vector<char> ok, unresolved, redo;
};
using CellFn = std::function<void(const CellJob&, CellResult&)>;

// Throws p2m::Error on invalid input.  With `gpu`, the list stage's
// sphere-union tests run through it (sites with more than kDeviceBalls balls stay on
// the host); with `gpu_checks`, the Voronoi stage's corner checks and the
// seed grid's nearest sites do; with `gpu_cells` as well, whole cells are
// built through it.  The structure is the same either way.
void build_host(const p2m_mesh_desc& mesh, const p2m_build_opts& opts, HostStructure& out,
                const GpuListFn* gpu = nullptr, const CheckFn* gpu_checks = nullptr,
                const CellFn* gpu_cells = nullptr);

// The device implementation of CheckFn (current HIP device).
void gpu_corner_checks(const CornerChecks& job, std::vector<int32_t>& out);

// The device implementation of CellFn (current HIP device).
void gpu_cells(const CellJob& job, CellResult& out);

// The device implementation of GpuListFn (current HIP device).
void gpu_build_lists(const GpuListJob& job, std::vector<int64_t>& off, std::vector<int32_t>& ids,
                     std::vector<char>& redo);

}  // namespace p2m
