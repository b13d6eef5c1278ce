// Host preprocessing of P2M++: from a triangle mesh to the flat arrays the
// query kernels read (sites, Delaunay adjacency, interception lists,
// triangle records, seed grid, fallback BVH).
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"
#include "p2m.h"

namespace p2m {

struct HostStructure {
    int64_t n_vertices = 0, n_triangles = 0;
    double diag = 0;  // mesh AABB diagonal

    // Sites in device order.  site_xyz: x, y, z, 0.  site_rng: adjacency
    // begin/end and list begin/end.
    int32_t n_sites = 0, n_aux = 0;
    std::vector<float> site_xyz;
    std::vector<int32_t> site_rng;
    std::vector<uint8_t> site_is_aux;
    // Adjacency entries: neighbour x, y, z and its site id (int bits).
    std::vector<float> adj;
    // List entries: bounding sphere (cx, cy, cz, r) and (triangle slot, ell bits).
    std::vector<float> list_sph;
    std::vector<int32_t> list_aux;
    // Triangles in slot order (BVH leaf order): v0, |e1|^2 | e1, e1.e2 | e2, |e2|^2.
    std::vector<float> tri_rec;
    std::vector<int32_t> tri_user;  // slot -> caller's triangle id
    std::vector<int32_t> tri_vid;   // slot -> caller's vertex ids a, b, c, 0
    // Seed grid: exact nearest site of every cell centre.
    std::vector<int32_t> seed;
    int32_t gdim[3] = {0, 0, 0};
    float gorg[3] = {0, 0, 0};
    float gcell = 1;
    // Domain box: queries inside use the site lists, outside the BVH.
    float dlo[3] = {0, 0, 0}, dhi[3] = {0, 0, 0};
    // Fallback BVH nodes: lo xyz, a | hi xyz, b (see Bvh::Node; leaf ranges in slots).
    std::vector<float> bvh;
    // Host-side views for inspection.
    std::vector<int32_t> site_of_vertex;  // caller vertex -> site id or -1

    p2m_stats stats{};
};

// Throws p2m::Error on invalid input.
void build_host(const p2m_mesh_desc& mesh, const p2m_build_opts& opts, HostStructure& out);

}  // namespace p2m
