// A convex polytope stored as its face polygons, with coordinates relative
// to a centre point (the Voronoi site), clipped by half-spaces n.x <= h.
//
// Used to compute the Voronoi cell of a site inside the domain box: start
// from the box and clip by the bisector half-space of each site that can
// cut it.  Faces are kept as independent polygons (no shared topology), so
// degenerate configurations (many co-spherical sites, planes through a
// common corner) cost only duplicated vertices, never an inconsistent
// structure.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

namespace p2m {

class ClipCell {
public:
    // Box [lo, hi] given relative to the centre; plane ids -1..-6.
    void init_box(d3 lo, d3 hi);
    // Clip by n.x <= h (x relative to the centre).  Returns true if the cell
    // changed.  `id` tags the new face.
    bool clip(d3 n, double h, int32_t id);
    // Distinct corners (deduplicated), relative to the centre.
    void corners(std::vector<d3>& out) const;
    // Largest squared corner norm.
    double max_norm2() const;
    // Ids of the planes that bound a face of positive extent.
    void face_ids(std::vector<int32_t>& out) const;
    int32_t n_faces() const { return (int32_t)faces_.size(); }
    bool empty() const { return faces_.size() < 4; }

private:
    struct Face {
        int32_t id;
        int32_t begin, count;  // vertex range in v_
        d3 c;                  // bounding sphere of the face's vertices
        double r;
    };
    void seal(Face& f) const;  // sets the bounding sphere
    void compact();
    std::vector<Face> faces_;
    std::vector<d3> v_, tmp_;  // v_ also holds dead ranges until compact()
    std::vector<double> sd_;
    std::vector<d3> cut_;
    size_t live_ = 0;          // vertices referenced by faces_
    double scale_ = 1.0;  // typical coordinate magnitude, for tolerances
};

}  // namespace p2m
