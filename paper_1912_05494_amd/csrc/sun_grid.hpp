// sun_grid.hpp -- host builder of the sun-aligned candidate grid.
//
// Every shadow ray of a scene runs along the one sun direction (eq. (3): the
// direct term toward a directional sun), so its candidates can be found by
// projecting the triangles onto the plane perpendicular to that direction:
// the ray is a point there, and only triangles whose projection (padded)
// covers that point can be crossed.  The grid bins the padded projections;
// each cell lists its triangles by increasing smallest depth along the sun.
#pragma once
#include <stdint.h>

#include <vector>

#include "sdm_types.hpp"

namespace sdm {

struct SunGrid {
    bool use = false;            // false: the scene keeps the BVH walk for shadow rays
    float e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
    float u0 = 0, v0 = 0, idu = 0, idv = 0, marg = 0;
    int32_t nx = 0, ny = 0;
    std::vector<int32_t> start;  // [nx * ny + 1]
    std::vector<GridCand> cand;
};

// tris: the scene's triangles in leaf order (material index in b.w);
// mat_type: material index -> type; sun: the scene's sun direction; extent:
// scene diagonal plus the largest coordinate magnitude (sets the padding).
SunGrid build_sun_grid(const TriDev *tris, int32_t nt, const int32_t *mat_type, const float sun[3],
                       double extent);

}  // namespace sdm
