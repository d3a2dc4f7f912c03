// subdomain.hpp -- geometric sub-domains of a scene (Sec. 5): the host build
// of the cell grid and its per-cell BVHs (subdomain.cpp).
#pragma once
#include <stdint.h>

#include <vector>

#include "sdm_types.hpp"

namespace sdm {

constexpr int kMaxCellsPerAxis = 64;

struct SubdomainBuild {
    std::vector<CellDev> cells;
    std::vector<BvhNode> nodes;
    std::vector<TriDev> tris;       // copies in each cell's leaf order
    std::vector<int32_t> leaf;      // copy -> the scene's leaf-order triangle
    float lo[3] = {0, 0, 0}, size[3] = {0, 0, 0};
    int stack = 0;                  // most traversal stack entries a cell's walk can hold
    bool ok = true;                 // false: a cell's BVH has a leaf at the depth cap too large
};

// Grid of n[0] x n[1] x n[2] cells over [lo, hi] (widened by a margin); each
// cell lists the triangles whose bounding boxes overlap it (also widened), so
// that a hit within the margin of a cell face is found from both sides.
// leaf_tris / o2l: the scene's triangles in leaf order and the caller index
// -> leaf map.
SubdomainBuild build_subdomains(const float *pos, int32_t nv, const int32_t *idx, int32_t nt,
                                const std::vector<TriDev> &leaf_tris, const std::vector<int32_t> &o2l,
                                const int32_t n[3], const double lo[3], const double hi[3]);

}  // namespace sdm
