// bvh_build.hpp -- host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

#include "sdm_types.hpp"

namespace sdm {

struct BvhResult {
    std::vector<BvhNode> nodes;   // breadth-first; empty for an empty scene
    std::vector<int32_t> order;   // leaf slot -> caller's triangle index
    int depth = 0;                // levels of inner nodes plus leaves
    bool ok = true;               // false: a leaf at the depth cap is too large
};

BvhResult build_bvh(const float *pos, int32_t nv, const int32_t *idx, int32_t nt);

}  // namespace sdm
