// bvh_build.hpp -- host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

#include "sdm_types.hpp"

namespace sdm {

struct BvhResult {
    std::vector<BvhNode> nodes;   // wide nodes, breadth-first; empty for an empty scene
    std::vector<int32_t> order;   // leaf slot -> caller's triangle index
    int depth = 0;                // levels of wide nodes plus leaves
    int stack = 0;                // most traversal stack entries any walk can hold
    bool ok = true;               // false: a leaf at the depth cap is too large
};

// Per-thread levels of the global part of the traversal stack for a scene
// whose walks hold at most `stack` entries.
inline int global_stack_levels(int stack) { return stack > kLdsStack ? stack - kLdsStack + 1 : 1; }

BvhResult build_bvh(const float *pos, int32_t nv, const int32_t *idx, int32_t nt);

}  // namespace sdm
