#pragma once

#include <stdint.h>

#include <vector>

#include "srp_internal.h"

namespace srp {

struct BvhBuildResult {
    std::vector<BvhNode> nodes;   // node 0 is the root (always an inner node)
    std::vector<int32_t> perm;    // BVH triangle position -> original triangle index
    int depth = 0;                // deepest node level (root = 0)
};

// Builds the BVH of n_tris triangles (vertex indices into verts [][3]).  Child boxes are rounded
// outward to float and widened by `pad` metres so that float slab tests stay conservative.
BvhBuildResult build_bvh(const double* verts, const int32_t* tris, int64_t n_tris, double pad);

// Refits the child boxes of an existing tree to moved vertices (same topology and triangle order):
// nodes are in pre-order (every child after its parent), so one reverse sweep sees children first.
// perm maps BVH triangle positions to original triangles.  Boxes are rounded outward and padded as
// in build_bvh.
void refit_bvh(std::vector<BvhNode>& nodes, const std::vector<int32_t>& perm, const double* verts,
               const int32_t* tris, double pad);

}  // namespace srp
