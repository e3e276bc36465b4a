// Level meshes of the octree multigrid (host side, built in octree.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "amrto.h"

namespace amrto {

struct LevelMesh {
  int n_nodes = 0, n_elems = 0;
  int L = 0;                        // a leaf of level l has edge 2^(L - l)
  std::vector<int32_t> xyz;         // 3 per node
  std::vector<int32_t> elem_nodes;  // 8 per element, local vertex i + 2 j + 4 k
  std::vector<int8_t> level;
  std::vector<int32_t> anchor;      // 3 per element
  std::vector<int32_t> hang_node, hang_ptr, hang_master;
  std::vector<double> hang_w;
  std::vector<uint8_t> fixed;       // 3 per node
};

// k == 0: the tree's current mesh (its last build_mesh).  k >= 1: the mesh of
// the level-k coarsening of the current leaves: for k <= max_level every leaf
// finer than level max_level - k is replaced by its ancestor at that level;
// for k > max_level the uniform base grid is coarsened by two per axis
// k - max_level times; nodes of levels k >= 1 are numbered with x fastest.
// Supports are the regions of the last build_mesh.
// Returns false when level k cannot be built (no mesh yet, or a base extent
// not divisible by 2^(k - max_level)).
bool octree_level_mesh(const amrto_octree* t, int k, LevelMesh* out);

}  // namespace amrto
