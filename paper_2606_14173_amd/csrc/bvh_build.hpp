// Host BVH builder interface.
#pragma once
#include <cstdint>
#include <vector>

namespace hpt {

constexpr uint32_t kBvhDepthMax = 64;   // traversal stack entries
constexpr uint32_t kBvhTopNodes = 256;  // nodes stored first, in breadth-first order from the root

struct BvhResult {
  std::vector<float> nodes;   // 16 floats per node
  std::vector<float> prims;   // 12 floats per primitive, leaf order
  uint32_t n_nodes = 0, max_depth = 0;
  float bounds[6] = {0, 0, 0, 0, 0, 0};
  double build_ms = 0.0;
};

// Build over spheres [0, n_sph) then triangles [n_sph, n_sph + n_tri)
// (global ids). Returns false if the input is empty, too large, or the
// tree is deeper than the traversal stack.
bool build_bvh(const float *tri, uint32_t n_tri, const float *sph, uint32_t n_sph, BvhResult &out);

}  // namespace hpt
