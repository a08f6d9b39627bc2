// Host check of the BVH builder, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py. Inputs: random
// triangle soups, triangles with spheres, and degenerate sets (coincident
// triangles, zero-area triangles on a line, a long thin strip, one to three
// primitives). Invariants checked on each tree: every primitive sits in
// exactly one leaf, each primitive's box lies inside the box its parent
// stores for the subtree, links are in range, the depth stays below the
// traversal stack, and the first nodes (the top levels, breadth-first) only
// link forward.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2606_14173_amd/csrc/bvh_build.hpp"

using namespace hpt;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { std::printf("FAIL: " __VA_ARGS__); std::printf("\n"); ++fails; return; } } while (0)

static void prim_box(const std::vector<float> &tri, const std::vector<float> &sph, uint32_t n_sph, uint32_t g,
                     float lo[3], float hi[3]) {
  if (g < n_sph) {
    for (int a = 0; a < 3; ++a) { lo[a] = sph[4 * g + a] - sph[4 * g + 3]; hi[a] = sph[4 * g + a] + sph[4 * g + 3]; }
    return;
  }
  const float *t = &tri[9 * (size_t)(g - n_sph)];
  for (int a = 0; a < 3; ++a) {
    lo[a] = std::fmin(t[a], std::fmin(t[3 + a], t[6 + a]));
    hi[a] = std::fmax(t[a], std::fmax(t[3 + a], t[6 + a]));
  }
}

// Walk the subtree at `link` inside the box (lo, hi) its parent stores.
static void walk(const BvhResult &B, const std::vector<float> &tri, const std::vector<float> &sph, uint32_t n_sph,
                 int32_t link, const float lo[3], const float hi[3], uint32_t depth, std::vector<int> &seen,
                 uint32_t n) {
  CHECK(depth < kBvhDepthMax, "depth %u", depth);
  if (link < 0) {
    uint32_t v = (uint32_t)(~link), first = v >> 3, cnt = (v & 7u) + 1u;
    CHECK(first + cnt <= n, "leaf range %u+%u of %u", first, cnt, n);
    for (uint32_t k = 0; k < cnt; ++k) {
      uint32_t gid;
      std::memcpy(&gid, &B.prims[12 * (size_t)(first + k) + 3], 4);
      CHECK(gid < n, "gid %u", gid);
      seen[gid]++;
      float pl[3], ph[3];
      prim_box(tri, sph, n_sph, gid, pl, ph);
      for (int a = 0; a < 3; ++a) CHECK(pl[a] >= lo[a] && ph[a] <= hi[a], "primitive %u outside its box", gid);
    }
    return;
  }
  CHECK((uint32_t)link < B.n_nodes, "node %d of %u", link, B.n_nodes);
  const float *nd = &B.nodes[16 * (size_t)link];
  int32_t c[2];
  std::memcpy(&c[0], &nd[12], 4);
  std::memcpy(&c[1], &nd[13], 4);
  const float l0[3] = {nd[0], nd[2], nd[8]}, h0[3] = {nd[1], nd[3], nd[9]};
  const float l1[3] = {nd[4], nd[6], nd[10]}, h1[3] = {nd[5], nd[7], nd[11]};
  walk(B, tri, sph, n_sph, c[0], l0, h0, depth + 1, seen, n);
  if (!(n <= 2 && c[1] == c[0])) walk(B, tri, sph, n_sph, c[1], l1, h1, depth + 1, seen, n);
}

static void check(const char *name, const std::vector<float> &tri, const std::vector<float> &sph) {
  uint32_t n_tri = (uint32_t)(tri.size() / 9), n_sph = (uint32_t)(sph.size() / 4), n = n_tri + n_sph;
  BvhResult B;
  bool ok = build_bvh(tri.data(), n_tri, sph.data(), n_sph, B);
  CHECK(ok, "%s: build failed", name);
  std::vector<int> seen(n, 0);
  const float inf[3] = {INFINITY, INFINITY, INFINITY}, ninf[3] = {-INFINITY, -INFINITY, -INFINITY};
  walk(B, tri, sph, n_sph, 0, ninf, inf, 0, seen, n);
  for (uint32_t g = 0; g < n; ++g) CHECK(seen[g] == 1, "%s: primitive %u seen %d times", name, g, seen[g]);
  // the first nodes are the top of the tree in breadth-first order: the
  // children of node i that are inner nodes and among the first ones come
  // after i
  uint32_t top = B.n_nodes < kBvhTopNodes ? B.n_nodes : kBvhTopNodes;
  for (uint32_t i = 0; i < top; ++i)
    for (int k = 0; k < 2; ++k) {
      int32_t c;
      std::memcpy(&c, &B.nodes[16 * (size_t)i + 12 + k], 4);
      CHECK(c < 0 || (uint32_t)c > i, "%s: node %u links back to %d", name, i, c);
    }
  std::printf("ok %-22s prims %7u nodes %7u depth %u\n", name, n, B.n_nodes, B.max_depth);
}

int main() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<float> U(-1.f, 1.f);
  for (uint32_t n : {1u, 2u, 3u, 17u, 1000u, 60000u}) {
    std::vector<float> tri(9 * (size_t)n), sph;
    for (auto &x : tri) x = U(rng);
    check(("soup " + std::to_string(n)).c_str(), tri, sph);
  }
  {  // spheres and triangles together
    std::vector<float> tri(9 * 500), sph;
    for (auto &x : tri) x = U(rng);
    for (int i = 0; i < 300; ++i) { sph.push_back(U(rng)); sph.push_back(U(rng)); sph.push_back(U(rng)); sph.push_back(0.01f + 0.05f * std::fabs(U(rng))); }
    check("mixed", tri, sph);
  }
  {  // coincident triangles (no split separates them)
    std::vector<float> tri;
    for (int i = 0; i < 5000; ++i) for (float v : {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f, 0.f}) tri.push_back(v);
    check("coincident", tri, {});
  }
  {  // zero-area triangles on a line
    std::vector<float> tri;
    for (int i = 0; i < 3000; ++i) for (float v : {(float)i, 0.f, 0.f, (float)i + 1, 0.f, 0.f, (float)i + 2, 0.f, 0.f}) tri.push_back(v);
    check("degenerate line", tri, {});
  }
  {  // a long thin strip (deep median splits)
    std::vector<float> tri;
    for (int i = 0; i < 200000; ++i) {
      float x = (float)i * 1e-3f;
      for (float v : {x, 0.f, 0.f, x + 1e-3f, 0.f, 0.f, x, 1e-3f, 0.f}) tri.push_back(v);
    }
    check("strip", tri, {});
  }
  std::printf("%s\n", fails ? "FAILED" : "ALL OK");
  return fails ? 1 : 0;
}
