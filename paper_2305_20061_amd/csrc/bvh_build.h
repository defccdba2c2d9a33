// bvh_build.h -- host BVH2 construction (Sec. 3.1.4: a BVH2 built on the
// host and compacted into pointer-less nodes) for the GPU traversal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace npt {

struct BuildInput {
  const float* verts = nullptr;   // [nv][3]
  uint64_t nv = 0;
  const uint32_t* tris = nullptr; // [nt][3]
  uint64_t nt = 0;
  const uint32_t* tri_mat = nullptr;
  const float* spheres = nullptr; // [ns][4]
  uint64_t ns = 0;
  const uint32_t* sph_mat = nullptr;
  // box mode (a top-level tree over instances): when nboxes > 0 the tree is
  // built over these boxes [nboxes][lo xyz, hi xyz] instead, and slot i
  // holds the input box index in the .w of its first float4
  const float* boxes = nullptr;
  uint64_t nboxes = 0;
};

struct FlatBvh {
  std::vector<float4> nodes;  // 4 float4 per node (npt_shared.h layout)
  std::vector<float4> slots;  // 3 float4 per primitive slot
  uint32_t width = 2;         // children per node (2 or 4)
  uint32_t node_float4s = 4;  // float4s per node (4 for width 2, 7 for width 4)
  uint32_t lds_nodes = 0;     // BFS-ordered top nodes staged in LDS
  uint32_t max_depth = 0;     // deepest inner node (root = 0)
  uint64_t leaves = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // bounds of all primitives
};

// Caps the host threads of the builds this thread runs while it lives (n = 0:
// every hardware thread, at most 64).  The tree does not depend on it: a
// build on any number of threads gives the single-threaded tree byte for
// byte.
class BuildThreads {
 public:
  explicit BuildThreads(int n);
  ~BuildThreads();
  BuildThreads(const BuildThreads&) = delete;
  BuildThreads& operator=(const BuildThreads&) = delete;

 private:
  int prev_;
};

// Binned-SAH build of a binary tree (bins per axis, primitives per leaf <=
// max_leaf), collapsed to `width` children per node (2 or 4), then
// flattening: the nodes of the top lds_levels levels first in BFS order, the
// rest depth-first.  Returns false with a message on failure.
bool build_bvh(const BuildInput& in, uint32_t bins, uint32_t max_leaf, uint32_t lds_levels, uint32_t width,
               FlatBvh& out,
               std::string& err);

// Rewrites the 7-row FP32 nodes of a 4-wide tree (one- or two-level) as
// 6-row nodes with binary16 extents (npt_shared.h layout); node indices and
// slots are unchanged.  Each extent is the smallest binary16 value whose
// FP32 sum with the lower plane is >= the upper plane.  Fails for extents
// beyond 65504.
bool compress_half_extents(FlatBvh& b, std::string& err);

// Rewrites the 7-row FP32 nodes of a 4-wide tree as 4-row nodes with 8-bit
// child planes on a per-node, per-axis power-of-two step (npt_shared.h
// layout), each decoded plane rounded outward and checked in FP32.
bool compress_q8_nodes(FlatBvh& b, std::string& err);

// Rewrites the 7-row FP32 nodes of a 4-wide tree (one- or two-level) as
// 5-row nodes with binary16 planes on an FP32 corner (npt_shared.h layout):
// each lower plane the largest and each upper plane the smallest binary16
// offset whose FP32 sum with the corner still contains the child's box.
// Fails where a node spans more than 65504 on an axis.
bool compress_corner_nodes(FlatBvh& b, std::string& err);

// One object of a two-level scene: bottom tree `tree` placed in the world at
// translate + scale * x (scale > 0), hits reported with instance id `id`.
struct Placement {
  uint32_t tree;
  float translate[3];
  float scale;
  uint32_t id;
};

// Two-level layout for instancing: a 4-wide top tree (one object per leaf)
// over the world boxes of `objects`, followed in one node array and one slot
// array by the 4-wide bottom trees with their refs moved by their offsets.
// The top tree's first lds_levels levels come first in BFS order
// (out.lds_nodes of them), for the traversal to stage in LDS.
// records receives two float4 per top-tree leaf (translate, scale) and
// (bottom root, id); stack_entries the traversal stack the layout needs.
bool build_two_level(const std::vector<FlatBvh>& bottoms, const std::vector<Placement>& objects, uint32_t bins,
                     uint32_t lds_levels, FlatBvh& out, std::vector<float4>& records, uint32_t& stack_entries,
                     std::string& err);

}  // namespace npt
