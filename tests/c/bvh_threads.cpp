// Host BVH builder on all threads against one thread, byte for byte, for the
// sanitizer builds of tests/test_sanitizers.py (ThreadSanitizer, then
// AddressSanitizer + UndefinedBehaviorSanitizer).  A seeded soup of small
// triangles large enough for every threaded stage of the build: subtrees on
// their own threads, bounds and bins split over threads, threaded slot fill
// and binary16 extent compression (the sanitizer builds lower the
// thresholds of those stages so that a small soup reaches them); and a
// two-level layout over instances of a smaller mesh.
// Exit status 0 when every pair of builds is identical.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bvh_build.h"

using namespace npt;

namespace {

// xorshift64*: the soup's coordinates, deterministic across runs
struct Rng {
  uint64_t s;
  float next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (float)((s * 2685821657736338717ull) >> 40) * (1.0f / 16777216.0f);
  }
};

struct Soup {
  std::vector<float> verts;
  std::vector<uint32_t> tris, mat;
};

Soup make_soup(uint32_t nt, uint64_t seed) {
  Soup s;
  Rng r{seed};
  s.verts.resize(9 * (size_t)nt);
  s.tris.resize(3 * (size_t)nt);
  s.mat.assign(nt, 0u);
  for (uint32_t t = 0; t < nt; ++t) {
    const float c[3] = {100.0f * r.next(), 20.0f * r.next(), 100.0f * r.next()};
    for (int k = 0; k < 3; ++k) {
      for (int a = 0; a < 3; ++a) s.verts[9 * (size_t)t + 3 * k + a] = c[a] + 0.2f * (r.next() - 0.5f);
      s.tris[3 * (size_t)t + k] = 3 * t + k;
    }
  }
  return s;
}

BuildInput input_of(const Soup& s) {
  BuildInput in;
  in.verts = s.verts.data();
  in.nv = s.verts.size() / 3;
  in.tris = s.tris.data();
  in.nt = s.tris.size() / 3;
  in.tri_mat = s.mat.data();
  return in;
}

template <class T>
bool same_bytes(const std::vector<T>& a, const std::vector<T>& b) {
  return a.size() == b.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0;
}

bool same_tree(const FlatBvh& a, const FlatBvh& b) {
  return same_bytes(a.nodes, b.nodes) && same_bytes(a.slots, b.slots) && a.max_depth == b.max_depth &&
         a.leaves == b.leaves && a.node_float4s == b.node_float4s;
}

bool build(const BuildInput& in, int threads, uint32_t width, int format, FlatBvh& out) {
  const BuildThreads cap(threads);
  std::string err;
  if (!build_bvh(in, 32, 2, 0, width, out, err)) {
    std::fprintf(stderr, "build failed: %s\n", err.c_str());
    return false;
  }
  if (format == 1 && !compress_half_extents(out, err)) {
    std::fprintf(stderr, "binary16 extents failed: %s\n", err.c_str());
    return false;
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  const uint32_t nt = argc > 1 ? (uint32_t)std::strtoul(argv[1], nullptr, 10) : 1200000u;
  const Soup soup = make_soup(nt, 0x9E3779B97F4A7C15ull);
  const BuildInput in = input_of(soup);
  int failures = 0;
  const struct {
    uint32_t width;
    int format;
  } cases[] = {{4, 0}, {4, 1}, {2, 0}};
  for (const auto& cs : cases) {
    FlatBvh one, all, three;
    if (!build(in, 1, cs.width, cs.format, one) || !build(in, 0, cs.width, cs.format, all) ||
        !build(in, 3, cs.width, cs.format, three))
      return 2;
    const bool ok = same_tree(one, all) && same_tree(one, three);
    std::printf("%u triangles, width %u, format %d: %zu node bytes, threads 1 / all / 3 %s\n", nt, cs.width,
                cs.format, one.nodes.size() * sizeof(float4), ok ? "identical" : "DIFFER");
    failures += ok ? 0 : 1;
  }
  // two-level: 40 instances of a mesh of an eighth of the soup's triangles
  const Soup mesh = make_soup(nt / 8 > 1000 ? nt / 8 : 1000, 12345);
  std::vector<Placement> objects;
  for (uint32_t i = 0; i < 40; ++i) objects.push_back(Placement{0, {120.0f * (i % 8), 0.0f, 120.0f * (i / 8)}, 1.0f + 0.01f * i, i});
  FlatBvh levels[2];
  std::vector<float4> records[2];
  for (int k = 0; k < 2; ++k) {
    const BuildThreads cap(k == 0 ? 1 : 0);
    std::vector<FlatBvh> bottoms(1);
    std::string err;
    uint32_t stack = 0;
    if (!build_bvh(input_of(mesh), 32, 2, 0, 4, bottoms[0], err) ||
        !build_two_level(bottoms, objects, 32, 2, levels[k], records[k], stack, err)) {
      std::fprintf(stderr, "two-level build failed: %s\n", err.c_str());
      return 2;
    }
  }
  const bool ok2 = same_tree(levels[0], levels[1]) && same_bytes(records[0], records[1]);
  std::printf("two-level, 40 instances: threads 1 / all %s\n", ok2 ? "identical" : "DIFFER");
  failures += ok2 ? 0 : 1;
  return failures == 0 ? 0 : 1;
}
