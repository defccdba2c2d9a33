// bvh_build.cpp -- binned-SAH BVH2 builder and flattening to the two-box
// node layout the traversal kernel reads.
#include "bvh_build.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>

#include "npt_shared.h"

namespace npt {
namespace {

struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float p[3]) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double half_area() const {
    if (!(lo[0] <= hi[0])) return 0.0;
    const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    return dx * dy + dy * dz + dz * dx;
  }
};

struct Node {
  Box box;
  int32_t child[2] = {-1, -1};
  uint32_t first = 0, count = 0;  // leaf range in the order array
  uint32_t depth = 0;
  bool leaf() const { return child[0] < 0; }
};

struct Builder {
  std::vector<Box> pbox;
  std::vector<float> cen;  // [n][3]
  std::vector<uint32_t> order;
  std::vector<Node> nodes;
  uint32_t bins = 32, max_leaf = 4;

  int build(uint32_t first, uint32_t count, uint32_t depth) {
    const int id = (int)nodes.size();
    nodes.emplace_back();
    Box b, cb;
    for (uint32_t i = first; i < first + count; ++i) {
      b.grow(pbox[order[i]]);
      cb.grow(&cen[3 * (size_t)order[i]]);
    }
    nodes[id].box = b;
    nodes[id].depth = depth;
    if (count <= max_leaf) {
      nodes[id].first = first;
      nodes[id].count = count;
      return id;
    }
    uint32_t mid = first;
    int axis = -1, split = -1;
    double best = INFINITY;
    if (depth < 56) {
      // SAH over `bins` bins per axis of the centroid bounds
      std::vector<Box> bbox(bins);
      std::vector<uint32_t> bcnt(bins);
      std::vector<double> right_area(bins);
      std::vector<uint32_t> right_cnt(bins);
      for (int a = 0; a < 3; ++a) {
        const float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0f)) continue;
        std::fill(bbox.begin(), bbox.end(), Box());
        std::fill(bcnt.begin(), bcnt.end(), 0u);
        const float scale = (float)bins / ext;
        for (uint32_t i = first; i < first + count; ++i) {
          const uint32_t p = order[i];
          int k = (int)((cen[3 * (size_t)p + a] - cb.lo[a]) * scale);
          k = std::min(std::max(k, 0), (int)bins - 1);
          bbox[k].grow(pbox[p]);
          ++bcnt[k];
        }
        Box acc;
        uint32_t c = 0;
        for (int k = (int)bins - 1; k > 0; --k) {
          acc.grow(bbox[k]);
          c += bcnt[k];
          right_area[k] = acc.half_area();
          right_cnt[k] = c;
        }
        Box left;
        uint32_t lc = 0;
        for (int k = 0; k < (int)bins - 1; ++k) {
          left.grow(bbox[k]);
          lc += bcnt[k];
          if (lc == 0 || right_cnt[k + 1] == 0) continue;
          const double cost = left.half_area() * lc + right_area[k + 1] * right_cnt[k + 1];
          if (cost < best) {
            best = cost;
            axis = a;
            split = k;
          }
        }
      }
    }
    if (axis >= 0) {
      const float ext = cb.hi[axis] - cb.lo[axis];
      const float scale = (float)bins / ext;
      const float lo = cb.lo[axis];
      const int a = axis, sp = split;
      const uint32_t* it = std::partition(order.data() + first, order.data() + first + count, [&](uint32_t p) {
        int k = (int)((cen[3 * (size_t)p + a] - lo) * scale);
        k = std::min(std::max(k, 0), (int)bins - 1);
        return k <= sp;
      });
      mid = (uint32_t)(it - order.data());
    }
    if (mid <= first || mid >= first + count) {
      // degenerate centroids or depth limit: object median on the widest axis
      int a = 0;
      for (int k = 1; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
      mid = first + count / 2;
      std::nth_element(order.begin() + first, order.begin() + mid, order.begin() + first + count,
                       [&](uint32_t x, uint32_t y) { return cen[3 * (size_t)x + a] < cen[3 * (size_t)y + a]; });
    }
    const int l = build(first, mid - first, depth + 1);
    const int r = build(mid, first + count - mid, depth + 1);
    nodes[id].child[0] = l;
    nodes[id].child[1] = r;
    return id;
  }
};

// Outward padding of a box written to a node: 1e-5 of its largest coordinate
// magnitude, so FP32 slab-test rounding can only add work, never drop a hit.
void padded(const Box& b, float lo[3], float hi[3]) {
  float mag = 0.0f;
  for (int a = 0; a < 3; ++a) mag = std::max(mag, std::max(std::fabs(b.lo[a]), std::fabs(b.hi[a])));
  const float pad = 1e-5f * mag + 1e-30f;
  for (int a = 0; a < 3; ++a) {
    lo[a] = b.lo[a] - pad;
    hi[a] = b.hi[a] + pad;
  }
}

inline float bits(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace

bool build_bvh(const BuildInput& in, uint32_t bins, uint32_t max_leaf, uint32_t lds_levels, FlatBvh& out,
               std::string& err) {
  out = FlatBvh();
  const uint64_t n = in.nt + in.ns;
  if (n == 0) {
    err = "no primitives";
    return false;
  }
  if (n > kMaxSlots) {
    err = "too many primitives for 28-bit slot indices";
    return false;
  }
  Builder B;
  B.bins = bins;
  B.max_leaf = max_leaf;
  B.pbox.resize(n);
  B.cen.resize(3 * n);
  B.order.resize(n);
  for (uint64_t p = 0; p < n; ++p) {
    Box b;
    if (p < in.nt) {
      for (int k = 0; k < 3; ++k) b.grow(&in.verts[3 * (size_t)in.tris[3 * p + k]]);
    } else {
      const float* s = &in.spheres[4 * (p - in.nt)];
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::nextafter(s[a] - s[3], -INFINITY);
        b.hi[a] = std::nextafter(s[a] + s[3], INFINITY);
      }
    }
    B.pbox[p] = b;
    for (int a = 0; a < 3; ++a) B.cen[3 * p + a] = 0.5f * (b.lo[a] + b.hi[a]);
    B.order[p] = (uint32_t)p;
  }
  B.nodes.reserve(2 * n / std::max(1u, max_leaf) + 16);
  B.build(0, (uint32_t)n, 0);

  // root box
  for (int a = 0; a < 3; ++a) {
    out.lo[a] = B.nodes[0].box.lo[a];
    out.hi[a] = B.nodes[0].box.hi[a];
  }
  // a leaf root becomes an inner node with the leaf as both children
  if (B.nodes[0].leaf()) {
    Node leaf = B.nodes[0];
    leaf.depth = 1;
    B.nodes.push_back(leaf);
    B.nodes[0].child[0] = B.nodes[0].child[1] = (int32_t)B.nodes.size() - 1;
  }

  // flat index of every inner node: BFS for depth < lds_levels, then DFS
  std::vector<int64_t> flat(B.nodes.size(), -1);
  uint32_t next = 0;
  {
    std::deque<int> q;
    q.push_back(0);
    while (!q.empty()) {
      const int id = q.front();
      q.pop_front();
      const Node& nd = B.nodes[id];
      if (nd.leaf() || nd.depth >= lds_levels || next >= kMaxLdsNodes) continue;
      flat[id] = next++;
      q.push_back(nd.child[0]);
      q.push_back(nd.child[1]);
    }
    out.lds_nodes = next;
  }
  {
    std::vector<int> st{0};
    while (!st.empty()) {
      const int id = st.back();
      st.pop_back();
      const Node& nd = B.nodes[id];
      if (nd.leaf()) continue;
      if (flat[id] < 0) flat[id] = next++;
      out.max_depth = std::max(out.max_depth, nd.depth);
      st.push_back(nd.child[1]);
      st.push_back(nd.child[0]);
    }
  }
  out.nodes.assign((size_t)next * 4, make_float4(0, 0, 0, 0));
  for (size_t id = 0; id < B.nodes.size(); ++id) {
    const Node& nd = B.nodes[id];
    if (nd.leaf() || flat[id] < 0) continue;
    float lo[2][3], hi[2][3];
    uint32_t ref[2];
    for (int c = 0; c < 2; ++c) {
      const Node& ch = B.nodes[nd.child[c]];
      padded(ch.box, lo[c], hi[c]);
      if (ch.leaf()) {
        ref[c] = kLeafBit | (ch.first << 3) | (ch.count - 1);
      } else {
        ref[c] = (uint32_t)flat[nd.child[c]];
      }
    }
    float4* o = &out.nodes[(size_t)flat[id] * 4];
    o[0] = make_float4(lo[0][0], hi[0][0], lo[0][1], hi[0][1]);
    o[1] = make_float4(lo[1][0], hi[1][0], lo[1][1], hi[1][1]);
    o[2] = make_float4(lo[0][2], hi[0][2], lo[1][2], hi[1][2]);
    o[3] = make_float4(bits(ref[0]), bits(ref[1]), 0.0f, 0.0f);
  }
  for (const Node& nd : B.nodes)
    if (nd.leaf()) ++out.leaves;
  if (B.nodes.size() > 1 && B.nodes[0].child[0] == B.nodes[0].child[1]) out.leaves = 1;

  // primitive slots in leaf order
  out.slots.resize(3 * n);
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t p = B.order[i];
    float4* s = &out.slots[3 * i];
    if (p < in.nt) {
      const uint32_t* t = &in.tris[3 * (size_t)p];
      const float* v0 = &in.verts[3 * (size_t)t[0]];
      const float* v1 = &in.verts[3 * (size_t)t[1]];
      const float* v2 = &in.verts[3 * (size_t)t[2]];
      const uint32_t m = in.tri_mat ? in.tri_mat[p] : 0u;
      s[0] = make_float4(v0[0], v0[1], v0[2], bits(p));
      s[1] = make_float4(v1[0], v1[1], v1[2], bits(m));
      s[2] = make_float4(v2[0], v2[1], v2[2], bits(kPrimTriangle));
    } else {
      const float* sp = &in.spheres[4 * (size_t)(p - in.nt)];
      const uint32_t m = in.sph_mat ? in.sph_mat[p - in.nt] : 0u;
      s[0] = make_float4(sp[0], sp[1], sp[2], bits(p));
      s[1] = make_float4(sp[3], 0.0f, 0.0f, bits(m));
      s[2] = make_float4(0.0f, 0.0f, 0.0f, bits(kPrimSphere));
    }
  }
  return true;
}

}  // namespace npt
