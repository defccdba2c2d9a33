// bvh_build.cpp -- binned-SAH BVH2 builder and flattening to the two-box
// node layout the traversal kernel reads.
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <exception>
#include <thread>

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

// A primitive as the builder sorts it: its box, centroid and input index,
// moved together so that binning reads memory in order.
struct Prim {
  Box box;
  float c[3];
  uint32_t id;
};

struct Node {
  Box box;
  int32_t child[2] = {-1, -1};
  uint32_t first = 0, count = 0;  // leaf range in the primitive array
  uint32_t depth = 0;
  bool leaf() const { return child[0] < 0; }
};

// Host threads of one build: subtrees of at least kParallelPrims primitives
// build their second child on another thread while workers are free.  (The
// sanitizer tests build the builder with smaller thresholds, so that a small
// scene reaches every threaded stage.)
#ifndef NPT_BVH_PARALLEL_PRIMS
#define NPT_BVH_PARALLEL_PRIMS 100000u
#endif
#ifndef NPT_BVH_PARALLEL_BIN
#define NPT_BVH_PARALLEL_BIN (1u << 20)
#endif
#ifndef NPT_BVH_PARALLEL_RANGE
#define NPT_BVH_PARALLEL_RANGE (1u << 16)
#endif
constexpr uint32_t kParallelPrims = NPT_BVH_PARALLEL_PRIMS;

// the calling thread's cap on the build's threads (BuildThreads), 0 = none
thread_local int t_thread_cap = 0;

int host_threads() {
  const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  return t_thread_cap > 0 ? (int)std::min<unsigned>(hw, (unsigned)t_thread_cap) : (int)hw;
}

// fn(begin, end) over [0, n) in contiguous ranges on up to host_threads()
// threads (one range for small n)
template <class F>
void parallel_ranges(uint64_t n, F&& fn) {
  const uint64_t per = NPT_BVH_PARALLEL_RANGE;
  const int t = (int)std::min<uint64_t>((uint64_t)host_threads(), (n + per - 1) / per);
  if (t <= 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int i = 1; i < t; ++i) th.emplace_back([&, i] { fn(n * i / t, n * (i + 1) / t); });
  fn(0, n / t);
  for (auto& x : th) x.join();
}

// fn(chunk j, begin, end) over [0, n) split into t contiguous chunks, one thread each
template <class F>
void parallel_chunks(uint64_t n, int t, F&& fn) {
  std::vector<std::thread> th;
  for (int j = 1; j < t; ++j) th.emplace_back([&, j] { fn(j, n * j / t, n * (j + 1) / t); });
  fn(0, 0, n / t);
  for (auto& x : th) x.join();
}

// node ranges at least this large bound and bin their primitives on all threads
constexpr uint32_t kParallelBin = NPT_BVH_PARALLEL_BIN;

struct Builder {
  Prim* prims = nullptr;  // subtrees partition disjoint ranges of it in place
  std::vector<Node> nodes;
  uint32_t bins = 32, max_leaf = 4;
  int threads = 1;                      // threads that bound and bin one large range
  std::atomic<int>* workers = nullptr;  // threads that may still be started

  // appends a subtree built by another builder: its root becomes node
  // nodes.size(), its child indices move by the same offset
  int splice(const std::vector<Node>& sub) {
    const int off = (int)nodes.size();
    for (Node nd : sub) {
      if (!nd.leaf()) {
        nd.child[0] += off;
        nd.child[1] += off;
      }
      nodes.push_back(nd);
    }
    return off;
  }

  // Primitive and centroid bounds of prims[first, first + count).  Large
  // ranges are split over threads; min / max merge exactly in any order, so
  // the result is the same as one thread's.
  void bounds(uint32_t first, uint32_t count, Box& b, Box& cb) const {
    auto part = [&](uint64_t i0, uint64_t i1, Box& pb, Box& pc) {
      for (uint64_t i = first + i0; i < first + i1; ++i) {
        pb.grow(prims[i].box);
        pc.grow(prims[i].c);
      }
    };
    if (count < kParallelBin) {
      part(0, count, b, cb);
      return;
    }
    const int t = threads;
    std::vector<Box> pb(t), pc(t);
    parallel_chunks(count, t, [&](int j, uint64_t i0, uint64_t i1) { part(i0, i1, pb[j], pc[j]); });
    for (int j = 0; j < t; ++j) {
      b.grow(pb[j]);
      cb.grow(pc[j]);
    }
  }

  // SAH bins of prims[first, first + count) on axis a: boxes and counts (exact
  // merges: threads give the same bins as one)
  void bin_axis(uint32_t first, uint32_t count, int a, float lo, float scale, Box* bbox, uint32_t* bcnt) const {
    auto part = [&](uint64_t i0, uint64_t i1, Box* bb, uint32_t* bc) {
      for (uint64_t i = first + i0; i < first + i1; ++i) {
        const Prim& q = prims[i];
        int k = (int)((q.c[a] - lo) * scale);
        k = std::min(std::max(k, 0), (int)bins - 1);
        bb[k].grow(q.box);
        ++bc[k];
      }
    };
    std::fill(bbox, bbox + bins, Box());
    std::fill(bcnt, bcnt + bins, 0u);
    if (count < kParallelBin) {
      part(0, count, bbox, bcnt);
      return;
    }
    const int t = threads;
    std::vector<Box> bb((size_t)t * bins);
    std::vector<uint32_t> bc((size_t)t * bins, 0u);
    parallel_chunks(count, t, [&](int j, uint64_t i0, uint64_t i1) { part(i0, i1, &bb[(size_t)j * bins], &bc[(size_t)j * bins]); });
    for (int j = 0; j < t; ++j)
      for (uint32_t k = 0; k < bins; ++k) {
        bbox[k].grow(bb[(size_t)j * bins + k]);
        bcnt[k] += bc[(size_t)j * bins + k];
      }
  }

  int build(uint32_t first, uint32_t count, uint32_t depth) {
    const int id = (int)nodes.size();
    nodes.emplace_back();
    Box b, cb;
    bounds(first, count, b, cb);
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
        bin_axis(first, count, a, cb.lo[a], (float)bins / ext, bbox.data(), bcnt.data());
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
      const Prim* it = std::partition(prims + first, prims + first + count, [&](const Prim& q) {
        int k = (int)((q.c[a] - lo) * scale);
        k = std::min(std::max(k, 0), (int)bins - 1);
        return k <= sp;
      });
      mid = (uint32_t)(it - prims);
    }
    if (mid <= first || mid >= first + count) {
      // degenerate centroids or depth limit: object median on the widest axis
      int a = 0;
      for (int k = 1; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
      mid = first + count / 2;
      std::nth_element(prims + first, prims + mid, prims + first + count,
                       [&](const Prim& x, const Prim& y) { return x.c[a] < y.c[a]; });
    }
    const uint32_t rc = first + count - mid;
    int l, r;
    if (workers && rc >= kParallelPrims && workers->fetch_sub(1) > 0) {
      // the right subtree on its own thread and node array, spliced after
      // the left one: the tree is the one a single thread builds
      Builder sub;
      sub.prims = prims;
      sub.bins = bins;
      sub.max_leaf = max_leaf;
      sub.workers = workers;
      std::exception_ptr failed;  // an exception of the other thread, raised here after the join
      std::thread t([&] {
        try {
          sub.build(mid, rc, depth + 1);
        } catch (...) {
          failed = std::current_exception();
        }
        workers->fetch_add(1);  // free for other subtrees as soon as this one is done
      });
      try {
        l = build(first, mid - first, depth + 1);
      } catch (...) {
        t.join();
        throw;
      }
      t.join();
      if (failed) std::rethrow_exception(failed);
      r = splice(sub.nodes);
    } else {
      if (workers && rc >= kParallelPrims) workers->fetch_add(1);  // the claim above failed: give it back
      l = build(first, mid - first, depth + 1);
      r = build(mid, rc, depth + 1);
    }
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

inline uint32_t ubits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

// Structural check of a flattened tree before it is uploaded: every ref in
// range, every node reached exactly once from the root, every primitive slot
// covered by exactly one leaf, depth within max_depth.
bool check_flat(const FlatBvh& b, std::string& err) {
  const size_t nn = b.nodes.size() / b.node_float4s, ns = b.slots.size() / 3;
  std::vector<uint8_t> seen(nn, 0), covered(ns, 0);
  std::vector<std::pair<uint32_t, uint32_t>> st{{0u, 0u}};
  while (!st.empty()) {
    const auto [id, depth] = st.back();
    st.pop_back();
    if (id >= nn || seen[id]) {
      err = "flattened BVH: node reached twice or out of range";
      return false;
    }
    if (depth > b.max_depth) {
      err = "flattened BVH: depth exceeds max_depth";
      return false;
    }
    seen[id] = 1;
    const float4* o = &b.nodes[(size_t)id * b.node_float4s];
    uint32_t refs[4];
    int nref = 0;
    if (b.width == 2) {
      refs[nref++] = ubits(o[3].x);
      if (ubits(o[3].y) != ubits(o[3].x)) refs[nref++] = ubits(o[3].y);
    } else {
      const uint32_t r[4] = {ubits(o[6].x), ubits(o[6].y), ubits(o[6].z), ubits(o[6].w)};
      for (uint32_t x : r)
        if (x != kEmptyChild) refs[nref++] = x;
    }
    for (int k = 0; k < nref; ++k) {
      const uint32_t r = refs[k];
      if (r & kLeafBit) {
        const uint32_t first = (r >> 3) & 0x0FFFFFFFu, count = (r & 7u) + 1u;
        if ((uint64_t)first + count > ns) {
          err = "flattened BVH: leaf beyond the primitive slots";
          return false;
        }
        for (uint32_t i = first; i < first + count; ++i) {
          if (covered[i]) {
            err = "flattened BVH: primitive slot in two leaves";
            return false;
          }
          covered[i] = 1;
        }
      } else {
        st.push_back({r, depth + 1});
      }
    }
  }
  for (size_t i = 0; i < nn; ++i)
    if (!seen[i]) {
      err = "flattened BVH: unreachable node";
      return false;
    }
  for (size_t i = 0; i < ns; ++i)
    if (!covered[i]) {
      err = "flattened BVH: primitive slot in no leaf";
      return false;
    }
  return true;
}

// smallest binary16 value >= v (v >= 0, finite), as bits; false beyond 65504
bool half_up(double v, uint16_t& h) {
  if (!(v <= 65504.0)) return false;
  if (v <= 0.0) {
    h = 0;
    return true;
  }
  int e;
  (void)std::frexp(v, &e);  // v in [2^(e-1), 2^e)
  int lead = std::max(e - 1, -14);
  double q = std::ldexp(1.0, lead - 10);
  double m = std::ceil(v / q);  // v <= m q, m < 2^11
  if (m >= 2048.0) {            // rounded up into the next binade
    m = 1024.0;
    lead += 1;
  }
  if (lead == -14 && m < 1024.0) {
    h = (uint16_t)m;  // subnormal: mantissa only
  } else {
    h = (uint16_t)(((lead + 15) << 10) | ((uint32_t)m - 1024u));
  }
  return lead <= 15;
}

float half_value(uint16_t h) {
  const int ex = (h >> 10) & 31, man = h & 1023;
  if (ex == 0) return (float)std::ldexp((double)man, -24);
  return (float)std::ldexp((double)(1024 + man), ex - 25);
}

uint16_t half_next(uint16_t h) { return (uint16_t)(h + 1); }  // next larger non-negative binary16

// largest binary16 value <= v (v >= 0, finite, at most 65504), as bits
uint16_t half_down(double v) {
  uint16_t h = 0;
  if (!half_up(v, h)) return 0x7BFF;  // 65504
  while (h > 0 && (double)half_value(h) > v) --h;
  return h;
}

}  // namespace

bool compress_half_extents(FlatBvh& b, std::string& err) {
  if (b.width != 4 || b.node_float4s != kNode4Float4s) {
    err = "FP16 extents need 4-wide FP32 nodes";
    return false;
  }
  const size_t nn = b.nodes.size() / kNode4Float4s;
  std::vector<float4> out(nn * kNode4HalfFloat4s);
  // one node; false when an extent does not fit binary16
  auto node = [&](size_t i) -> bool {
    const float4* o = &b.nodes[i * kNode4Float4s];
    float4* h = &out[i * kNode4HalfFloat4s];
    uint16_t ext[3][4];
    float lo[3][4];
    for (int a = 0; a < 3; ++a) {
      const float l4[4] = {o[2 * a].x, o[2 * a].y, o[2 * a].z, o[2 * a].w};
      const float h4[4] = {o[2 * a + 1].x, o[2 * a + 1].y, o[2 * a + 1].z, o[2 * a + 1].w};
      const uint32_t r4[4] = {ubits(o[6].x), ubits(o[6].y), ubits(o[6].z), ubits(o[6].w)};
      for (int c = 0; c < 4; ++c) {
        if (r4[c] == kEmptyChild) {
          lo[a][c] = INFINITY;
          ext[a][c] = 0;
          continue;
        }
        lo[a][c] = l4[c];
        uint16_t e;
        if (!half_up((double)h4[c] - (double)l4[c], e)) return false;
        // the traversal forms the upper plane as an FP32 sum: make sure it
        // does not fall below the true one
        while ((float)(l4[c] + half_value(e)) < h4[c]) {
          e = half_next(e);
          if (half_value(e) > 65504.0f || ((e >> 10) & 31) == 31) return false;
        }
        ext[a][c] = e;
      }
    }
    auto pack = [](uint16_t a, uint16_t b2) { return bits((uint32_t)a | ((uint32_t)b2 << 16)); };
    h[0] = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
    h[1] = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
    h[2] = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
    h[3] = make_float4(pack(ext[0][0], ext[0][1]), pack(ext[0][2], ext[0][3]), pack(ext[1][0], ext[1][1]),
                       pack(ext[1][2], ext[1][3]));
    h[4] = make_float4(pack(ext[2][0], ext[2][1]), pack(ext[2][2], ext[2][3]), 0.0f, 0.0f);
    h[5] = o[6];
    return true;
  };
  std::atomic<bool> wide{false};
  parallel_ranges(nn, [&](uint64_t i0, uint64_t i1) {
    for (uint64_t i = i0; i < i1; ++i)
      if (!node(i)) wide = true;
  });
  if (wide) {
    err = "FP16 extents: a box is wider than 65504";
    return false;
  }
  b.nodes = std::move(out);
  b.node_float4s = kNode4HalfFloat4s;
  return true;
}

bool compress_q8_nodes(FlatBvh& b, std::string& err) {
  if (b.width != 4 || b.node_float4s != kNode4Float4s) {
    err = "quantized nodes need 4-wide FP32 nodes";
    return false;
  }
  const size_t nn = b.nodes.size() / kNode4Float4s;
  std::vector<float4> out(nn * kNode4Q8Float4s);
  for (size_t i = 0; i < nn; ++i) {
    const float4* o = &b.nodes[i * kNode4Float4s];
    const uint32_t r4[4] = {ubits(o[6].x), ubits(o[6].y), ubits(o[6].z), ubits(o[6].w)};
    float origin[3];
    uint32_t qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0}, ebits = 0;
    for (int a = 0; a < 3; ++a) {
      const float l4[4] = {o[2 * a].x, o[2 * a].y, o[2 * a].z, o[2 * a].w};
      const float h4[4] = {o[2 * a + 1].x, o[2 * a + 1].y, o[2 * a + 1].z, o[2 * a + 1].w};
      float lo = INFINITY, hi = -INFINITY;
      for (int c = 0; c < 4; ++c)
        if (r4[c] != kEmptyChild) {
          lo = std::min(lo, l4[c]);
          hi = std::max(hi, h4[c]);
        }
      if (!(lo <= hi)) {
        err = "quantized nodes: node without children";
        return false;
      }
      origin[a] = lo;
      // smallest power-of-two step 2^e with 254 steps covering the children;
      // raised until every child's rounded-outward planes fit in 0..255
      const double span = (double)hi - (double)lo;
      int e = span > 0.0 ? (int)std::ceil(std::log2(span / 254.0)) : -126;
      e = std::max(e, -126);
      for (;; ++e) {
        const float s = std::ldexp(1.0f, e);
        bool fit = true;
        uint32_t ql = 0, qh = 0;
        for (int c = 0; c < 4 && fit; ++c) {
          uint32_t a_lo = 255, a_hi = 0;  // empty child: inverted box
          if (r4[c] != kEmptyChild) {
            // decoded planes are the FP32 values lo + q s (q s is exact):
            // lower plane rounded down, upper plane rounded up
            double fl = std::floor(((double)l4[c] - (double)lo) / (double)s);
            double fh = std::ceil(((double)h4[c] - (double)lo) / (double)s);
            int64_t q0 = (int64_t)std::max(0.0, fl), q1 = (int64_t)fh;
            while (q0 > 0 && lo + (float)q0 * s > l4[c]) --q0;
            while (q1 <= 255 && lo + (float)q1 * s < h4[c]) ++q1;
            if (q1 > 255 || !(lo + (float)q0 * s <= l4[c])) {
              fit = false;
              break;
            }
            a_lo = (uint32_t)q0;
            a_hi = (uint32_t)q1;
          }
          ql |= a_lo << (8 * c);
          qh |= a_hi << (8 * c);
        }
        if (fit) {
          qlo[a] = ql;
          qhi[a] = qh;
          break;
        }
        if (e > 127) {
          err = "quantized nodes: no step covers a box";
          return false;
        }
      }
      ebits |= (uint32_t)(e + 128) << (8 * a);
    }
    float4* h = &out[i * kNode4Q8Float4s];
    h[0] = make_float4(origin[0], origin[1], origin[2], bits(ebits));
    h[1] = make_float4(bits(qlo[0]), bits(qhi[0]), bits(qlo[1]), bits(qhi[1]));
    h[2] = make_float4(bits(qlo[2]), bits(qhi[2]), 0.0f, 0.0f);
    h[3] = o[6];
  }
  b.nodes = std::move(out);
  b.node_float4s = kNode4Q8Float4s;
  return true;
}

bool compress_corner_nodes(FlatBvh& b, std::string& err) {
  if (b.width != 4 || b.node_float4s != kNode4Float4s) {
    err = "corner nodes need 4-wide FP32 nodes";
    return false;
  }
  const size_t nn = b.nodes.size() / kNode4Float4s;
  std::vector<float4> out(nn * kNode4CornerFloat4s);
  // one node; false when a plane offset does not fit binary16
  auto node = [&](size_t i) -> bool {
    const float4* o = &b.nodes[i * kNode4Float4s];
    float4* h = &out[i * kNode4CornerFloat4s];
    const uint32_t r4[4] = {ubits(o[6].x), ubits(o[6].y), ubits(o[6].z), ubits(o[6].w)};
    float corner[3];
    uint32_t words[3][4];
    for (int a = 0; a < 3; ++a) {
      const float l4[4] = {o[2 * a].x, o[2 * a].y, o[2 * a].z, o[2 * a].w};
      const float h4[4] = {o[2 * a + 1].x, o[2 * a + 1].y, o[2 * a + 1].z, o[2 * a + 1].w};
      float c0 = INFINITY;
      for (int c = 0; c < 4; ++c)
        if (r4[c] != kEmptyChild) c0 = std::min(c0, l4[c]);
      if (!(c0 < INFINITY)) return false;
      corner[a] = c0;
      uint16_t qlo[4], qhi[4];
      for (int c = 0; c < 4; ++c) {
        if (r4[c] == kEmptyChild) {
          qlo[c] = 0x7C00;  // +inf
          qhi[c] = 0;
          continue;
        }
        // the traversal forms each plane as the FP32 sum corner + q
        uint16_t lo = half_down((double)l4[c] - (double)c0);
        while (lo > 0 && c0 + half_value(lo) > l4[c]) --lo;
        if (c0 + half_value(lo) > l4[c]) return false;
        uint16_t hi;
        if (!half_up((double)h4[c] - (double)c0, hi)) return false;
        while (c0 + half_value(hi) < h4[c]) {
          hi = half_next(hi);
          if (((hi >> 10) & 31) == 31) return false;
        }
        qlo[c] = lo;
        qhi[c] = hi;
      }
      words[a][0] = (uint32_t)qlo[0] | ((uint32_t)qlo[1] << 16);
      words[a][1] = (uint32_t)qlo[2] | ((uint32_t)qlo[3] << 16);
      words[a][2] = (uint32_t)qhi[0] | ((uint32_t)qhi[1] << 16);
      words[a][3] = (uint32_t)qhi[2] | ((uint32_t)qhi[3] << 16);
    }
    h[0] = make_float4(corner[0], corner[1], corner[2], 0.0f);
    for (int a = 0; a < 3; ++a)
      h[1 + a] = make_float4(bits(words[a][0]), bits(words[a][1]), bits(words[a][2]), bits(words[a][3]));
    h[4] = o[6];
    return true;
  };
  std::atomic<bool> bad{false};
  parallel_ranges(nn, [&](uint64_t i0, uint64_t i1) {
    for (uint64_t i = i0; i < i1; ++i)
      if (!node(i)) bad = true;
  });
  if (bad) {
    err = "binary16 corner nodes: a node spans more than 65504";
    return false;
  }
  b.nodes = std::move(out);
  b.node_float4s = kNode4CornerFloat4s;
  return true;
}

BuildThreads::BuildThreads(int n) : prev_(t_thread_cap) { t_thread_cap = n > 0 ? n : 0; }
BuildThreads::~BuildThreads() { t_thread_cap = prev_; }

bool build_bvh(const BuildInput& in, uint32_t bins, uint32_t max_leaf, uint32_t lds_levels, uint32_t width,
               FlatBvh& out,
               std::string& err) {
  out = FlatBvh();
  const uint64_t n = in.nboxes ? in.nboxes : in.nt + in.ns;
  if (n == 0) {
    err = "no primitives";
    return false;
  }
  if (n > kMaxSlots) {
    err = "too many primitives for 28-bit slot indices";
    return false;
  }
  std::vector<Prim> prims(n);
  parallel_ranges(n, [&](uint64_t p0, uint64_t p1) {
    for (uint64_t p = p0; p < p1; ++p) {
      Box b;
      if (in.nboxes) {
        b.grow(&in.boxes[6 * p]);
        b.grow(&in.boxes[6 * p + 3]);
      } else if (p < in.nt) {
        for (int k = 0; k < 3; ++k) b.grow(&in.verts[3 * (size_t)in.tris[3 * p + k]]);
      } else {
        const float* s = &in.spheres[4 * (p - in.nt)];
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = std::nextafter(s[a] - s[3], -INFINITY);
          b.hi[a] = std::nextafter(s[a] + s[3], INFINITY);
        }
      }
      Prim& q = prims[p];
      q.box = b;
      for (int a = 0; a < 3; ++a) q.c[a] = 0.5f * (b.lo[a] + b.hi[a]);
      q.id = (uint32_t)p;
    }
  });
  std::atomic<int> workers{host_threads() - 1};
  Builder B;
  B.threads = host_threads();
  B.bins = bins;
  B.max_leaf = max_leaf;
  B.prims = prims.data();
  B.workers = &workers;
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

  // wide nodes: the children of a binary inner node, widened (for width 4) by
  // repeatedly opening the inner child with the largest surface area
  std::vector<std::vector<int>> kids(B.nodes.size());
  std::vector<uint32_t> wdepth(B.nodes.size(), 0);
  std::vector<int> wide;  // binary ids that become wide nodes, parents first
  {
    std::vector<int> st{0};
    while (!st.empty()) {
      const int id = st.back();
      st.pop_back();
      wide.push_back(id);
      std::vector<int> ch{B.nodes[id].child[0], B.nodes[id].child[1]};
      if (ch[0] == ch[1]) ch.pop_back();  // leaf root
      while ((int)ch.size() < (int)width) {
        int best = -1;
        double area = -1.0;
        for (size_t i = 0; i < ch.size(); ++i) {
          const Node& c = B.nodes[ch[i]];
          if (!c.leaf() && c.box.half_area() > area) {
            area = c.box.half_area();
            best = (int)i;
          }
        }
        if (best < 0) break;
        const int open = ch[best];
        ch.erase(ch.begin() + best);
        ch.push_back(B.nodes[open].child[0]);
        ch.push_back(B.nodes[open].child[1]);
      }
      for (int c : ch) {
        if (B.nodes[c].leaf()) continue;
        wdepth[c] = wdepth[id] + 1;
        st.push_back(c);
      }
      kids[id] = std::move(ch);
    }
  }
  // flat index of every wide node: BFS for depth < lds_levels, then DFS
  std::vector<int64_t> flat(B.nodes.size(), -1);
  uint32_t next = 0;
  {
    std::deque<int> q;
    q.push_back(0);
    while (!q.empty()) {
      const int id = q.front();
      q.pop_front();
      if (B.nodes[id].leaf() || wdepth[id] >= lds_levels || next >= kMaxLdsNodes) continue;
      flat[id] = next++;
      for (int c : kids[id]) q.push_back(c);
    }
    out.lds_nodes = next;
  }
  {
    std::vector<int> st{0};
    while (!st.empty()) {
      const int id = st.back();
      st.pop_back();
      if (B.nodes[id].leaf()) continue;
      if (flat[id] < 0) flat[id] = next++;
      out.max_depth = std::max(out.max_depth, wdepth[id]);
      for (auto it = kids[id].rbegin(); it != kids[id].rend(); ++it) st.push_back(*it);
    }
  }
  out.width = width;
  out.node_float4s = width == 2 ? 4 : kNode4Float4s;
  out.nodes.assign((size_t)next * out.node_float4s, make_float4(0, 0, 0, 0));
  for (int id : wide) {
    const std::vector<int>& ch = kids[id];
    float lo[4][3], hi[4][3];
    uint32_t ref[4];
    for (int c = 0; c < 4; ++c) {
      if (c < (int)ch.size()) {
        const Node& k = B.nodes[ch[c]];
        padded(k.box, lo[c], hi[c]);
        ref[c] = k.leaf() ? (kLeafBit | (k.first << 3) | (k.count - 1)) : (uint32_t)flat[ch[c]];
      } else {
        for (int a = 0; a < 3; ++a) {
          lo[c][a] = INFINITY;
          hi[c][a] = -INFINITY;
        }
        ref[c] = kEmptyChild;
      }
    }
    float4* o = &out.nodes[(size_t)flat[id] * out.node_float4s];
    if (width == 2) {
      if (ch.size() == 1) {  // single-leaf scene: the leaf as both children
        for (int a = 0; a < 3; ++a) {
          lo[1][a] = lo[0][a];
          hi[1][a] = hi[0][a];
        }
        ref[1] = ref[0];
      }
      o[0] = make_float4(lo[0][0], hi[0][0], lo[0][1], hi[0][1]);
      o[1] = make_float4(lo[1][0], hi[1][0], lo[1][1], hi[1][1]);
      o[2] = make_float4(lo[0][2], hi[0][2], lo[1][2], hi[1][2]);
      o[3] = make_float4(bits(ref[0]), bits(ref[1]), 0.0f, 0.0f);
    } else {
      for (int a = 0; a < 3; ++a) {
        o[2 * a] = make_float4(lo[0][a], lo[1][a], lo[2][a], lo[3][a]);
        o[2 * a + 1] = make_float4(hi[0][a], hi[1][a], hi[2][a], hi[3][a]);
      }
      o[6] = make_float4(bits(ref[0]), bits(ref[1]), bits(ref[2]), bits(ref[3]));
    }
  }
  for (const Node& nd : B.nodes)
    if (nd.leaf()) ++out.leaves;
  if (B.nodes.size() > 1 && B.nodes[0].child[0] == B.nodes[0].child[1]) out.leaves = 1;

  // primitive slots in leaf order
  out.slots.resize(3 * n);
  parallel_ranges(n, [&](uint64_t i0, uint64_t i1) {
    for (uint64_t i = i0; i < i1; ++i) {
      const uint32_t p = prims[i].id;
      float4* s = &out.slots[3 * i];
      if (in.nboxes) {
        // box mode: the slot only names the input box it holds
        s[0] = make_float4(0.0f, 0.0f, 0.0f, bits(p));
        s[1] = s[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      } else if (p < in.nt) {
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
  });
  return check_flat(out, err);
}

bool build_two_level(const std::vector<FlatBvh>& bottoms, const std::vector<Placement>& objects, uint32_t bins,
                     uint32_t lds_levels, FlatBvh& out, std::vector<float4>& records, uint32_t& stack_entries,
                     std::string& err) {
  out = FlatBvh();
  records.clear();
  if (objects.empty()) {
    err = "no objects";
    return false;
  }
  // world box of every object: the bottom tree's bounds, scaled and moved
  std::vector<float> boxes(6 * objects.size());
  for (size_t i = 0; i < objects.size(); ++i) {
    const Placement& o = objects[i];
    if (o.tree >= bottoms.size() || bottoms[o.tree].width != 4 || !(o.scale > 0.0f)) {
      err = "two-level layout: bad placement";
      return false;
    }
    const FlatBvh& b = bottoms[o.tree];
    for (int a = 0; a < 3; ++a) {
      boxes[6 * i + a] = b.lo[a] * o.scale + o.translate[a];
      boxes[6 * i + 3 + a] = b.hi[a] * o.scale + o.translate[a];
    }
  }
  BuildInput tin;
  tin.boxes = boxes.data();
  tin.nboxes = objects.size();
  FlatBvh top;
  if (!build_bvh(tin, bins, 1, lds_levels, 4, top, err)) return false;

  out.width = 4;
  out.node_float4s = kNode4Float4s;
  out.nodes = top.nodes;
  out.leaves = top.leaves;
  out.lds_nodes = top.lds_nodes;  // the top tree's BFS-ordered first levels
  for (int a = 0; a < 3; ++a) {
    out.lo[a] = top.lo[a];
    out.hi[a] = top.hi[a];
  }
  std::vector<uint32_t> root(bottoms.size());
  uint32_t deepest = 0;
  size_t total_nodes = out.nodes.size(), total_slots = 0;
  for (const FlatBvh& b : bottoms) {
    total_nodes += b.nodes.size();
    total_slots += b.slots.size();
  }
  if (total_nodes / kNode4Float4s >= kEmptyChild || total_slots / 3 > kMaxSlots) {
    err = "two-level layout: too many nodes or primitive slots";
    return false;
  }
  out.nodes.resize(total_nodes);
  out.slots.resize(total_slots);
  size_t nf = top.nodes.size(), sf = 0;  // float4s placed so far
  for (size_t t = 0; t < bottoms.size(); ++t) {
    const FlatBvh& b = bottoms[t];
    const uint32_t node_off = (uint32_t)(nf / kNode4Float4s), slot_off = (uint32_t)(sf / 3);
    root[t] = node_off;
    // each node moves by node_off, its child refs by node_off (inner) or
    // slot_off (leaves)
    parallel_ranges(b.nodes.size() / kNode4Float4s, [&](uint64_t i0, uint64_t i1) {
      for (uint64_t i = i0; i < i1; ++i) {
        const float4* src = &b.nodes[i * kNode4Float4s];
        float4* dst = &out.nodes[nf + i * kNode4Float4s];
        for (uint32_t k = 0; k < kNode4Float4s; ++k) dst[k] = src[k];
        float* r4[4] = {&dst[6].x, &dst[6].y, &dst[6].z, &dst[6].w};
        for (float* f : r4) {
          uint32_t r = ubits(*f);
          if (r == kEmptyChild) continue;
          if (r & kLeafBit) {
            const uint32_t first = ((r >> 3) & 0x0FFFFFFFu) + slot_off;
            r = kLeafBit | (first << 3) | (r & 7u);
          } else {
            r += node_off;
          }
          *f = bits(r);
        }
      }
    });
    std::copy(b.slots.begin(), b.slots.end(), out.slots.begin() + sf);
    nf += b.nodes.size();
    sf += b.slots.size();
    out.leaves += b.leaves;
    deepest = std::max(deepest, b.max_depth);
  }
  // one record per top-tree leaf, in the top tree's slot order
  const size_t nrec = top.slots.size() / 3;
  records.resize(2 * nrec);
  for (size_t i = 0; i < nrec; ++i) {
    const uint32_t p = ubits(top.slots[3 * i].w);
    const Placement& o = objects[p];
    records[2 * i] = make_float4(o.translate[0], o.translate[1], o.translate[2], o.scale);
    records[2 * i + 1] = make_float4(bits(root[o.tree]), bits(o.id), 1.0f / o.scale, 0.0f);
  }
  // top leaves hold one object each (leaf size 1)
  for (size_t i = 0; i < top.nodes.size(); i += kNode4Float4s) {
    const float4 rf = top.nodes[i + 6];
    for (float f : {rf.x, rf.y, rf.z, rf.w}) {
      const uint32_t r = ubits(f);
      if (r != kEmptyChild && (r & kLeafBit) && ((r & 7u) != 0u || ((r >> 3) & 0x0FFFFFFFu) >= nrec)) {
        err = "two-level layout: top leaf with more than one object";
        return false;
      }
    }
  }
  out.max_depth = top.max_depth + 1 + deepest;
  // at most three deferred children per 4-wide level, plus the three of the
  // deepest node, in each of the two trees
  stack_entries = 3 * (top.max_depth + 1) + 3 * (deepest + 1);
  return true;
}

}  // namespace npt
