// k_render.hip -- wavefront path-tracing kernels (Sec. 3.1, 3.3 of the paper):
// camera rays, closest-hit traversal + shading with wave-level queue
// compaction, bilinear environment lookup, per-pixel accumulation.
#include <hip/hip_runtime.h>

#include "npt_device.h"
#include "npt_kernels.h"
#include "npt_shared.h"
#include "npt_train.h"

namespace npt {

#ifndef NPT_TRACE_BLOCK
#define NPT_TRACE_BLOCK 64  // one wave per workgroup: measured fastest (64 < 128 < 256)
#endif
#ifndef NPT_SHORT_STACK
#define NPT_SHORT_STACK 16  // traversal stack entries per lane kept in LDS
#endif
constexpr int kTraceBlock = NPT_TRACE_BLOCK;
constexpr int kWave = 64;
constexpr uint32_t kMaxVisits = 1u << 22;
#ifndef NPT_REFILL_AT
#define NPT_REFILL_AT 48  // lanes still traversing at which a wave takes new rays
#endif
constexpr int kRefillAt = NPT_REFILL_AT;
#ifndef NPT_LEAF_PERCENT
#define NPT_LEAF_PERCENT 100  // leaf step once waiting leaf lanes reach this % of the lanes at inner nodes
#endif
constexpr uint32_t kLeafPercent = NPT_LEAF_PERCENT;
static_assert(kLeafPercent <= 100000u, "the leaf-step rule is evaluated in 32 bits");

// Lanes of the wave for which b holds, straight from the lane mask the
// compare leaves (HIP's __ballot takes an int and turns the mask into a
// value and back: two vector instructions more).
__device__ __forceinline__ uint64_t lanes(bool b) { return __builtin_amdgcn_ballot_w64(b); }
#ifndef NPT_EXTEND_WAVES
#define NPT_EXTEND_WAVES 6  // waves per SIMD the extend kernel's register budget is set for
#endif

// ---------------------------------------------------------------------------
// camera (pinhole) -- same definitions as the host-side basis
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 camera_direction(const CameraView& cam, uint32_t W, uint32_t H,
                                               uint32_t x, uint32_t y, float jx, float jy) {
  const float px = ((float)x + jx) / (float)W;
  const float py = ((float)y + jy) / (float)H;
  const float sx = 2.0f * px - 1.0f;
  const float sy = 1.0f - 2.0f * py;
  const float cx = sx * cam.tan_x;
  const float cy = sy * cam.tan_y;
  const V3 d{(cam.fwd[0] + cx * cam.right[0]) + cy * cam.up[0],
             (cam.fwd[1] + cx * cam.right[1]) + cy * cam.up[1],
             (cam.fwd[2] + cx * cam.right[2]) + cy * cam.up[2]};
  return normalized(d);
}

// ---------------------------------------------------------------------------
// closest hit: stack traversal of the BVH (binary, 4-wide, or two-level over
// instances); the top `lds_nodes` nodes of a one-level tree come from LDS.
// Ties on t go to the lowest (instance, primitive).
// ---------------------------------------------------------------------------
struct Hit {
  float t;
  uint32_t slot;  // primitive slot (its id in the slot's first .w)
  uint32_t inst;  // 0 for the base geometry, k + 1 for instance k
};

__device__ __forceinline__ uint32_t slot_prim(const float4* slots, uint32_t slot) {
  return __float_as_uint(slots[3 * (size_t)slot].w);
}

// Pointers typed as LDS (address space 3): their loads and stores are
// ds_read / ds_write.  Through a generic pointer the compiler may fall back
// to flat instructions, which go through the texture address and data units
// (the traversal's busiest path) and wait on both memory counters.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) float lds_f32;

// Per-lane traversal stack of kCap entries: the first kShort live in LDS at
// lds[i * kStride], deeper ones in a private array that only deep
// traversals reach.  The LDS part is what bounds the occupancy of the trace
// kernels.  A push beyond kCap is dropped; kCap is sized from the tree depth
// so that it never is.
template <int kCap, int kStride>
struct LaneStack {
  static constexpr int kShort = kCap < NPT_SHORT_STACK ? kCap : NPT_SHORT_STACK;
  static constexpr int kDeep = kCap - kShort;
  lds_u32* lds;
  uint32_t deep[kDeep > 0 ? kDeep : 1];
  __device__ __forceinline__ void push(int& sp, uint32_t v) {
    if (sp < kShort) {
      lds[sp * kStride] = v;
    } else if (kDeep > 0 && sp < kCap) {
      deep[sp - kShort] = v;
    } else {
      return;
    }
    ++sp;
  }
  // r3, r2, r1 in this order, each only if its flag is set, where the
  // flags are a prefix (h3 implies h2 implies h1: the entered children of a
  // sorted node).  While three entries fit in LDS, slots sp, sp + 1, sp + 2
  // are written unconditionally from one address (immediate offsets; a
  // store above the final top is dead) and sp grows by the count.
  __device__ __forceinline__ void push3(int& sp, uint32_t r3, bool h3, uint32_t r2, bool h2, uint32_t r1, bool h1) {
    if (sp + 3 <= kShort) {
      lds_u32* p = lds + sp * kStride;
      p[0] = h3 ? r3 : (h2 ? r2 : r1);
      p[kStride] = h3 ? r2 : r1;
      p[2 * kStride] = r1;
      sp += (int)h1 + (int)h2 + (int)h3;
    } else {
      if (h3) push(sp, r3);
      if (h2) push(sp, r2);
      if (h1) push(sp, r1);
    }
  }
  __device__ __forceinline__ uint32_t pop(int& sp) {
    --sp;
    if (kDeep == 0 || sp < kShort) return lds[sp * kStride];
    return deep[sp - kShort];
  }
};

// Reciprocal of a direction component for the slab tests: the hardware
// reciprocal (within 1 ulp) of x with |x| clamped to [1e-20, 2^126], so that
// it is finite, normal and of x's sign.  Its error is part of what
// kSlabSlack covers (below); no hit depends on it beyond that, since the
// slab tests only decide which boxes are opened.
__device__ __forceinline__ float safe_inverse(float x) {
  return __builtin_amdgcn_rcpf(copysignf(fminf(fmaxf(fabsf(x), 1e-20f), 0x1p126f), x));
}

// Ray in the frame a tree is traversed in: origin, direction, the shear of
// the watertight triangle test and the slab-test terms.
//
// A slab distance is formed as fma(plane, ix, -o * ix).  Against the exact
// (plane - o) / d it errs by a part relative to the distance itself (the
// reciprocal's error, at most 1 ulp, scales plane and origin term alike,
// plus the fma's rounding: 1.5 ulp together) and a part of up to one
// rounding of o * ix, which does not shrink with the distance.  The second
// part is taken out per ray: the origin term of the entry (near) plane of
// each axis is moved up by 4 ulp-units of |o * ix| and that of the exit
// (far) plane down, so the computed interval of every axis contains the
// exact one up to the relative part, which kSlabSlack (8 ulp, against the
// 3 ulp that entry and exit distance can drift apart) covers.  Boxes are
// then never missed by a ray that enters them, whatever the distance
// between origin and box.
//
// Which plane of an axis is the entry plane depends only on the sign of the
// direction, so 4-wide nodes are read plane row by plane row: near_x is the
// byte offset of the entry-plane row of x in a node (lo.x at 0 or hi.x at
// 16; y at 32 / 48, z at 64 / 80), and no per-child min / max is needed.
struct RayFrame {
  V3 o, d;
  float ix, iy, iz;
  float ox_n, oy_n, oz_n;  // origin terms of the entry planes
  float ox_f, oy_f, oz_f;  // and of the exit planes
  uint32_t near_x, near_y, near_z;
  uint32_t wx, wy, wz;  // binary16 pair per axis: entry-plane weight (low), exit-plane weight (high)
  uint32_t mx, my, mz;  // all ones where the direction component is >= 0
};

constexpr float kSlabSlack = 1.0f + 0x1p-20f;

__device__ __forceinline__ void origin_terms(float o, float inv, float& near_t, float& far_t) {
  const float oi = o * inv;
  const float e = fabsf(oi) * 0x1p-22f;
  near_t = oi + e;
  far_t = oi - e;
}

__device__ __forceinline__ RayFrame make_frame(V3 o, V3 d) {
  RayFrame f;
  f.o = o;
  f.d = d;
  f.ix = safe_inverse(d.x);
  f.iy = safe_inverse(d.y);
  f.iz = safe_inverse(d.z);
  origin_terms(o.x, f.ix, f.ox_n, f.ox_f);
  origin_terms(o.y, f.iy, f.oy_n, f.oy_f);
  origin_terms(o.z, f.iz, f.oz_n, f.oz_f);
  f.near_x = f.ix >= 0.0f ? 0u : 16u;
  f.near_y = f.iy >= 0.0f ? 32u : 48u;
  f.near_z = f.iz >= 0.0f ? 64u : 80u;
  f.wx = f.ix >= 0.0f ? 0x3C000000u : 0x00003C00u;
  f.wy = f.iy >= 0.0f ? 0x3C000000u : 0x00003C00u;
  f.wz = f.iz >= 0.0f ? 0x3C000000u : 0x00003C00u;
  f.mx = f.ix >= 0.0f ? ~0u : 0u;
  f.my = f.iy >= 0.0f ? ~0u : 0u;
  f.mz = f.iz >= 0.0f ? ~0u : 0u;
  return f;
}

// entry and exit distance of one box against [0, lim] (binary nodes, whose
// lo / hi planes are interleaved per child)
__device__ __forceinline__ void slab(const RayFrame& f, float lx, float hx, float ly, float hy, float lz, float hz,
                                     float lim, float& tn, float& tf) {
  const bool px = f.ix >= 0.0f, py = f.iy >= 0.0f, pz = f.iz >= 0.0f;
  const float a0 = __builtin_fmaf(lx, f.ix, -(px ? f.ox_n : f.ox_f)), a1 = __builtin_fmaf(hx, f.ix, -(px ? f.ox_f : f.ox_n));
  const float b0 = __builtin_fmaf(ly, f.iy, -(py ? f.oy_n : f.oy_f)), b1 = __builtin_fmaf(hy, f.iy, -(py ? f.oy_f : f.oy_n));
  const float c0 = __builtin_fmaf(lz, f.iz, -(pz ? f.oz_n : f.oz_f)), c1 = __builtin_fmaf(hz, f.iz, -(pz ? f.oz_f : f.oz_n));
  tn = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
  tf = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), lim)) * kSlabSlack;
}

// primitive tests of one leaf; the hit is kept on a smaller t, or on equal t
// with a smaller (instance, primitive)
template <bool kCount>
__device__ __forceinline__ void test_leaf(const SceneView& sc, const RayFrame& f, uint32_t ref, uint32_t inst,
                                          Hit& h, uint32_t* n_prims) {
  // the shear constants of the watertight test are recomputed per leaf
  // rather than kept per lane: six fewer live registers during traversal
  const Shear sh = make_shear(f.d);
  const uint32_t first = (ref >> 3) & 0x0FFFFFFFu;
  const uint32_t count = (ref & 7u) + 1u;
  if constexpr (kCount) *n_prims += count;
  for (uint32_t i = 0; i < count; ++i) {
    const float4* s = sc.slots + 3 * (size_t)(first + i);
    const float4 s0 = s[0], s1 = s[1], s2 = s[2];
    // three whole 16-byte rows: split into the fields each primitive kind
    // uses, they would take five loads through the texture path instead
    __asm__ volatile("" : : "v"(s0.x), "v"(s0.y), "v"(s0.z), "v"(s0.w), "v"(s1.x), "v"(s1.y), "v"(s1.z),
                     "v"(s1.w), "v"(s2.x), "v"(s2.y), "v"(s2.z), "v"(s2.w));
    const uint32_t prim = __float_as_uint(s0.w);
    float t = 0.0f;
    bool hit;
    if (__float_as_uint(s2.w) == kPrimTriangle)
      hit = hit_triangle(f.o, sh, V3{s0.x, s0.y, s0.z}, V3{s1.x, s1.y, s1.z}, V3{s2.x, s2.y, s2.z}, h.t, t);
    else
      hit = hit_sphere(f.o, f.d, V3{s0.x, s0.y, s0.z}, s1.x, h.t, t);
    // a hit has t <= h.t, so "t < h.t or a smaller key" is the tie rule;
    // the kept hit's primitive id is read back only on a tie
    if (hit) {
      bool take = t < h.t || inst < h.inst;
      if (!take && inst == h.inst) take = prim < slot_prim(sc.slots, h.slot);
      if (take) {
        h.t = t;
        h.slot = first + i;
        h.inst = inst;
      }
    }
  }
}

// compare-exchange of (entry distance, ref) pairs, ascending by distance
__device__ __forceinline__ void order2(float& ka, uint32_t& ra, float& kb, uint32_t& rb) {
  const bool sw = kb < ka;
  const float k = sw ? kb : ka;
  const uint32_t r = sw ? rb : ra;
  kb = sw ? ka : kb;
  rb = sw ? ra : rb;
  ka = k;
  ra = r;
}

// one child of a 4-wide node from its entry-plane (n) and exit-plane (f)
// coordinates: entry distance, or +inf when missed.  An empty child (box
// +inf / -inf) has an infinite entry distance on every axis and misses.
__device__ __forceinline__ float child_entry(const RayFrame& f, float nx, float fx, float ny, float fy, float nz,
                                             float fz, float lim) {
  const float tn = fmaxf(fmaxf(__builtin_fmaf(nx, f.ix, -f.ox_n), __builtin_fmaf(ny, f.iy, -f.oy_n)),
                         fmaxf(__builtin_fmaf(nz, f.iz, -f.oz_n), 0.0f));
  const float tf = fminf(fminf(__builtin_fmaf(fx, f.ix, -f.ox_f), __builtin_fmaf(fy, f.iy, -f.oy_f)),
                         fminf(__builtin_fmaf(fz, f.iz, -f.oz_f), lim)) * kSlabSlack;
  return tn <= tf ? tn : __builtin_inff();
}

// One 4-wide node at byte offset `off` from `base` (32-bit offsets: the
// loads take the scalar-base + vector-offset form): the children the ray
// enters, nearest first in `ref`, the others pushed far to near.  Returns
// false when no child is entered.
template <class S>
__device__ __forceinline__ bool visit4(const char* base, uint32_t off, const RayFrame& f, float lim, S& st, int& sp,
                                       uint32_t& ref) {
  auto row = [&](uint32_t o) { return *reinterpret_cast<const float4*>(base + o); };
  const float4 nx = row(off + f.near_x), fx = row(off + (16u - f.near_x));
  const float4 ny = row(off + f.near_y), fy = row(off + (80u - f.near_y));
  const float4 nz = row(off + f.near_z), fz = row(off + (144u - f.near_z));
  const float4 rf = row(off + 96u);
  uint32_t r0 = __float_as_uint(rf.x), r1 = __float_as_uint(rf.y), r2 = __float_as_uint(rf.z),
           r3 = __float_as_uint(rf.w);
  float k0 = child_entry(f, nx.x, fx.x, ny.x, fy.x, nz.x, fz.x, lim);
  float k1 = child_entry(f, nx.y, fx.y, ny.y, fy.y, nz.y, fz.y, lim);
  float k2 = child_entry(f, nx.z, fx.z, ny.z, fy.z, nz.z, fz.z, lim);
  float k3 = child_entry(f, nx.w, fx.w, ny.w, fy.w, nz.w, fz.w, lim);
  order2(k0, r0, k1, r1);
  order2(k2, r2, k3, r3);
  order2(k0, r0, k2, r2);
  order2(k1, r1, k3, r3);
  order2(k1, r1, k2, r2);
  // the child refs are fetched with the boxes, not after the test
  __asm__ volatile("" : : "v"(r0), "v"(r1), "v"(r2), "v"(r3));
  const float inf = __builtin_inff();
  if (!(k0 < inf)) return false;
  // the entered children are a prefix of the sorted four
  st.push3(sp, r3, k3 < inf, r2, k2 < inf, r1, k1 < inf);
  ref = r0;
  return true;
}

// One 4-wide node with binary16 extents (kNode4HalfFloat4s layout).  A
// child's upper plane on an axis is the FP32 sum lo + ext, which the builder
// made >= the true plane; it is the entry plane where the direction is
// negative and the exit plane otherwise.  Both planes are formed as
// fma(ext, w, lo) with per-ray weights w in {0, 1} (fma(ext, 1, lo) is that
// rounded sum, fma(ext, 0, lo) is lo), so no per-child select is needed; the
// weights are binary16 halves of one register per axis, set once per ray.
// Empty children (lo = +inf, ext = 0) miss as in visit4.
template <class S>
__device__ __forceinline__ bool visit4h(const char* base, uint32_t off, const RayFrame& f, float lim, S& st,
                                        int& sp, uint32_t& ref) {
  const float4 lx = *reinterpret_cast<const float4*>(base + off);
  const float4 ly = *reinterpret_cast<const float4*>(base + off + 16u);
  const float4 lz = *reinterpret_cast<const float4*>(base + off + 32u);
  const uint4 exy = *reinterpret_cast<const uint4*>(base + off + 48u);
  const uint4 ezr = *reinterpret_cast<const uint4*>(base + off + 64u);
  const float4 rf = *reinterpret_cast<const float4*>(base + off + 80u);
  uint32_t r0 = __float_as_uint(rf.x), r1 = __float_as_uint(rf.y), r2 = __float_as_uint(rf.z),
           r3 = __float_as_uint(rf.w);
  auto lo16 = [](uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu)); };
  auto hi16 = [](uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16)); };
  const float wnx = lo16(f.wx), wny = lo16(f.wy), wnz = lo16(f.wz);
  const float wfx = hi16(f.wx), wfy = hi16(f.wy), wfz = hi16(f.wz);
  auto child = [&](float lox, float ex, float loy, float ey, float loz, float ez) {
    return child_entry(f, __builtin_fmaf(ex, wnx, lox), __builtin_fmaf(ex, wfx, lox), __builtin_fmaf(ey, wny, loy),
                       __builtin_fmaf(ey, wfy, loy), __builtin_fmaf(ez, wnz, loz), __builtin_fmaf(ez, wfz, loz), lim);
  };
  float k0 = child(lx.x, lo16(exy.x), ly.x, lo16(exy.z), lz.x, lo16(ezr.x));
  float k1 = child(lx.y, hi16(exy.x), ly.y, hi16(exy.z), lz.y, hi16(ezr.x));
  float k2 = child(lx.z, lo16(exy.y), ly.z, lo16(exy.w), lz.z, lo16(ezr.y));
  float k3 = child(lx.w, hi16(exy.y), ly.w, hi16(exy.w), lz.w, hi16(ezr.y));
  order2(k0, r0, k1, r1);
  order2(k2, r2, k3, r3);
  order2(k0, r0, k2, r2);
  order2(k1, r1, k3, r3);
  order2(k1, r1, k2, r2);
  __asm__ volatile("" : : "v"(r0), "v"(r1), "v"(r2), "v"(r3));
  const float inf = __builtin_inff();
  if (!(k0 < inf)) return false;
  st.push3(sp, r3, k3 < inf, r2, k2 < inf, r1, k1 < inf);
  ref = r0;
  return true;
}

// One 4-wide node with binary16 planes on an FP32 corner (kNode4CornerFloat4s
// layout): a plane is the FP32 sum corner + q, formed by one mixed-precision
// FMA exactly as the builder checked it.  The entry-plane and exit-plane
// words of an axis (lower planes where the direction is >= 0, else upper)
// are picked per ray with the frame's masks, one bit-select per word.
// Empty children (lo = +inf, hi = 0) miss on any direction.
template <class S>
__device__ __forceinline__ bool visit4c(const char* base, uint32_t off, const RayFrame& f, float lim, S& st,
                                        int& sp, uint32_t& ref) {
  const float4 cn = *reinterpret_cast<const float4*>(base + off);
  const uint4 qx = *reinterpret_cast<const uint4*>(base + off + 16u);
  const uint4 qy = *reinterpret_cast<const uint4*>(base + off + 32u);
  const uint4 qz = *reinterpret_cast<const uint4*>(base + off + 48u);
  const float4 rf = *reinterpret_cast<const float4*>(base + off + 64u);
  uint32_t r0 = __float_as_uint(rf.x), r1 = __float_as_uint(rf.y), r2 = __float_as_uint(rf.z),
           r3 = __float_as_uint(rf.w);
  auto pick = [](uint32_t m, uint32_t a, uint32_t b) { return (a & m) | (b & ~m); };
  const uint32_t nx01 = pick(f.mx, qx.x, qx.z), nx23 = pick(f.mx, qx.y, qx.w);
  const uint32_t fx01 = pick(f.mx, qx.z, qx.x), fx23 = pick(f.mx, qx.w, qx.y);
  const uint32_t ny01 = pick(f.my, qy.x, qy.z), ny23 = pick(f.my, qy.y, qy.w);
  const uint32_t fy01 = pick(f.my, qy.z, qy.x), fy23 = pick(f.my, qy.w, qy.y);
  const uint32_t nz01 = pick(f.mz, qz.x, qz.z), nz23 = pick(f.mz, qz.y, qz.w);
  const uint32_t fz01 = pick(f.mz, qz.z, qz.x), fz23 = pick(f.mz, qz.w, qz.y);
  auto lo16 = [](uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu)); };
  auto hi16 = [](uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16)); };
  // 1.0 in a scalar register the compiler cannot see through: an FMA by a
  // known 1.0 would become a conversion and an add, two instructions where
  // v_fma_mix_f32 reads the binary16 operand directly
  float one = 1.0f;
  __asm__("" : "+s"(one));
  auto plane = [one](float q, float c) { return __builtin_fmaf(q, one, c); };
  auto child = [&](float nx, float fx, float ny, float fy, float nz, float fz) {
    return child_entry(f, plane(nx, cn.x), plane(fx, cn.x), plane(ny, cn.y), plane(fy, cn.y), plane(nz, cn.z),
                       plane(fz, cn.z), lim);
  };
  float k0 = child(lo16(nx01), lo16(fx01), lo16(ny01), lo16(fy01), lo16(nz01), lo16(fz01));
  float k1 = child(hi16(nx01), hi16(fx01), hi16(ny01), hi16(fy01), hi16(nz01), hi16(fz01));
  float k2 = child(lo16(nx23), lo16(fx23), lo16(ny23), lo16(fy23), lo16(nz23), lo16(fz23));
  float k3 = child(hi16(nx23), hi16(fx23), hi16(ny23), hi16(fy23), hi16(nz23), hi16(fz23));
  order2(k0, r0, k1, r1);
  order2(k2, r2, k3, r3);
  order2(k0, r0, k2, r2);
  order2(k1, r1, k3, r3);
  order2(k1, r1, k2, r2);
  __asm__ volatile("" : : "v"(r0), "v"(r1), "v"(r2), "v"(r3));
  const float inf = __builtin_inff();
  if (!(k0 < inf)) return false;
  st.push3(sp, r3, k3 < inf, r2, k2 < inf, r1, k1 < inf);
  ref = r0;
  return true;
}

// One 4-wide node with 8-bit child planes (kNode4Q8Float4s layout): per
// axis the entry and exit plane words are chosen once per ray from the
// direction sign, and child c's plane is fma(q_c, 2^e, origin), the FP32
// value the builder checked.  An empty child (qlo 255 > qhi 0) has an
// inverted box, which a far-away tiny node's slack could still accept, so
// it is also dropped by its ref.
template <class S>
__device__ __forceinline__ bool visit4q(const char* base, uint32_t off, const RayFrame& f, float lim, S& st,
                                        int& sp, uint32_t& ref) {
  const float4 q0 = *reinterpret_cast<const float4*>(base + off);
  const uint4 q1 = *reinterpret_cast<const uint4*>(base + off + 16u);
  const uint4 q2 = *reinterpret_cast<const uint4*>(base + off + 32u);
  const float4 rf = *reinterpret_cast<const float4*>(base + off + 48u);
  uint32_t r0 = __float_as_uint(rf.x), r1 = __float_as_uint(rf.y), r2 = __float_as_uint(rf.z),
           r3 = __float_as_uint(rf.w);
  const uint32_t eb = __float_as_uint(q0.w);
  const float sx = ldexpf(1.0f, (int)(eb & 255u) - 128), sy = ldexpf(1.0f, (int)((eb >> 8) & 255u) - 128),
              sz = ldexpf(1.0f, (int)((eb >> 16) & 255u) - 128);
  const bool px = f.ix >= 0.0f, py = f.iy >= 0.0f, pz = f.iz >= 0.0f;
  const uint32_t nx = px ? q1.x : q1.y, fx = px ? q1.y : q1.x;
  const uint32_t ny = py ? q1.z : q1.w, fy = py ? q1.w : q1.z;
  const uint32_t nz = pz ? q2.x : q2.y, fz = pz ? q2.y : q2.x;
  auto plane = [](uint32_t w, int c, float s, float o) {
    return __builtin_fmaf((float)((w >> (8 * c)) & 255u), s, o);
  };
  auto child = [&](int c) {
    return child_entry(f, plane(nx, c, sx, q0.x), plane(fx, c, sx, q0.x), plane(ny, c, sy, q0.y),
                       plane(fy, c, sy, q0.y), plane(nz, c, sz, q0.z), plane(fz, c, sz, q0.z), lim);
  };
  const float inf = __builtin_inff();
  float k0 = child(0), k1 = child(1), k2 = child(2), k3 = child(3);
  k1 = r1 == kEmptyChild ? inf : k1;
  k2 = r2 == kEmptyChild ? inf : k2;
  k3 = r3 == kEmptyChild ? inf : k3;
  order2(k0, r0, k1, r1);
  order2(k2, r2, k3, r3);
  order2(k0, r0, k2, r2);
  order2(k1, r1, k3, r3);
  order2(k1, r1, k2, r2);
  __asm__ volatile("" : : "v"(r0), "v"(r1), "v"(r2), "v"(r3));
  if (!(k0 < inf)) return false;
  st.push3(sp, r3, k3 < inf, r2, k2 < inf, r1, k1 < inf);
  ref = r0;
  return true;
}

// Tree kinds of the traversal (the kWidth template argument): widths 2 and
// 4 of one-level trees, the instanced (two-level, 4-wide) traversal, and
// the 4-wide kinds with binary16-extent, 8-bit and binary16-corner nodes.
constexpr int kTwoLevel = 1;
constexpr int kTwoLevelHalf = 3;
constexpr int kHalf4 = 5;
constexpr int kQ84 = 6;
constexpr int kTwoLevelQ8 = 7;
constexpr int kCorner4 = 8;
constexpr int kTwoLevelCorner = 9;
__host__ __device__ constexpr bool is_two_level(int w) {
  return w == kTwoLevel || w == kTwoLevelHalf || w == kTwoLevelQ8 || w == kTwoLevelCorner;
}
__host__ __device__ constexpr bool half_nodes(int w) { return w == kHalf4 || w == kTwoLevelHalf; }
__host__ __device__ constexpr bool q8_nodes(int w) { return w == kQ84 || w == kTwoLevelQ8; }
__host__ __device__ constexpr bool corner_nodes(int w) { return w == kCorner4 || w == kTwoLevelCorner; }

// The world ray of a two-level traversal waits in LDS (six values per lane,
// stride kStride) rather than in registers: it is needed only when an
// instance is entered or left.  The reads go through an address the
// compiler cannot see through (an empty asm statement), so it neither keeps
// a register copy across the traversal nor serialises the six reads.
template <int kStride>
struct WorldRay {
  lds_f32* p;
  __device__ __forceinline__ void store(V3 o, V3 d) const {
    p[0] = o.x; p[kStride] = o.y; p[2 * kStride] = o.z;
    p[3 * kStride] = d.x; p[4 * kStride] = d.y; p[5 * kStride] = d.z;
  }
  __device__ __forceinline__ void load(V3& o, V3& d) const {
    lds_f32* v = p;
    __asm__ volatile("" : "+v"(v));
    o = V3{v[0], v[kStride], v[2 * kStride]};
    d = V3{v[3 * kStride], v[4 * kStride], v[5 * kStride]};
  }
};

// Traversal state of one ray, advanced one node or leaf at a time so that
// a lane can take a new ray while others in its wave still traverse.
// Two-level scenes: mark is the stack height at which the current
// instance's bottom tree began (kInTopTree in the top tree), inst its id.
// Top-tree leaves are instances: entering one moves the ray into object
// space; once the stack is back at the mark the world ray returns.  Both
// frame changes happen in trav_frame, the only place that rewrites the ray
// frame after trav_begin: node and leaf steps leave it alone (a bottom tree
// that is done sets mark to kLeavePending), so the compiler keeps the
// frame's twenty-odd registers in place across steps instead of copying
// them at every join of the node and leaf paths.
constexpr int kInTopTree = -1;
constexpr int kLeavePending = -2;
struct Trav {
  RayFrame f;
  Hit h;
  uint32_t ref;
  int sp;
  int mark;
  uint32_t inst;
};

// Starts a traversal at the root; false when the scene has no geometry
// (the ray then misses).  Two-level callers store (o, d) in their WorldRay.
__device__ __forceinline__ bool trav_begin(const SceneView& sc, V3 o, V3 d, Trav& tv) {
  tv.h = Hit{__builtin_inff(), kMiss, kMiss};
  tv.ref = 0;
  tv.sp = 0;
  tv.mark = kInTopTree;
  tv.inst = 0;
  tv.f = make_frame(o, d);
  return sc.has_geometry != 0;
}

// After a node without an entered child or a tested leaf: the next
// deferred entry (a bottom tree that is done leaves the world frame to
// trav_frame).  Returns false once the stack is empty.
template <int kWidth, class S>
__device__ __forceinline__ bool trav_pop(S& st, Trav& tv) {
  if constexpr (is_two_level(kWidth)) {
    if (tv.sp == tv.mark) tv.mark = kLeavePending;
  }
  if (tv.sp == 0) return false;
  tv.ref = st.pop(tv.sp);
  return true;
}

// True when the next step of a two-level traversal is a frame change: a
// bottom tree is done, or the ray is at a top-tree leaf.  Such lanes wait
// with the lanes at leaves and change frames in leaf steps, so that the
// change's code (six divisions on entry) runs for many lanes at once.
template <int kWidth>
__device__ __forceinline__ bool needs_frame(const Trav& tv) {
  if constexpr (is_two_level(kWidth))
    return tv.mark == kLeavePending || (tv.mark == kInTopTree && (tv.ref & kLeafBit) != 0u);
  return false;
}

// The frame change needs_frame asks for: back to the world ray when a
// bottom tree is done, and into object space when the ray is at a top-tree
// leaf (its instance entered; the bottom tree's root becomes tv.ref).  Both
// at once when the entry popped after a finished bottom tree is another
// instance.
template <int kWidth, int kStride>
__device__ __forceinline__ void trav_frame(const SceneView& sc, const WorldRay<kStride>& wr, Trav& tv) {
  if constexpr (is_two_level(kWidth)) {
    if (tv.mark == kLeavePending) tv.mark = kInTopTree;
    const bool enter = tv.mark == kInTopTree && (tv.ref & kLeafBit) != 0u;
    {
      V3 o, d;
      wr.load(o, d);
      if (enter) {
        const uint32_t k = (tv.ref >> 3) & 0x0FFFFFFFu;
        const float4 r0 = sc.instances[2 * (size_t)k], r1 = sc.instances[2 * (size_t)k + 1];
        const float r = r1.z;  // 1 / scale, rounded to FP32 on the host
        o = V3{(o.x - r0.x) * r, (o.y - r0.y) * r, (o.z - r0.z) * r};
        d = V3{d.x * r, d.y * r, d.z * r};
        tv.inst = __float_as_uint(r1.y);
        tv.ref = __float_as_uint(r1.x);
        tv.mark = tv.sp;
      }
      tv.f = make_frame(o, d);
    }
  }
}

// Inner node tv.ref: the children the ray enters are pushed far to near and
// the nearest taken; with none, a pop.  Returns false once the traversal is
// complete.  kCount: also count inner-node fetches; kLds: the first
// sc.lds_nodes nodes (the top levels in BFS order; of a two-level scene, its
// top tree's) are read from the LDS copy (FP32 and binary16-extent nodes).
template <int kWidth, bool kCount, bool kLds, class S>
__device__ __forceinline__ bool trav_node(const SceneView& sc, const float4* lds_nodes, S& st, Trav& tv,
                                          uint32_t& n_nodes) {
  if constexpr (kCount) ++n_nodes;
  const float lim = tv.h.t * 1.000001f;
  if constexpr (kWidth == 2) {
    float4 n0, n1, n2, n3;
    if (kLds && tv.ref < sc.lds_nodes) {
      const float4* p = lds_nodes + 4 * tv.ref;
      n0 = p[0]; n1 = p[1]; n2 = p[2]; n3 = p[3];
    } else {
      const float4* p = sc.nodes + 4 * (size_t)tv.ref;
      n0 = p[0]; n1 = p[1]; n2 = p[2]; n3 = p[3];
    }
    float lo0, hi0, lo1, hi1;
    slab(tv.f, n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, lim, lo0, hi0);
    slab(tv.f, n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, lim, lo1, hi1);
    const bool h0 = lo0 <= hi0, h1 = lo1 <= hi1;
    const uint32_t r0 = __float_as_uint(n3.x), r1 = __float_as_uint(n3.y);
    if (h0 && h1) {
      const bool near0 = lo0 <= lo1;
      st.push(tv.sp, near0 ? r1 : r0);
      tv.ref = near0 ? r0 : r1;
      return true;
    }
    if (h0 || h1) {
      tv.ref = h0 ? r0 : r1;
      return true;
    }
  } else if constexpr (half_nodes(kWidth)) {
    const uint32_t off = tv.ref * (kNode4HalfFloat4s * 16u);  // node arrays stay below 4 GiB
    bool entered;
    if (kLds && tv.ref < sc.lds_nodes)
      entered = visit4h(reinterpret_cast<const char*>(lds_nodes), off, tv.f, lim, st, tv.sp, tv.ref);
    else
      entered = visit4h(reinterpret_cast<const char*>(sc.nodes), off, tv.f, lim, st, tv.sp, tv.ref);
    if (entered) return true;
  } else if constexpr (q8_nodes(kWidth)) {
    const uint32_t off = tv.ref * (kNode4Q8Float4s * 16u);
    if (visit4q(reinterpret_cast<const char*>(sc.nodes), off, tv.f, lim, st, tv.sp, tv.ref)) return true;
  } else if constexpr (corner_nodes(kWidth)) {
    // ref * 80 (node arrays stay below 4 GiB) as ((ref << 2) + ref) << 4: two
    // full-rate instructions instead of a quarter-rate 32-bit multiply
    static_assert(kNode4CornerFloat4s * 16u == 80u, "binary16-corner nodes are 80 bytes");
    uint32_t four = tv.ref << 2;
    __asm__("" : "+v"(four));  // keeps the compiler from folding this back into a multiply
    const uint32_t off = (four + tv.ref) << 4;
    if (visit4c(reinterpret_cast<const char*>(sc.nodes), off, tv.f, lim, st, tv.sp, tv.ref)) return true;
  } else {
    bool entered;
    const uint32_t off = tv.ref * (kNode4Float4s * 16u);  // node arrays stay below 4 GiB
    if (kLds && kWidth == 4 && tv.ref < sc.lds_nodes)
      entered = visit4(reinterpret_cast<const char*>(lds_nodes), off, tv.f, lim, st, tv.sp, tv.ref);
    else
      entered = visit4(reinterpret_cast<const char*>(sc.nodes), off, tv.f, lim, st, tv.sp, tv.ref);
    if (entered) return true;
  }
  return trav_pop<kWidth>(st, tv);
}

// Leaf tv.ref (of a two-level scene: of a bottom tree, since trav_frame
// enters top-tree leaves): its primitives tested, then a pop.  Returns false
// once the traversal is complete.  kCount: also count primitive tests.
template <int kWidth, bool kCount, class S>
__device__ __forceinline__ bool trav_leaf(const SceneView& sc, S& st, Trav& tv, uint32_t& n_prims) {
  test_leaf<kCount>(sc, tv.f, tv.ref, is_two_level(kWidth) ? tv.inst : 0u, tv.h, &n_prims);
  return trav_pop<kWidth>(st, tv);
}

// Closest hit of one ray, traversed to completion (the first-hit kernel).
// A well-formed tree visits each node at most once per ray; kMaxVisits only
// guards against a malformed upload.
template <int kWidth, class S, int kStride>
__device__ __forceinline__ Hit trace_closest(const SceneView& sc, const float4* lds_nodes, S& st,
                                             const WorldRay<kStride>& wr, V3 o, V3 d) {
  Trav tv;
  uint32_t nn = 0, np = 0;
  if (!trav_begin(sc, o, d, tv)) return tv.h;
  for (uint32_t v = 0; v < kMaxVisits; ++v) {
    if (needs_frame<kWidth>(tv)) {
      trav_frame<kWidth>(sc, wr, tv);
      continue;
    }
    const bool more = (tv.ref & kLeafBit) == 0u ? trav_node<kWidth, false, (kWidth == 2 || kWidth == 4 ||
                                                                              half_nodes(kWidth))>(sc, lds_nodes, st, tv, nn)
                                                : trav_leaf<kWidth, false>(sc, st, tv, np);
    if (!more) break;
  }
  return tv.h;
}

// geometric normal of a hit slot (unit for triangles; (p - c) / r for spheres)
__device__ __forceinline__ V3 slot_normal(const float4* slots, uint32_t slot, V3 p, uint32_t& material) {
  const float4* s = slots + 3 * (size_t)slot;
  const float4 s0 = s[0], s1 = s[1], s2 = s[2];
  // three whole rows (split by the fields each primitive kind uses, they
  // would take six loads)
  __asm__ volatile("" : : "v"(s0.x), "v"(s0.y), "v"(s0.z), "v"(s0.w), "v"(s1.x), "v"(s1.y), "v"(s1.z),
                   "v"(s1.w), "v"(s2.x), "v"(s2.y), "v"(s2.z), "v"(s2.w));
  material = __float_as_uint(s1.w);
  if (__float_as_uint(s2.w) == kPrimTriangle) {
    const V3 p0{s0.x, s0.y, s0.z};
    return normalized(cross(sub(V3{s1.x, s1.y, s1.z}, p0), sub(V3{s2.x, s2.y, s2.z}, p0)));
  }
  return V3{(p.x - s0.x) / s1.x, (p.y - s0.y) / s1.x, (p.z - s0.z) / s1.x};
}

__device__ __forceinline__ void stage_lds_nodes(const SceneView& sc, float4* lds) {
  for (uint32_t i = threadIdx.x; i < sc.node_float4s * sc.lds_nodes; i += blockDim.x) lds[i] = sc.nodes[i];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// generate: one camera ray per path slot of the pass
// ---------------------------------------------------------------------------
// Queue position -> pixel, in 8 x 8 tiles (bands of 8 rows, 8-column tiles
// within a band; the last band and tile of a row may be narrower), so the 64
// camera rays of a wave cover a compact block of the image.  A bijection on
// [0, W*H); the path's identity (pixel, sample) is what the random numbers
// and the accumulation use, so the order changes no result.
__device__ __forceinline__ void tile_pixel(uint32_t p, uint32_t W, uint32_t H, uint32_t& x, uint32_t& y) {
  const uint32_t full_bands = H / 8u, band_px = 8u * W;
  uint32_t band, hb, q;
  if (p < full_bands * band_px) {
    band = p / band_px;
    hb = 8u;
    q = p - band * band_px;
  } else {
    band = full_bands;
    hb = H - 8u * full_bands;
    q = p - full_bands * band_px;
  }
  const uint32_t tile_px = 8u * hb, full_tiles = W / 8u;
  if (q < full_tiles * tile_px) {
    const uint32_t t = q / tile_px, r = q - t * tile_px;
    x = 8u * t + (r & 7u);
    y = 8u * band + (r >> 3);
  } else {
    const uint32_t wt = W - 8u * full_tiles, r = q - full_tiles * tile_px;
    x = 8u * full_tiles + r % wt;
    y = 8u * band + r / wt;
  }
}

__global__ __launch_bounds__(256) void k_generate(CameraView cam, PassView pv, RayQueue q, float4* L) {
  const uint32_t n = pv.pixels * pv.samples;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t s = i / pv.pixels;
    uint32_t x, y;
    tile_pixel(i - s * pv.pixels, pv.width, pv.height, x, y);
    const uint32_t pixel = y * pv.width + x;
    const uint32_t sample = pv.sample0 + s;
    const U4 r = philox(pixel, sample, 0, kRngCamera, pv.key0, pv.key1);
    const V3 d = camera_direction(cam, pv.width, pv.height, x, y, unit_float(r.x), unit_float(r.y));
    q.o[i] = make_float4(cam.eye[0], cam.eye[1], cam.eye[2], __uint_as_float(pixel));
    q.d[i] = make_float4(d.x, d.y, d.z, __uint_as_float(sample));
    q.b[i] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    L[s * pv.pixels + pixel] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

__global__ void k_pass_init(uint32_t* cnt, uint32_t paths) {
  for (int i = threadIdx.x; i < kCntWords; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) cnt[kCntRays + 1] = paths;
}

// ---------------------------------------------------------------------------
// extend: closest hit of every ray entering depth `depth`, written to
// hits[i] = (t, slot, instance) for queue entry i.  Lanes advance their own
// traversals one step at a time; once no more than kRefillAt lanes of a
// wave still traverse, the idle ones take new rays from a per-wave pool of
// 64 queue entries (one atomic per pool), so lanes whose rays finish early
// do not wait for the slowest ray of their wave.
// ---------------------------------------------------------------------------
template <int kWidth, int kStack, bool kCount, bool kLds>
// Six waves per SIMD (at most 80 VGPRs): the extra waves hide texture-cache
// latency; measured 11 % faster on the large-BVH scene than the five the
// unconstrained allocation allows, seven spills too much.
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(NPT_EXTEND_WAVES))) void k_extend(SceneView sc, uint32_t depth, RayQueue in, float4* hits,
                                                        uint32_t* cnt, unsigned long long* visit_cnt,
                                                        const uint32_t* order) {
  extern __shared__ float4 lds_nodes[];
  using Stack = LaneStack<kStack, kTraceBlock>;
  __shared__ uint32_t stack_mem[(Stack::kShort > 0 ? Stack::kShort : 1) * kTraceBlock];
  __shared__ float world_mem[(is_two_level(kWidth) ? 6 : 1) * kTraceBlock];
  Stack st;
  st.lds = (lds_u32*)(stack_mem + threadIdx.x);
  const WorldRay<kTraceBlock> wr{(lds_f32*)(world_mem + threadIdx.x)};
  // the grid is sized for the largest possible queue; workgroups beyond the
  // actual ray count leave before any staging or atomic (the others drain
  // the whole queue)
  const uint32_t n = cnt[kCntRays + depth];
  if ((uint64_t)blockIdx.x * kTraceBlock >= n) return;
  if constexpr (kLds) stage_lds_nodes(sc, lds_nodes);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t* work = &cnt[kCntWork + depth];
  uint32_t n_nodes = 0, n_prims = 0;
  Trav tv;
  uint32_t ray = 0, steps = 0;
  bool busy = false;
  uint32_t pool = 0, pool_end = 0;  // this wave's unclaimed queue entries
  bool drained = false;             // the queue has no entries left
  for (;;) {
    // hand queued rays to the idle lanes, lowest lane first
    uint64_t idle = lanes(!busy);
    while (idle != 0 && !drained) {
      if (pool == pool_end) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(work, (uint32_t)kWave);
        b = __builtin_amdgcn_readfirstlane(b);  // wave-uniform: the pool bounds live in SGPRs
        if (b >= n) {
          drained = true;
          break;
        }
        pool = b;
        pool_end = min(b + (uint32_t)kWave, n);
      }
      const uint32_t rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
      const uint32_t take = min(pool_end - pool, (uint32_t)__popcll(idle));
      if (!busy && rank < take) {
        ray = order ? order[pool + rank] : pool + rank;  // queue slot of the ray
        const float* qo = reinterpret_cast<const float*>(in.o + ray);
        const float* qd = reinterpret_cast<const float*>(in.d + ray);
        const V3 o{qo[0], qo[1], qo[2]}, d{qd[0], qd[1], qd[2]};
        if constexpr (is_two_level(kWidth)) wr.store(o, d);
        busy = trav_begin(sc, o, d, tv);
        steps = 0;
        if (!busy) hits[ray] = make_float4(tv.h.t, __uint_as_float(kMiss), __uint_as_float(kMiss), 0.0f);
      }
      pool += take;
      idle = lanes(!busy);
    }
    if (lanes(busy) == 0) break;
    // advance until few lanes still traverse (none, once the queue is
    // drained).  Each wave step is either a node step (the lanes at inner
    // nodes visit them) or a leaf step (the lanes at leaves test them; the
    // lanes that enter or leave an instance change frames), never both, so
    // that node and leaf code do not diverge within a step.  A leaf step is
    // taken once the lanes waiting at leaves or for a frame change reach
    // kLeafPercent % of the lanes at inner nodes: waiting for every lane to
    // reach a leaf would leave most lanes idle through the long node
    // sequences of the wave's slowest rays.
    const uint32_t floor_busy = drained ? 0u : (uint32_t)kRefillAt;
    for (;;) {
      const bool at_node = busy && (tv.ref & kLeafBit) == 0u && !needs_frame<kWidth>(tv);
      uint32_t nn = (uint32_t)__popcll(lanes(at_node));
      uint32_t nl = (uint32_t)__popcll(lanes(busy && !at_node));
      // 32-bit scalars the compiler cannot widen again: it would compare
      // the 64-bit popcounts on the vector unit (no scalar 64-bit ordered
      // compare), two vector instructions per use
      __asm__("" : "+s"(nn), "+s"(nl));
      if (nn + nl <= floor_busy) break;
      bool more = true;
      // counts of at most 64 lanes: 32-bit products, a scalar compare
      const bool leaf_step = 100u * nl >= kLeafPercent * nn;
      // frame changes first, ahead of the leaf / node branch: the frame is
      // then rewritten in one place only, which keeps its registers in place
      const bool change = leaf_step && busy && needs_frame<kWidth>(tv);
      if (change) trav_frame<kWidth>(sc, wr, tv);
      if (leaf_step) {
        if (busy && !at_node && !change) {
          more = trav_leaf<kWidth, kCount>(sc, st, tv, n_prims);
          if (++steps >= kMaxVisits) more = false;
        }
      } else if (at_node) {
        more = trav_node<kWidth, kCount, kLds>(sc, lds_nodes, st, tv, n_nodes);
        if (++steps >= kMaxVisits) more = false;
      }
      if (busy && !more) {
        hits[ray] = make_float4(tv.h.t, __uint_as_float(tv.h.slot), __uint_as_float(tv.h.inst), 0.0f);
        busy = false;
      }
    }
  }
  if constexpr (kCount) {
    atomicAdd(&visit_cnt[depth - 1], (unsigned long long)n_nodes);
    atomicAdd(&visit_cnt[64 + depth - 1], (unsigned long long)n_prims);
  }
}

// ---------------------------------------------------------------------------
// ray order (optional): every chunk of kSortChunk queued rays is sorted by a
// key of direction octant (3 bits), origin (Morton code of a 32^3 grid over
// the scene bounds, 15 bits) and direction (|d.x|, |d.y| in quarters, 4
// bits), ties by queue slot; the extend kernel then takes the chunk's rays
// in that order through `order` and writes each hit to the ray's own slot.
// ---------------------------------------------------------------------------
constexpr int kSortChunk = 1024, kSortBlock = 256;

__device__ __forceinline__ uint32_t spread5(uint32_t x) {  // bit i -> bit 3 i
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) r |= ((x >> i) & 1u) << (3 * i);
  return r;
}

__device__ __forceinline__ uint32_t grid5(float x, float lo, float scale) {
  return (uint32_t)fminf(fmaxf((x - lo) * scale, 0.0f), 31.0f);
}

__global__ __launch_bounds__(kSortBlock) void k_sort_chunks(RayQueue in, const uint32_t* cnt, uint32_t depth,
                                                           float3 lo, float3 scale, uint32_t* order) {
  __shared__ uint32_t key[kSortChunk];
  const uint32_t n = cnt[kCntRays + depth];
  const uint32_t base = blockIdx.x * kSortChunk;
  if (base >= n) return;
  for (int i = threadIdx.x; i < kSortChunk; i += kSortBlock) {
    const uint32_t r = base + i;
    uint32_t k = 0x3FFFFFu;  // past the queue's end: last (ties go by slot)
    if (r < n) {
      const float4 o = in.o[r], d = in.d[r];
      const uint32_t oct = (d.x < 0.0f ? 1u : 0u) | (d.y < 0.0f ? 2u : 0u) | (d.z < 0.0f ? 4u : 0u);
      const uint32_t m = spread5(grid5(o.x, lo.x, scale.x)) | (spread5(grid5(o.y, lo.y, scale.y)) << 1) |
                         (spread5(grid5(o.z, lo.z, scale.z)) << 2);
      const uint32_t dq = (min(3u, (uint32_t)(fabsf(d.x) * 4.0f)) << 2) | min(3u, (uint32_t)(fabsf(d.y) * 4.0f));
      k = (oct << 19) | (m << 4) | dq;
    }
    key[i] = (k << 10) | (uint32_t)i;
  }
  __syncthreads();
  // bitonic sort, ascending
  for (int k2 = 2; k2 <= kSortChunk; k2 <<= 1)
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kSortChunk / 2; t += kSortBlock) {
        const int i = (t / j) * 2 * j + t % j, l = i + j;
        const uint32_t a = key[i], b = key[l];
        if ((a > b) == ((i & k2) == 0)) {
          key[i] = b;
          key[l] = a;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < kSortChunk; i += kSortBlock)
    if (base + i < n) order[base + i] = base + (key[i] & (uint32_t)(kSortChunk - 1));
}

hipError_t launch_sort_chunks(const RayQueue& in, const uint32_t* cnt, uint32_t depth, uint64_t max_rays,
                              const float lo[3], const float hi[3], uint32_t* order, hipStream_t s) {
  float3 l3 = make_float3(lo[0], lo[1], lo[2]), sc3;
  const float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  sc3.x = ext[0] > 0.0f ? 32.0f / ext[0] : 0.0f;
  sc3.y = ext[1] > 0.0f ? 32.0f / ext[1] : 0.0f;
  sc3.z = ext[2] > 0.0f ? 32.0f / ext[2] : 0.0f;
  const uint64_t chunks = (max_rays + kSortChunk - 1) / kSortChunk;
  hipLaunchKernelGGL(k_sort_chunks, dim3((uint32_t)chunks), dim3(kSortBlock), 0, s, in, cnt, depth, l3, sc3, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shade: emission, BSDF sampling and roulette for every ray of depth
// `depth` from its hit record.  Escaped rays go to the environment queue;
// survivors to the next queue.  Whole workgroups iterate together: queue
// slots are reserved with one atomic per workgroup and queue.
// ---------------------------------------------------------------------------
// 512-thread workgroups, a grid of eight per CU (the same threads as four
// of 1024): on the large-BVH frame 1024 threads were 9 % slower and 256
// threads, with four times the queue-counter atomics of 1024, 53 % slower
constexpr int kShadeBlock = 512;

// Queue slots for two predicates at once: the wave counts meet in LDS and
// thread 0 reserves both ranges.  Every thread of the workgroup calls it.
__device__ __forceinline__ void block_append2(bool pa, uint32_t* ca, bool pb, uint32_t* cb, uint32_t& ia,
                                              uint32_t& ib) {
  constexpr int kWaves = kShadeBlock / kWave;
  __shared__ uint32_t off_a[kWaves], off_b[kWaves];
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t ma = __ballot(pa), mb = __ballot(pb);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    off_a[wave] = (uint32_t)__popcll(ma);
    off_b[wave] = (uint32_t)__popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sa = 0, sb = 0;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t a = off_a[w], b = off_b[w];
      off_a[w] = sa;
      off_b[w] = sb;
      sa += a;
      sb += b;
    }
    const uint32_t base_a = sa ? atomicAdd(ca, sa) : 0u, base_b = sb ? atomicAdd(cb, sb) : 0u;
    for (int w = 0; w < kWaves; ++w) {
      off_a[w] += base_a;
      off_b[w] += base_b;
    }
  }
  __syncthreads();
  ia = off_a[wave] + __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
  ib = off_b[wave] + __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
  __syncthreads();  // the offsets are rewritten by the next call
}

__global__ __launch_bounds__(kShadeBlock) void k_shade(SceneView sc, PassView pv, uint32_t depth, RayQueue in,
                                               const float4* hits, RayQueue out, EnvQueue env, float4* L,
                                               uint32_t* cnt) {
  const uint32_t n = cnt[kCntRays + depth];
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < n;
    V3 o{0, 0, 0}, d{0, 0, 1}, beta{0, 0, 0};
    uint32_t pixel = 0, sample = 0;
    Hit h{__builtin_inff(), kMiss, 0u};
    if (valid) {
      const float4 qo = in.o[i], qd = in.d[i], qb = in.b[i], hr = hits[i];
      o = V3{qo.x, qo.y, qo.z};
      d = V3{qd.x, qd.y, qd.z};
      beta = V3{qb.x, qb.y, qb.z};
      pixel = __float_as_uint(qo.w);
      sample = __float_as_uint(qd.w);
      h = Hit{hr.x, __float_as_uint(hr.y), __float_as_uint(hr.z)};
    }
    const uint32_t slot = (sample - pv.sample0) * pv.pixels + pixel;
    const bool escaped = valid && h.slot == kMiss;
    bool alive = false;
    V3 no{0, 0, 0}, nd{0, 0, 1};
    if (valid && !escaped) {
      const V3 p{o.x + h.t * d.x, o.y + h.t * d.y, o.z + h.t * d.z};
      uint32_t mat;
      const V3 n = slot_normal(sc.slots, h.slot, p, mat);
      const float4 m0 = sc.materials[2 * mat], m1 = sc.materials[2 * mat + 1];
      const float dn = dot(d, n);
      if (dn < 0.0f && (m1.x != 0.0f || m1.y != 0.0f || m1.z != 0.0f)) {
        float4 l = L[slot];
        l.x += beta.x * m1.x;
        l.y += beta.y * m1.y;
        l.z += beta.z * m1.z;
        L[slot] = l;
      }
      const uint32_t mtype = __float_as_uint(m0.w);
      alive = !(depth == pv.max_depth || mtype == kEmitter);
      if (alive) {
        const U4 r = philox(pixel, sample, depth, kRngScatter, pv.key0, pv.key1);
        if (mtype == kLambert) {
          const V3 nf = dn > 0.0f ? neg(n) : n;
          nd = sample_cosine(nf, unit_float(r.x), unit_float(r.y));
          beta = V3{beta.x * m0.x, beta.y * m0.y, beta.z * m0.z};
        } else if (mtype == kMirror) {
          const float k2 = 2.0f * dn;
          nd = V3{d.x - k2 * n.x, d.y - k2 * n.y, d.z - k2 * n.z};
          beta = V3{beta.x * m0.x, beta.y * m0.y, beta.z * m0.z};
        } else {
          nd = sample_dielectric(d, n, m1.w, unit_float(r.z));
        }
        if (depth >= pv.rr_start) {
          const float q = fminf(1.0f, fmaxf(fmaxf(beta.x, beta.y), beta.z));
          if (unit_float(r.w) >= q) {
            alive = false;
          } else {
            beta = V3{beta.x / q, beta.y / q, beta.z / q};
          }
        }
        if (alive) {
          const float sd = dot(nd, n);
          no = offset_origin(p, sd > 0.0f ? n : neg(n));
        }
      }
    }
    uint32_t ei, oi;
    block_append2(escaped, &cnt[kCntEnv + depth], alive, &cnt[kCntRays + depth + 1], ei, oi);
    if (escaped) {
      env.d[ei] = make_float4(d.x, d.y, d.z, __uint_as_float(slot));
      env.b[ei] = make_float4(beta.x, beta.y, beta.z, 0.0f);
    }
    if (alive) {
      out.o[oi] = make_float4(no.x, no.y, no.z, __uint_as_float(pixel));
      out.d[oi] = make_float4(nd.x, nd.y, nd.z, __uint_as_float(sample));
      out.b[oi] = make_float4(beta.x, beta.y, beta.z, 0.0f);
    }
  }
}

// ---------------------------------------------------------------------------
// environment: bilinear lookup of the equirect map
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_env_lookup(const float4* map, int W, int H, EnvQueue env,
                                                    float4* L, const uint32_t* cnt, uint32_t depth) {
  const uint32_t n = cnt[kCntEnv + depth];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float4 ed = env.d[i], eb = env.b[i];
    float u, v;
    direction_to_uv(V3{ed.x, ed.y, ed.z}, u, v);
    const float3 c = env_bilinear(map, W, H, u, v);
    const uint32_t slot = __float_as_uint(ed.w);
    float4 l = L[slot];
    l.x += eb.x * c.x;
    l.y += eb.y * c.y;
    l.z += eb.z * c.z;
    L[slot] = l;
  }
}

// direct queries (npt_env_query): dirs [n][3] -> rgb [n][3]
__global__ __launch_bounds__(256) void k_env_query_map(const float4* map, int W, int H, const float* dirs,
                                                       uint64_t n, float* rgb) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    float u, v;
    direction_to_uv(V3{dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]}, u, v);
    const float3 c = env_bilinear(map, W, H, u, v);
    rgb[3 * i] = c.x;
    rgb[3 * i + 1] = c.y;
    rgb[3 * i + 2] = c.z;
  }
}

// ---------------------------------------------------------------------------
// accumulate the pass's samples per pixel in sample order, then finalize
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accumulate(const float4* L, float4* accum, PassView pv, int first_pass) {
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < pv.pixels; p += gridDim.x * blockDim.x) {
    float4 a = first_pass ? make_float4(0, 0, 0, 0) : accum[p];
    for (uint32_t s = 0; s < pv.samples; ++s) {
      const float4 l = L[(size_t)s * pv.pixels + p];
      a.x += l.x;
      a.y += l.y;
      a.z += l.z;
    }
    accum[p] = a;
  }
}

__global__ __launch_bounds__(256) void k_finalize(const float4* accum, float* out, uint32_t pixels, float inv_spp) {
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < pixels; p += gridDim.x * blockDim.x) {
    const float4 a = accum[p];
    out[3 * (size_t)p] = a.x * inv_spp;
    out[3 * (size_t)p + 1] = a.y * inv_spp;
    out[3 * (size_t)p + 2] = a.z * inv_spp;
  }
}

// ---------------------------------------------------------------------------
// primary hits (Table 3-style checks)
// ---------------------------------------------------------------------------
template <int kWidth, int kStack>
__global__ __launch_bounds__(kTraceBlock) void k_trace_primary(SceneView sc, CameraView cam, PassView pv,
                                                               uint32_t* prim, uint32_t* inst, float* tout,
                                                               float* normal) {
  extern __shared__ float4 lds_nodes[];
  using Stack = LaneStack<kStack, kTraceBlock>;
  __shared__ uint32_t stack_mem[(Stack::kShort > 0 ? Stack::kShort : 1) * kTraceBlock];
  stage_lds_nodes(sc, lds_nodes);
  __shared__ float world_mem[(is_two_level(kWidth) ? 6 : 1) * kTraceBlock];
  Stack st;
  st.lds = (lds_u32*)(stack_mem + threadIdx.x);
  const WorldRay<kTraceBlock> wr{(lds_f32*)(world_mem + threadIdx.x)};
  const uint32_t nblocks = (pv.pixels + kTraceBlock - 1) / kTraceBlock;
  for (uint32_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const uint32_t pixel = b * kTraceBlock + threadIdx.x;
    if (pixel >= pv.pixels) continue;
    const uint32_t x = pixel % pv.width, y = pixel / pv.width;
    const U4 r = philox(pixel, pv.sample0, 0, kRngCamera, pv.key0, pv.key1);
    const V3 d = camera_direction(cam, pv.width, pv.height, x, y, unit_float(r.x), unit_float(r.y));
    const V3 o{cam.eye[0], cam.eye[1], cam.eye[2]};
    if constexpr (is_two_level(kWidth)) wr.store(o, d);
    const Hit h = trace_closest<kWidth>(sc, lds_nodes, st, wr, o, d);
    V3 n{0, 0, 0};
    if (h.slot != kMiss) {
      uint32_t mat;
      n = slot_normal(sc.slots, h.slot, V3{o.x + h.t * d.x, o.y + h.t * d.y, o.z + h.t * d.z}, mat);
    }
    if (prim) prim[pixel] = h.slot == kMiss ? kMiss : slot_prim(sc.slots, h.slot);
    if (inst) inst[pixel] = h.slot == kMiss ? kMiss : h.inst;
    if (tout) tout[pixel] = h.t;
    if (normal) {
      normal[3 * (size_t)pixel] = n.x;
      normal[3 * (size_t)pixel + 1] = n.y;
      normal[3 * (size_t)pixel + 2] = n.z;
    }
  }
}

// per-depth counters summed over passes (npt_get_stats)
__global__ void k_stats_clear(unsigned long long* st) {
  for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) st[i] = 0ull;
}

__global__ void k_stats_add(const uint32_t* cnt, unsigned long long* st) {
  const int k = threadIdx.x;
  if (k < 64) {
    st[k] += cnt[kCntRays + k + 1];
    st[64 + k] += cnt[kCntEnv + k + 1];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_stats_clear(unsigned long long* st, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_clear, dim3(1), dim3(128), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_stats_add(const uint32_t* cnt, unsigned long long* st, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_add, dim3(1), dim3(64), 0, s, cnt, st);
  return hipGetLastError();
}

static int grid_for(uint64_t n, int block, int cap) {
  const uint64_t g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > (uint64_t)cap ? cap : g));
}

hipError_t launch_pass_init(uint32_t* cnt, uint32_t paths, hipStream_t s) {
  hipLaunchKernelGGL(k_pass_init, dim3(1), dim3(256), 0, s, cnt, paths);
  return hipGetLastError();
}

hipError_t launch_generate(const CameraView& cam, const PassView& pv, const RayQueue& q, float4* L,
                           hipStream_t s) {
  const uint64_t n = (uint64_t)pv.pixels * pv.samples;
  hipLaunchKernelGGL(k_generate, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, cam, pv, q, L);
  return hipGetLastError();
}

hipError_t launch_extend(int stack_depth, const SceneView& sc, uint32_t depth, uint64_t max_rays,
                         const RayQueue& in, float4* hits, uint32_t* cnt, unsigned long long* visit_cnt,
                         const uint32_t* order, int num_cus, hipStream_t s) {
  const size_t lds = (size_t)sc.lds_nodes * sc.node_float4s * sizeof(float4);
  const int grid = grid_for(max_rays, kTraceBlock, num_cus * 32);
#define NPT_LAUNCH_EXTEND(W, S, C, L)                                                                        \
  hipLaunchKernelGGL((k_extend<W, S, C, L>), dim3(grid), dim3(kTraceBlock), L ? lds : 0, s, sc, depth, in, hits, cnt, \
                     visit_cnt, order)
#define NPT_LAUNCH_EXTEND_S(W, L)                                                                        \
  switch (stack_depth) {                                                                                \
    case 16: if (c) NPT_LAUNCH_EXTEND(W, 16, true, L); else NPT_LAUNCH_EXTEND(W, 16, false, L); break;    \
    case 32: if (c) NPT_LAUNCH_EXTEND(W, 32, true, L); else NPT_LAUNCH_EXTEND(W, 32, false, L); break;    \
    case 64: if (c) NPT_LAUNCH_EXTEND(W, 64, true, L); else NPT_LAUNCH_EXTEND(W, 64, false, L); break;    \
    case 128: if (c) NPT_LAUNCH_EXTEND(W, 128, true, L); else NPT_LAUNCH_EXTEND(W, 128, false, L); break; \
    default: return hipErrorInvalidValue;                                                               \
  }
  const bool c = visit_cnt != nullptr;
  const bool staged = sc.lds_nodes > 0;
  // node formats of 4-wide trees (a binary node is also four float4 long)
  const bool half = sc.width == 4 && sc.node_float4s == kNode4HalfFloat4s;
  const bool q8 = sc.width == 4 && sc.node_float4s == kNode4Q8Float4s;
  const bool corner = sc.width == 4 && sc.node_float4s == kNode4CornerFloat4s;
  if (sc.two_level && corner) {
    NPT_LAUNCH_EXTEND_S(kTwoLevelCorner, false)
  } else if (corner) {
    NPT_LAUNCH_EXTEND_S(kCorner4, false)
  } else if (sc.two_level && half) {
    if (staged) {
      NPT_LAUNCH_EXTEND_S(kTwoLevelHalf, true)
    } else {
      NPT_LAUNCH_EXTEND_S(kTwoLevelHalf, false)
    }
  } else if (sc.two_level && q8) {
    NPT_LAUNCH_EXTEND_S(kTwoLevelQ8, false)
  } else if (sc.two_level) {
    NPT_LAUNCH_EXTEND_S(kTwoLevel, false)
  } else if (half) {
    if (staged) {
      NPT_LAUNCH_EXTEND_S(kHalf4, true)
    } else {
      NPT_LAUNCH_EXTEND_S(kHalf4, false)
    }
  } else if (q8) {
    NPT_LAUNCH_EXTEND_S(kQ84, false)
  } else if (sc.width == 4) {
    if (staged) {
      NPT_LAUNCH_EXTEND_S(4, true)
    } else {
      NPT_LAUNCH_EXTEND_S(4, false)
    }
  } else {
    if (staged) {
      NPT_LAUNCH_EXTEND_S(2, true)
    } else {
      NPT_LAUNCH_EXTEND_S(2, false)
    }
  }
#undef NPT_LAUNCH_EXTEND_S
#undef NPT_LAUNCH_EXTEND
  return hipGetLastError();
}

hipError_t launch_shade(const SceneView& sc, const PassView& pv, uint32_t depth, uint64_t max_rays,
                        const RayQueue& in, const float4* hits, const RayQueue& out, const EnvQueue& env,
                        float4* L, uint32_t* cnt, int num_cus, hipStream_t s) {
  hipLaunchKernelGGL(k_shade, dim3(grid_for(max_rays, kShadeBlock, num_cus * 8)), dim3(kShadeBlock), 0, s, sc, pv,
                     depth, in, hits, out, env, L, cnt);
  return hipGetLastError();
}

// smallest supported traversal stack holding `entries`
int trace_stack_size(uint32_t entries) {
  const int sizes[] = {16, 32, 64, 128};
  for (int v : sizes)
    if ((uint32_t)v >= entries) return v;
  return 0;
}

hipError_t launch_env_lookup(const float4* map, int W, int H, const EnvQueue& env, float4* L,
                             const uint32_t* cnt, uint32_t depth, uint64_t max_rays, int num_cus,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_env_lookup, dim3(grid_for(max_rays, 256, num_cus * 8)), dim3(256), 0, s, map, W, H,
                     env, L, cnt, depth);
  return hipGetLastError();
}

hipError_t launch_env_query_map(const float4* map, int W, int H, const float* dirs, uint64_t n, float* rgb,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_env_query_map, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, map, W, H, dirs, n, rgb);
  return hipGetLastError();
}

hipError_t launch_accumulate(const float4* L, float4* accum, const PassView& pv, int first_pass, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for(pv.pixels, 256, 65536)), dim3(256), 0, s, L, accum, pv,
                     first_pass);
  return hipGetLastError();
}

hipError_t launch_finalize(const float4* accum, float* out, uint32_t pixels, float inv_spp, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(pixels, 256, 65536)), dim3(256), 0, s, accum, out, pixels,
                     inv_spp);
  return hipGetLastError();
}

hipError_t launch_trace_primary(int stack_depth, const SceneView& sc, const CameraView& cam, const PassView& pv,
                                uint32_t* prim, uint32_t* inst, float* t, float* normal, int num_cus,
                                hipStream_t s) {
  const size_t lds = (size_t)sc.lds_nodes * sc.node_float4s * sizeof(float4);
  const int grid = grid_for(pv.pixels, kTraceBlock, num_cus * 16);
#define NPT_LAUNCH_PRIMARY(W, S)                                                                                   \
  hipLaunchKernelGGL((k_trace_primary<W, S>), dim3(grid), dim3(kTraceBlock), lds, s, sc, cam, pv, prim, inst, t, \
                     normal)
#define NPT_LAUNCH_PRIMARY_S(W)                  \
  if (stack_depth <= 32) NPT_LAUNCH_PRIMARY(W, 32);      \
  else if (stack_depth <= 64) NPT_LAUNCH_PRIMARY(W, 64); \
  else NPT_LAUNCH_PRIMARY(W, 128);
  if (stack_depth > 128) return hipErrorInvalidValue;
  // node formats of 4-wide trees (a binary node is also four float4 long)
  const bool half = sc.width == 4 && sc.node_float4s == kNode4HalfFloat4s;
  const bool q8 = sc.width == 4 && sc.node_float4s == kNode4Q8Float4s;
  const bool corner = sc.width == 4 && sc.node_float4s == kNode4CornerFloat4s;
  if (sc.two_level && corner) {
    NPT_LAUNCH_PRIMARY_S(kTwoLevelCorner)
  } else if (corner) {
    NPT_LAUNCH_PRIMARY_S(kCorner4)
  } else if (sc.two_level && half) {
    NPT_LAUNCH_PRIMARY_S(kTwoLevelHalf)
  } else if (sc.two_level && q8) {
    NPT_LAUNCH_PRIMARY_S(kTwoLevelQ8)
  } else if (sc.two_level) {
    NPT_LAUNCH_PRIMARY_S(kTwoLevel)
  } else if (half) {
    NPT_LAUNCH_PRIMARY_S(kHalf4)
  } else if (q8) {
    NPT_LAUNCH_PRIMARY_S(kQ84)
  } else if (sc.width == 4) {
    NPT_LAUNCH_PRIMARY_S(4)
  } else {
    NPT_LAUNCH_PRIMARY_S(2)
  }
#undef NPT_LAUNCH_PRIMARY_S
#undef NPT_LAUNCH_PRIMARY
  return hipGetLastError();
}

}  // namespace npt
