// npt_shared.h -- plain structs passed from the host library to its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace npt {

// BVH2 node, 64 bytes, both child boxes stored in the parent:
//   n0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   n1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   n2 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   n3 = (ref0, ref1, -, -) as uint bits
// ref: inner child = node index; leaf = kLeafBit | first_slot << 3 | (count-1).
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kMaxLeaf = 8;
constexpr uint32_t kMaxSlots = 1u << 28;
constexpr uint32_t kMaxLdsNodes = 255;
constexpr uint32_t kEmptyChild = 0x7FFFFFFFu;  // unused child of a 4-wide node

// BVH4 node, 112 bytes (7 float4), child boxes as structure of arrays:
//   n0 = lo.x of children 0..3, n1 = hi.x, n2 = lo.y, n3 = hi.y, n4 = lo.z,
//   n5 = hi.z, n6 = (ref0, ref1, ref2, ref3); empty children have ref
//   kEmptyChild and an inverted (+inf, -inf) box.  (Padding nodes to one
//   128-byte cache line was measured: no faster.)
constexpr uint32_t kNode4Float4s = 7;

// BVH4 node with binary16 extents (Sec. 3.1.4 proposes FP16 box extents),
// 96 bytes (6 float4):
//   h0 = lo.x of children 0..3, h1 = lo.y, h2 = lo.z (FP32),
//   h3 = (ext.x of children 0,1 | 2,3, ext.y 0,1 | 2,3), h4 = (ext.z 0,1 | 2,3, -, -)
//        as binary16 pairs (child 2k in the low half),
//   h5 = (ref0, ref1, ref2, ref3).
// The upper plane of a child is the FP32 sum lo + ext (rounded to nearest),
// which the builder checks to be >= the true upper plane.  Empty children
// have lo = +inf and ext = 0.
constexpr uint32_t kNode4HalfFloat4s = 6;

// BVH4 node with 8-bit child boxes (after Ylitie et al. 2017), 64 bytes:
//   q0 = (origin.x, origin.y, origin.z, step exponents e_x | e_y << 8 | e_z << 16, each + 128)
//   q1 = (qlo.x, qhi.x, qlo.y, qhi.y), q2 = (qlo.z, qhi.z, -, -): byte c of a
//        word is child c's plane, origin + q 2^e (the FP32 sum; q 2^e is exact)
//   q3 = (ref0, ref1, ref2, ref3)
// The builder rounds lower planes down and upper planes up and checks the
// FP32 sums; empty children have qlo = 255, qhi = 0 and ref kEmptyChild.
constexpr uint32_t kNode4Q8Float4s = 4;

// BVH4 node with binary16 planes on an FP32 corner, 80 bytes:
//   c0 = (corner.x, corner.y, corner.z, -): the smallest lower plane of the
//        node's children on each axis
//   c1 = x planes: (lo of children 0,1 | 2,3, hi of children 0,1 | 2,3) as
//        binary16 pairs (child 2k in the low half); c2 = y, c3 = z likewise
//   c4 = (ref0, ref1, ref2, ref3)
// A plane is the FP32 sum corner + q (one rounding); the builder rounds q
// down for lower and up for upper planes and checks the sums.  Empty
// children have lo = +inf and hi = 0 (a box that no ray enters).
constexpr uint32_t kNode4CornerFloat4s = 5;

// Primitive slot, 48 bytes, leaf order:
//   triangle: s0 = (v0, prim id), s1 = (v1, material), s2 = (v2, kPrimTriangle)
//   sphere:   s0 = (centre, prim id), s1 = (radius, 0, 0, material), s2 = (0, 0, 0, kPrimSphere)
constexpr uint32_t kPrimTriangle = 0;
constexpr uint32_t kPrimSphere = 1;

constexpr uint32_t kMiss = 0xFFFFFFFFu;

// Material table entry (two float4): m0 = (albedo, type), m1 = (emission, ior).
enum : uint32_t { kLambert = 0, kMirror = 1, kDielectric = 2, kEmitter = 3 };

struct CameraView {
  float eye[3], fwd[3], right[3], up[3];
  float tan_x, tan_y;
};

// Two-level scenes (instancing): the top tree is a BVH4 over object boxes
// whose leaf refs (count 1) index instance records, two float4 each:
//   r0 = (translate.xyz, scale), r1 = (bottom root node, instance id, r, -)
// with r = 1 / scale rounded to FP32.  The base geometry is the record with
// translate 0, scale 1 and id 0.  The bottom trees follow the top tree in the
// node array, their primitive slots share one slot array, and a bottom slot's
// id is the primitive index within its own mesh.  An object ray is
// ((o - translate) * r, d * r): both scaled alike, so the ray parameter t,
// and hence the order of hits, is the same in both spaces.
struct SceneView {
  const float4* nodes;
  const float4* slots;
  const float4* materials;
  const float4* instances;  // instance records (two-level scenes only)
  uint32_t lds_nodes;  // nodes [0, lds_nodes) are staged in LDS
  uint32_t has_geometry;
  uint32_t width;       // 2 or 4 children per node
  uint32_t node_float4s;
  uint32_t two_level;   // 1: top tree over instances (width 4)
};

// Path queue (structure of float4 streams):
//   o = (origin, pixel), d = (direction, sample), b = (throughput, -)
struct RayQueue {
  float4* o;
  float4* d;
  float4* b;
};

// Environment queue: d = (direction, path slot), b = (throughput, -)
struct EnvQueue {
  float4* d;
  float4* b;
};

// Device counters (uint32 words), zeroed at the start of every pass.
//   [kCntRays + k]: rays entering depth k        (k = 1..64)
//   [kCntEnv + k]: escaped rays of depth k
//   [kCntWork + k]: work-distribution counter of the trace kernel at depth k
constexpr int kCntRays = 0;
constexpr int kCntEnv = 80;
constexpr int kCntWork = 160;
constexpr int kCntWords = 240;

// Fixed output colour matrix of the HDR-NIF (Sec. 3.2; the spaces of
// Sec. 4.3): log-space RGB = m (row-major 3x3) * network output.
struct ColourMatrix {
  float m[9];
};

struct PassView {
  uint32_t width, height, pixels;  // pixels = width * height
  uint32_t sample0, samples;        // samples of this pass: [sample0, sample0 + samples)
  uint32_t max_depth, rr_start;
  uint32_t key0, key1;              // Philox key = seed
};

}  // namespace npt
