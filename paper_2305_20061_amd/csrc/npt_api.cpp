// npt_api.cpp -- the C ABI of libnpt (include/npt.h): context, validation,
// scene / environment / NIF state, and the wavefront render loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bvh_build.h"
#include "npt.h"
#include "npt_kernels.h"
#include "npt_nif_layout.h"
#include "npt_shared.h"
#include "npt_train.h"

using namespace npt;

namespace {

// device allocation that grows on demand and is freed with its owner
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

bool finite_all(const float* a, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

struct npt_ctx {
  int device = -1;
  bool host_only = true;
  int num_cus = 256;
  bool fp8_capable = false;
  std::string err;

  // host scene
  std::vector<float> verts;
  std::vector<uint32_t> tris, tri_mat;
  std::vector<float> spheres;
  std::vector<uint32_t> sph_mat;
  std::vector<npt_material> materials;
  bool scene_dirty = true;
  FlatBvh bvh;
  bool bvh_built = false;
  // instancing: object-space meshes and their instances
  struct Mesh {
    std::vector<float> verts;
    std::vector<uint32_t> tris, mat;
  };
  std::vector<Mesh> blas;
  std::vector<npt_instance> instances;
  std::vector<float4> inst_records;  // two float4 per top-tree leaf
  bool two_level = false;

  // device scene
  DevBuf d_nodes, d_slots, d_mats, d_inst;
  int stack_depth = 32;

  bool have_camera = false;
  npt_camera camera{};
  npt_render_options opt{3, 0, 0};

  // environment
  DevBuf d_env;
  uint32_t env_w = 0, env_h = 0;
  int env_mode = NPT_ENV_MAP;

  // NIF
  bool have_nif = false;
  DevBuf d_master, d_adam_m, d_adam_v, d_frags, d_bias;
  uint32_t adam_step = 0;
  int nif_prec = NPT_FP16;
  ColourMatrix nif_cm{};  // output colour space of the uploaded network
  NifShape nif_shape{nif::ArchDefault::kHidden, nif::ArchDefault::kLayers, 0, nif::ArchDefault::kFreq};
  int nif_arch = 0;          // LDS-resident kernel of this shape (nif::resident_arch)
  bool nif_layered = false;  // layer-serial GEMM inference (shapes without a resident kernel, or on request)
  LayeredScratch layered;
  TrainScratch train;

  // render scratch
  DevBuf qa_o, qa_d, qa_b, qb_o, qb_d, qb_b, env_d, env_b, d_L, d_hits, d_accum, d_cnt, d_stats, d_order;
  void* noalloc_scratch = nullptr;  // this device's fixed scratch (npt_render_noalloc)
  hipError_t noalloc_status = hipErrorNotInitialized;
  npt_stats stats{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> event_pool, trace_events, shade_events, env_events;
  std::vector<uint32_t> env_depths;  // depth of each env_events pair
  bool timing_pending = false;

  ~npt_ctx() {
    DevBuf* all[] = {&d_nodes, &d_slots, &d_mats, &d_inst, &d_env, &d_master, &d_adam_m, &d_adam_v, &d_frags, &d_bias,
                     &qa_o, &qa_d, &qa_b, &qb_o, &qb_d, &qb_b, &env_d, &env_b, &d_L, &d_hits, &d_accum,
                     &d_cnt, &d_stats};
    for (DevBuf* b : all) b->release();
    train.release();
    layered.release();
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace {

int fail(npt_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int ok(npt_ctx* c) {
  c->err.clear();
  return NPT_OK;
}

// Nothing throws across the C ABI: a host allocation failure or another C++
// exception inside an entry point becomes NPT_E_OOM with a message.
template <class F>
int guarded(npt_ctx* c, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    if (c) c->err = "out of memory";  // short enough to need no allocation
  } catch (const std::exception& e) {
    try {
      if (c) c->err = e.what();
    } catch (...) {
    }
  } catch (...) {
    if (c) c->err = "host error";
  }
  return NPT_E_OOM;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, e_ == hipErrorOutOfMemory ? NPT_E_OOM : NPT_E_HIP,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

int need_device(npt_ctx* c) {
  if (c->host_only) return fail(c, NPT_E_NO_DEVICE, "host-only context has no GPU");
  HIP_TRY(c, hipSetDevice(c->device));
  return NPT_OK;
}

// Camera basis in FP32, formed on the host (fixed operation order, no
// contraction): fwd = |look_at - eye|, right = |fwd x up|, up' = right x fwd;
// tan(vfov/2) in FP64 rounded to FP32.
CameraView camera_view(const npt_camera& cam, uint32_t W, uint32_t H) {
  CameraView v;
  float f[3], r[3], u[3];
  for (int i = 0; i < 3; ++i) f[i] = cam.look_at[i] - cam.eye[i];
  float len = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
  for (int i = 0; i < 3; ++i) f[i] = f[i] / len;
  r[0] = f[1] * cam.up[2] - f[2] * cam.up[1];
  r[1] = f[2] * cam.up[0] - f[0] * cam.up[2];
  r[2] = f[0] * cam.up[1] - f[1] * cam.up[0];
  len = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
  for (int i = 0; i < 3; ++i) r[i] = r[i] / len;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  for (int i = 0; i < 3; ++i) {
    v.eye[i] = cam.eye[i];
    v.fwd[i] = f[i];
    v.right[i] = r[i];
    v.up[i] = u[i];
  }
  v.tan_y = (float)std::tan((double)cam.vfov_deg * (M_PI / 360.0));
  const float aspect = (float)W / (float)H;
  v.tan_x = v.tan_y * aspect;
  return v;
}

SceneView scene_view(npt_ctx* c) {
  SceneView s;
  s.nodes = c->d_nodes.as<float4>();
  s.slots = c->d_slots.as<float4>();
  s.materials = c->d_mats.as<float4>();
  s.lds_nodes = c->bvh.lds_nodes;
  s.has_geometry = c->bvh_built ? 1u : 0u;
  s.width = c->bvh.width;
  s.node_float4s = c->bvh.node_float4s;
  s.instances = c->d_inst.as<float4>();
  s.two_level = c->two_level ? 1u : 0u;
  return s;
}

int upload_materials(npt_ctx* c, hipStream_t s) {
  std::vector<npt_material> mats = c->materials;
  if (mats.empty()) mats.push_back(npt_material{NPT_LAMBERT, {0.5f, 0.5f, 0.5f}, {0, 0, 0}, 1.5f});
  std::vector<float4> m(2 * mats.size());
  for (size_t i = 0; i < mats.size(); ++i) {
    uint32_t t = mats[i].type;
    float tb;
    std::memcpy(&tb, &t, 4);
    m[2 * i] = make_float4(mats[i].albedo[0], mats[i].albedo[1], mats[i].albedo[2], tb);
    m[2 * i + 1] = make_float4(mats[i].emission[0], mats[i].emission[1], mats[i].emission[2], mats[i].ior);
  }
  HIP_TRY(c, c->d_mats.ensure(m.size() * sizeof(float4)));
  HIP_TRY(c, hipMemcpyAsync(c->d_mats.p, m.data(), m.size() * sizeof(float4), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return NPT_OK;
}

int repack_nif(npt_ctx* c, hipStream_t s) {
  if (!c->have_nif) return NPT_OK;
  if (c->nif_layered) {
    // row-major operand-precision copy of the weights; biases stay in the master
    const int64_t np = shape_params(c->nif_shape);
    HIP_TRY(c, c->d_frags.ensure((size_t)np * (c->nif_prec == NPT_FP32 ? 4 : 2)));
    HIP_TRY(c, launch_params_convert(c->nif_prec, c->d_master.as<float>(), c->d_frags.p, np, s));
    return NPT_OK;
  }
  const size_t bytes = nif_packed_bytes(c->nif_arch, c->nif_prec);
  if (bytes == 0) return fail(c, NPT_E_UNSUPPORTED, "precision not supported");
  HIP_TRY(c, c->d_frags.ensure(bytes));
  HIP_TRY(c, c->d_bias.ensure(nif_bias_bytes(c->nif_arch)));
  HIP_TRY(c, launch_nif_pack(c->nif_arch, c->nif_prec, c->d_master.as<float>(), c->d_frags.p,
                             c->d_bias.as<float>(), s));
  return NPT_OK;
}

}  // namespace

// ===========================================================================
// context
// ===========================================================================
extern "C" int npt_create(npt_ctx** out, int device) {
  return guarded(nullptr, [&]() -> int {
    if (!out) return NPT_E_INVALID_ARG;
    *out = nullptr;
    npt_ctx* c = new (std::nothrow) npt_ctx();
    if (!c) return NPT_E_OOM;
    if (device >= 0) {
      int count = 0;
      if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        delete c;
        return NPT_E_NO_DEVICE;
      }
      if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return NPT_E_HIP;
      }
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return NPT_E_HIP;
      }
      c->device = device;
      c->host_only = false;
      c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
      c->fp8_capable = std::strstr(prop.gcnArchName, "gfx950") != nullptr;
      if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return NPT_E_HIP;
      }
      // the device address of the fixed scratch, looked up once per device
      // with the device current; a failed lookup leaves only
      // npt_render_noalloc unavailable (it reports the error)
      c->noalloc_status = noalloc_scratch_ptr(device, &c->noalloc_scratch);
      if (c->noalloc_status != hipSuccess) c->noalloc_scratch = nullptr;
    }
    *out = c;
    return NPT_OK;
  });
}

extern "C" int npt_destroy(npt_ctx* ctx) {
  if (!ctx) return NPT_E_INVALID_ARG;
  if (!ctx->host_only) (void)hipSetDevice(ctx->device);
  delete ctx;
  return NPT_OK;
}

extern "C" const char* npt_last_error(npt_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ===========================================================================
// scene
// ===========================================================================
extern "C" int npt_scene_triangles(npt_ctx* c, const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt,
                                   const uint32_t* mat_of_tri) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if ((nv && !xyz) || (nt && !tri)) return fail(c, NPT_E_INVALID_ARG, "null array with nonzero size");
    if (nv > (1ull << 32) || nt >= kMaxSlots) return fail(c, NPT_E_INVALID_ARG, "too many vertices/triangles");
    if (!finite_all(xyz, 3 * nv)) return fail(c, NPT_E_NAN_INPUT, "non-finite vertex coordinate");
    for (uint64_t i = 0; i < 3 * nt; ++i)
      if (tri[i] >= nv) return fail(c, NPT_E_INVALID_ARG, "triangle index out of range");
    c->verts.assign(xyz, xyz + 3 * nv);
    c->tris.assign(tri, tri + 3 * nt);
    if (mat_of_tri) c->tri_mat.assign(mat_of_tri, mat_of_tri + nt);
    else c->tri_mat.assign(nt, 0u);
    c->scene_dirty = true;
    c->bvh_built = false;
    return ok(c);
  });
}

extern "C" int npt_scene_spheres(npt_ctx* c, const float* cxyzr, uint64_t n, const uint32_t* mat) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (n && !cxyzr) return fail(c, NPT_E_INVALID_ARG, "null sphere array");
    if (n >= kMaxSlots) return fail(c, NPT_E_INVALID_ARG, "too many spheres");
    if (!finite_all(cxyzr, 4 * n)) return fail(c, NPT_E_NAN_INPUT, "non-finite sphere");
    for (uint64_t i = 0; i < n; ++i)
      if (!(cxyzr[4 * i + 3] > 0.0f)) return fail(c, NPT_E_INVALID_ARG, "sphere radius must be > 0");
    c->spheres.assign(cxyzr, cxyzr + 4 * n);
    if (mat) c->sph_mat.assign(mat, mat + n);
    else c->sph_mat.assign(n, 0u);
    c->scene_dirty = true;
    c->bvh_built = false;
    return ok(c);
  });
}

extern "C" int npt_scene_blas_triangles(npt_ctx* c, uint32_t blas_id, const float* xyz, uint64_t nv,
                                        const uint32_t* tri, uint64_t nt, const uint32_t* mat_of_tri) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (blas_id > c->blas.size()) return fail(c, NPT_E_INVALID_ARG, "blas_id must be an existing id or the next one");
    if (nt == 0 || !xyz || !tri) return fail(c, NPT_E_INVALID_ARG, "an instanced mesh needs triangles");
    if (nv > (1ull << 32) || nt >= kMaxSlots) return fail(c, NPT_E_INVALID_ARG, "too many vertices/triangles");
    if (!finite_all(xyz, 3 * nv)) return fail(c, NPT_E_NAN_INPUT, "non-finite vertex coordinate");
    for (uint64_t i = 0; i < 3 * nt; ++i)
      if (tri[i] >= nv) return fail(c, NPT_E_INVALID_ARG, "triangle index out of range");
    npt_ctx::Mesh m;
    m.verts.assign(xyz, xyz + 3 * nv);
    m.tris.assign(tri, tri + 3 * nt);
    if (mat_of_tri) m.mat.assign(mat_of_tri, mat_of_tri + nt);
    else m.mat.assign(nt, 0u);
    if (blas_id == c->blas.size()) c->blas.push_back(std::move(m));
    else c->blas[blas_id] = std::move(m);
    c->scene_dirty = true;
    c->bvh_built = false;
    return ok(c);
  });
}

extern "C" int npt_scene_instances(npt_ctx* c, const npt_instance* inst, uint32_t n) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (n && !inst) return fail(c, NPT_E_INVALID_ARG, "null instance array");
    if (n >= (1u << 24)) return fail(c, NPT_E_INVALID_ARG, "too many instances");
    for (uint32_t i = 0; i < n; ++i) {
      if (inst[i].blas_id >= c->blas.size()) return fail(c, NPT_E_INVALID_ARG, "instance of an unknown blas_id");
      if (!finite_all(inst[i].translate, 3) || !std::isfinite(inst[i].scale))
        return fail(c, NPT_E_NAN_INPUT, "non-finite instance transform");
      if (!(inst[i].scale > 0.0f)) return fail(c, NPT_E_INVALID_ARG, "instance scale must be > 0");
    }
    c->instances.assign(inst, inst + n);
    c->scene_dirty = true;
    c->bvh_built = false;
    return ok(c);
  });
}

extern "C" int npt_scene_materials(npt_ctx* c, const npt_material* m, uint32_t n) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (n && !m) return fail(c, NPT_E_INVALID_ARG, "null material array");
    for (uint32_t i = 0; i < n; ++i) {
      if (m[i].type > NPT_EMITTER) return fail(c, NPT_E_INVALID_ARG, "unknown material type");
      if (!finite_all(m[i].albedo, 3) || !finite_all(m[i].emission, 3) || !std::isfinite(m[i].ior))
        return fail(c, NPT_E_NAN_INPUT, "non-finite material");
      if (m[i].type == NPT_DIELECTRIC && !(m[i].ior > 0.0f)) return fail(c, NPT_E_INVALID_ARG, "ior must be > 0");
    }
    c->materials.assign(m, m + n);
    if (!c->host_only) {
      int r = need_device(c);
      if (r) return r;
      r = upload_materials(c, nullptr);
      if (r) return r;
    }
    return ok(c);
  });
}

extern "C" int npt_build_bvh(npt_ctx* c, const npt_bvh_params* p, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    uint32_t bins = p && p->bins ? p->bins : 32, max_leaf = p && p->max_leaf ? p->max_leaf : 4;
    uint32_t lds_levels = p ? p->lds_levels : 0;
    const uint32_t width = p && p->width ? p->width : 4;
    const uint32_t node_format = p ? p->node_format : NPT_NODES_FP32;
    const BuildThreads threads(p ? (int)std::min<uint32_t>(p->threads, 64) : 0);
    if (width != 2 && width != 4) return fail(c, NPT_E_INVALID_ARG, "BVH width must be 2 or 4");
    if (node_format != NPT_NODES_FP32 && node_format != NPT_NODES_FP16_EXTENT && node_format != NPT_NODES_Q8 &&
        node_format != NPT_NODES_FP16_CORNER)
      return fail(c, NPT_E_INVALID_ARG, "unknown BVH node format");
    if (node_format != NPT_NODES_FP32 && width != 4)
      return fail(c, NPT_E_INVALID_ARG, "compressed nodes need width 4");
    if ((node_format == NPT_NODES_Q8 || node_format == NPT_NODES_FP16_CORNER) && lds_levels != 0)
      return fail(c, NPT_E_INVALID_ARG, "8-bit and binary16-corner nodes are read from memory: lds_levels must be 0");
    if (bins < 4 || bins > 256 || max_leaf < 1 || max_leaf > kMaxLeaf || lds_levels > 8)
      return fail(c, NPT_E_INVALID_ARG, "bvh params out of range");
    const bool has_base = !c->tris.empty() || !c->spheres.empty();
    const bool two_level = !c->instances.empty();
    if (!has_base && !two_level) return fail(c, NPT_E_NO_SCENE, "no geometry uploaded");
    if (two_level && width != 4) return fail(c, NPT_E_UNSUPPORTED, "instanced scenes use width 4");
    if (two_level && lds_levels != 0 && node_format == NPT_NODES_FP32)
      return fail(c, NPT_E_UNSUPPORTED, "LDS levels of an instanced scene need binary16-extent nodes");
    const uint32_t nmat = (uint32_t)std::max<size_t>(1, c->materials.size());
    for (uint32_t m : c->tri_mat)
      if (m >= nmat) return fail(c, NPT_E_INVALID_ARG, "triangle material id out of range");
    for (uint32_t m : c->sph_mat)
      if (m >= nmat) return fail(c, NPT_E_INVALID_ARG, "sphere material id out of range");
    for (const npt_instance& k : c->instances) {
      if (k.blas_id >= c->blas.size()) return fail(c, NPT_E_INVALID_ARG, "instance of an unknown blas_id");
      for (uint32_t m : c->blas[k.blas_id].mat)
        if (m >= nmat) return fail(c, NPT_E_INVALID_ARG, "instanced triangle material id out of range");
    }
    BuildInput in;
    in.verts = c->verts.data();
    in.nv = c->verts.size() / 3;
    in.tris = c->tris.data();
    in.nt = c->tris.size() / 3;
    in.tri_mat = c->tri_mat.data();
    in.spheres = c->spheres.data();
    in.ns = c->spheres.size() / 4;
    in.sph_mat = c->sph_mat.data();
    FlatBvh b;
    std::vector<float4> records;
    std::string e;
    uint32_t stack_need = 0;
    if (!two_level) {
      if (!build_bvh(in, bins, max_leaf, lds_levels, width, b, e)) return fail(c, NPT_E_INVALID_ARG, e);
      // deferred children: one per level (width 2); up to three per level,
      // plus the three of the deepest node (width 4)
      stack_need = width == 2 ? b.max_depth + 1 : 3 * b.max_depth + 3;
    } else {
      // bottom trees: the base geometry (instance 0) and each instanced mesh
      std::vector<FlatBvh> bottoms;
      std::vector<Placement> objects;
      if (has_base) {
        bottoms.emplace_back();
        if (!build_bvh(in, bins, max_leaf, 0, 4, bottoms.back(), e)) return fail(c, NPT_E_INVALID_ARG, e);
        objects.push_back(Placement{0u, {0.0f, 0.0f, 0.0f}, 1.0f, 0u});
      }
      std::vector<int64_t> tree_of(c->blas.size(), -1);
      for (size_t k = 0; k < c->instances.size(); ++k) {
        const npt_instance& x = c->instances[k];
        if (tree_of[x.blas_id] < 0) {
          const npt_ctx::Mesh& m = c->blas[x.blas_id];
          BuildInput bi;
          bi.verts = m.verts.data();
          bi.nv = m.verts.size() / 3;
          bi.tris = m.tris.data();
          bi.nt = m.tris.size() / 3;
          bi.tri_mat = m.mat.data();
          bottoms.emplace_back();
          if (!build_bvh(bi, bins, max_leaf, 0, 4, bottoms.back(), e)) return fail(c, NPT_E_INVALID_ARG, e);
          tree_of[x.blas_id] = (int64_t)bottoms.size() - 1;
        }
        objects.push_back(Placement{(uint32_t)tree_of[x.blas_id],
                                    {x.translate[0], x.translate[1], x.translate[2]},
                                    x.scale,
                                    (uint32_t)(k + 1)});
      }
      if (!build_two_level(bottoms, objects, bins, lds_levels, b, records, stack_need, e))
        return fail(c, NPT_E_INVALID_ARG, e);
    }
    if (node_format == NPT_NODES_FP16_EXTENT && !compress_half_extents(b, e)) return fail(c, NPT_E_UNSUPPORTED, e);
    if (node_format == NPT_NODES_Q8 && !compress_q8_nodes(b, e)) return fail(c, NPT_E_UNSUPPORTED, e);
    if (node_format == NPT_NODES_FP16_CORNER && !compress_corner_nodes(b, e)) return fail(c, NPT_E_UNSUPPORTED, e);
    if (trace_stack_size(stack_need) == 0)
      return fail(c, NPT_E_UNSUPPORTED, "BVH deeper than the 128-entry traversal stack");
    // the traversal addresses nodes with 32-bit byte offsets
    if ((uint64_t)b.nodes.size() * sizeof(float4) >= (1ull << 32))
      return fail(c, NPT_E_UNSUPPORTED, "BVH node array of 4 GiB or more (use a larger max_leaf)");
    c->bvh = std::move(b);
    c->inst_records = std::move(records);
    c->two_level = two_level;
    c->bvh_built = false;
    if (c->host_only) return fail(c, NPT_E_NO_DEVICE, "BVH built on the host; no device to upload to");
    int r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(c, c->d_nodes.ensure(c->bvh.nodes.size() * sizeof(float4)));
    HIP_TRY(c, c->d_slots.ensure(c->bvh.slots.size() * sizeof(float4)));
    HIP_TRY(c, hipMemcpyAsync(c->d_nodes.p, c->bvh.nodes.data(), c->bvh.nodes.size() * sizeof(float4),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_slots.p, c->bvh.slots.data(), c->bvh.slots.size() * sizeof(float4),
                              hipMemcpyHostToDevice, s));
    if (two_level) {
      HIP_TRY(c, c->d_inst.ensure(c->inst_records.size() * sizeof(float4)));
      HIP_TRY(c, hipMemcpyAsync(c->d_inst.p, c->inst_records.data(), c->inst_records.size() * sizeof(float4),
                                hipMemcpyHostToDevice, s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    r = upload_materials(c, s);
    if (r) return r;
    c->stack_depth = trace_stack_size(stack_need);
    c->bvh_built = true;
    c->scene_dirty = false;
    return ok(c);
  });
}

extern "C" int npt_bvh_info(npt_ctx* c, uint64_t* nodes, uint64_t* leaves, uint32_t* max_depth, uint64_t* slots,
                            uint32_t* width) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (c->bvh.nodes.empty()) return fail(c, NPT_E_STATE, "no BVH built");
    if (nodes) *nodes = c->bvh.nodes.size() / c->bvh.node_float4s;
    if (leaves) *leaves = c->bvh.leaves;
    if (max_depth) *max_depth = c->bvh.max_depth;
    if (slots) *slots = c->bvh.slots.size() / 3;
    if (width) *width = c->bvh.width;
    return ok(c);
  });
}

extern "C" int npt_bvh_export(npt_ctx* c, void* nodes, uint64_t* node_bytes, void* slots, uint64_t* slot_bytes,
                              void* records, uint64_t* record_bytes) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (c->bvh.nodes.empty()) return fail(c, NPT_E_STATE, "no BVH built");
    if (!node_bytes || !slot_bytes || !record_bytes) return fail(c, NPT_E_INVALID_ARG, "null size");
    const uint64_t nb = c->bvh.nodes.size() * sizeof(float4), sb = c->bvh.slots.size() * sizeof(float4),
                   rb = c->two_level ? c->inst_records.size() * sizeof(float4) : 0;
    const bool copy = nodes || slots || records;
    if (copy && ((nodes && *node_bytes < nb) || (slots && *slot_bytes < sb) || (records && *record_bytes < rb)))
      return fail(c, NPT_E_INVALID_ARG, "export buffer too small");
    if (nodes) std::memcpy(nodes, c->bvh.nodes.data(), nb);
    if (slots) std::memcpy(slots, c->bvh.slots.data(), sb);
    if (records && rb) std::memcpy(records, c->inst_records.data(), rb);
    *node_bytes = nb;
    *slot_bytes = sb;
    *record_bytes = rb;
    return ok(c);
  });
}

extern "C" int npt_set_camera(npt_ctx* c, const npt_camera* cam) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!cam) return fail(c, NPT_E_INVALID_ARG, "null camera");
    if (!finite_all(cam->eye, 3) || !finite_all(cam->look_at, 3) || !finite_all(cam->up, 3) ||
        !std::isfinite(cam->vfov_deg))
      return fail(c, NPT_E_NAN_INPUT, "non-finite camera");
    if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f)) return fail(c, NPT_E_INVALID_ARG, "vfov out of (0,180)");
    float f[3];
    for (int i = 0; i < 3; ++i) f[i] = cam->look_at[i] - cam->eye[i];
    const float cx = f[1] * cam->up[2] - f[2] * cam->up[1], cy = f[2] * cam->up[0] - f[0] * cam->up[2],
                cz = f[0] * cam->up[1] - f[1] * cam->up[0];
    if (f[0] == 0 && f[1] == 0 && f[2] == 0) return fail(c, NPT_E_INVALID_ARG, "eye == look_at");
    if (cx == 0 && cy == 0 && cz == 0) return fail(c, NPT_E_INVALID_ARG, "up parallel to view direction");
    c->camera = *cam;
    c->have_camera = true;
    return ok(c);
  });
}

extern "C" int npt_set_render_options(npt_ctx* c, const npt_render_options* o) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!o) return fail(c, NPT_E_INVALID_ARG, "null options");
    if (o->pool_paths > (1u << 30)) return fail(c, NPT_E_INVALID_ARG, "pool_paths > 2^30");
    c->opt = *o;
    return ok(c);
  });
}

// ===========================================================================
// environment
// ===========================================================================
extern "C" int npt_env_upload(npt_ctx* c, const float* rgb, uint32_t w, uint32_t h, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!rgb || w == 0 || h == 0 || (uint64_t)w * h > (1ull << 28)) return fail(c, NPT_E_INVALID_ARG, "bad env map");
    const uint64_t n = (uint64_t)w * h;
    for (uint64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(rgb[i]) || rgb[i] < 0.0f) return fail(c, NPT_E_NAN_INPUT, "non-finite or negative radiance");
    int r = need_device(c);
    if (r) return r;
    std::vector<float4> m(n);
    for (uint64_t i = 0; i < n; ++i) m[i] = make_float4(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], 0.0f);
    HIP_TRY(c, c->d_env.ensure(n * sizeof(float4)));
    HIP_TRY(c, hipMemcpyAsync(c->d_env.p, m.data(), n * sizeof(float4), hipMemcpyHostToDevice, (hipStream_t)stream));
    HIP_TRY(c, hipStreamSynchronize((hipStream_t)stream));
    c->env_w = w;
    c->env_h = h;
    return ok(c);
  });
}

extern "C" int npt_set_env_mode(npt_ctx* c, int mode) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (mode != NPT_ENV_MAP && mode != NPT_ENV_NIF && mode != NPT_ENV_NONE)
      return fail(c, NPT_E_INVALID_ARG, "unknown env mode");
    c->env_mode = mode;
    return ok(c);
  });
}

// ===========================================================================
// NIF
// ===========================================================================
static bool nif_desc_ok(const npt_nif_desc* d) {
  return d && d->n_freq >= 1 && d->n_freq <= (uint32_t)nif::kMaxFreq && d->hidden >= 32 && d->hidden <= 1024 &&
         d->hidden % 32 == 0 && d->layers >= 1 && d->layers <= 8 &&
         (d->skip == 0 || (d->skip < d->layers && d->hidden > 4 * d->n_freq));
}

// log-space RGB = M * network output for the colour spaces of Sec. 4.3:
// YUV (BT.601 analogue), RGB (identity), YCoCg (Malvar & Sullivan).
static ColourMatrix colour_matrix(uint32_t colour) {
  switch (colour) {
    case NPT_COLOUR_RGB: return ColourMatrix{{1, 0, 0, 0, 1, 0, 0, 0, 1}};
    case NPT_COLOUR_YCOCG: return ColourMatrix{{1, 1, -1, 1, 0, 1, 1, -1, -1}};
    default: return ColourMatrix{{1.0f, 0.0f, 1.13983f, 1.0f, -0.39465f, -0.58060f, 1.0f, 2.03211f, 0.0f}};
  }
}

extern "C" int npt_nif_upload(npt_ctx* c, const npt_nif_desc* desc, const float* params, uint64_t n, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!nif_desc_ok(desc))
      return fail(c, NPT_E_UNSUPPORTED,
                  "NIF shape must be n_freq 1..16, hidden 32..1024 (a multiple of 32), layers 1..8, "
                  "skip 0 or < layers with hidden > 4 n_freq");
    if (desc->colour > NPT_COLOUR_YCOCG) return fail(c, NPT_E_INVALID_ARG, "unknown NIF colour space");
    const NifShape shape{(int)desc->hidden, (int)desc->layers, (int)desc->skip, (int)desc->n_freq};
    const int arch = nif::resident_arch(shape.hidden, shape.layers, shape.skip, shape.n_freq);
    const bool layered = desc->layered != 0 || arch < 0;
    if (layered && c->nif_prec == NPT_FP8)
      return fail(c, NPT_E_UNSUPPORTED,
                  "FP8 inference needs a network shape with an LDS-resident kernel; set another precision first");
    if (!params || n != (uint64_t)shape_params(shape)) return fail(c, NPT_E_INVALID_ARG, "parameter count mismatch");
    if (!finite_all(params, n)) return fail(c, NPT_E_NAN_INPUT, "non-finite NIF parameter");
    int r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = n * sizeof(float);
    HIP_TRY(c, c->d_master.ensure(bytes));
    HIP_TRY(c, c->d_adam_m.ensure(bytes));
    HIP_TRY(c, c->d_adam_v.ensure(bytes));
    HIP_TRY(c, hipMemcpyAsync(c->d_master.p, params, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(c->d_adam_m.p, 0, bytes, s));
    HIP_TRY(c, hipMemsetAsync(c->d_adam_v.p, 0, bytes, s));
    c->adam_step = 0;
    c->have_nif = true;
    c->nif_cm = colour_matrix(desc->colour);
    c->nif_shape = shape;
    c->nif_layered = layered;
    c->nif_arch = layered ? 0 : arch;
    r = repack_nif(c, s);
    if (r) return r;
    HIP_TRY(c, hipStreamSynchronize(s));
    return ok(c);
  });
}

extern "C" int npt_nif_download(npt_ctx* c, float* params, uint64_t n) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
    if (!params || n != (uint64_t)shape_params(c->nif_shape))
      return fail(c, NPT_E_INVALID_ARG, "parameter count mismatch");
    int r = need_device(c);
    if (r) return r;
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(params, c->d_master.p, n * sizeof(float), hipMemcpyDeviceToHost));
    return ok(c);
  });
}

extern "C" int npt_nif_get_state(npt_ctx* c, float* params, float* m, float* v, uint64_t n, uint32_t* step) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
    if (n != (uint64_t)shape_params(c->nif_shape)) return fail(c, NPT_E_INVALID_ARG, "parameter count mismatch");
    int r = need_device(c);
    if (r) return r;
    HIP_TRY(c, hipDeviceSynchronize());
    const size_t bytes = n * sizeof(float);
    if (params) HIP_TRY(c, hipMemcpy(params, c->d_master.p, bytes, hipMemcpyDeviceToHost));
    if (m) HIP_TRY(c, hipMemcpy(m, c->d_adam_m.p, bytes, hipMemcpyDeviceToHost));
    if (v) HIP_TRY(c, hipMemcpy(v, c->d_adam_v.p, bytes, hipMemcpyDeviceToHost));
    if (step) *step = c->adam_step;
    return ok(c);
  });
}

extern "C" int npt_nif_set_state(npt_ctx* c, const float* params, const float* m, const float* v, uint64_t n,
                                 uint32_t step, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
    if (!params || !m || !v) return fail(c, NPT_E_INVALID_ARG, "null state array");
    if (n != (uint64_t)shape_params(c->nif_shape)) return fail(c, NPT_E_INVALID_ARG, "parameter count mismatch");
    if (!finite_all(params, n) || !finite_all(m, n) || !finite_all(v, n))
      return fail(c, NPT_E_NAN_INPUT, "non-finite training state");
    for (uint64_t i = 0; i < n; ++i)
      if (v[i] < 0.0f) return fail(c, NPT_E_NAN_INPUT, "negative second moment");
    int r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = n * sizeof(float);
    HIP_TRY(c, hipMemcpyAsync(c->d_master.p, params, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_adam_m.p, m, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_adam_v.p, v, bytes, hipMemcpyHostToDevice, s));
    c->adam_step = step;
    r = repack_nif(c, s);
    if (r) return r;
    HIP_TRY(c, hipStreamSynchronize(s));
    return ok(c);
  });
}

extern "C" int npt_nif_set_precision(npt_ctx* c, int prec) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (prec < NPT_FP32 || prec > NPT_FP8) return fail(c, NPT_E_INVALID_ARG, "unknown precision");
    if (prec == NPT_FP8 && (c->host_only || !c->fp8_capable))
      return fail(c, NPT_E_UNSUPPORTED, "FP8 NIF inference needs gfx950");
    if (nif_packed_bytes(0, prec) == 0) return fail(c, NPT_E_UNSUPPORTED, "precision not built");
    if (prec == NPT_FP8 && c->have_nif && c->nif_layered)
      return fail(c, NPT_E_UNSUPPORTED, "FP8 inference needs a network shape with an LDS-resident kernel");
    const int old = c->nif_prec;
    c->nif_prec = prec;
    if (c->have_nif) {
      int r = need_device(c);
      if (r) { c->nif_prec = old; return r; }
      r = repack_nif(c, nullptr);
      if (r) { c->nif_prec = old; return r; }
      HIP_TRY(c, hipStreamSynchronize(nullptr));
    }
    return ok(c);
  });
}

extern "C" int npt_nif_get_dequantized(npt_ctx* c, float* params, uint64_t n) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
    if (!params || n != (uint64_t)shape_params(c->nif_shape))
      return fail(c, NPT_E_INVALID_ARG, "parameter count mismatch");
    int r = need_device(c);
    if (r) return r;
    DevBuf tmp;
    HIP_TRY(c, tmp.ensure(n * sizeof(float)));
    hipError_t e = c->nif_layered
                      ? launch_params_dequant(c->nif_prec, c->nif_shape, c->d_master.as<float>(), c->d_frags.p,
                                              tmp.as<float>(), nullptr)
                      : launch_nif_dequant(c->nif_arch, c->nif_prec, c->d_master.as<float>(), c->d_bias.as<float>(),
                                           tmp.as<float>(), (int)n, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipMemcpy(params, tmp.p, n * sizeof(float), hipMemcpyDeviceToHost);
    tmp.release();
    HIP_TRY(c, e);
    return ok(c);
  });
}

static void train_defaults(npt_ctx* c, const npt_train_params* p, TrainConfig& t) {
  t.cm = c->nif_cm;
  t.shape = c->nif_shape;
  t.batch = p && p->batch ? p->batch : 65536;
  t.samples = p && p->samples ? p->samples : (1ull << 24);
  t.lr = p && p->lr > 0 ? p->lr : 1e-3f;
  t.beta1 = p && p->beta1 > 0 ? p->beta1 : 0.9f;
  t.beta2 = p && p->beta2 > 0 ? p->beta2 : 0.999f;
  t.eps = p && p->eps > 0 ? p->eps : 1e-7f;
  t.delta = p && p->huber_delta > 0 ? p->huber_delta : 1e-3f;
  t.seed = p ? p->seed : 0;
  t.prec = p ? (int)p->grad_prec : NPT_FP32;
  // Sec. 3.2.1 trains with FP16 gradients under a loss scale of 16384
  t.loss_scale = p && p->loss_scale > 0 ? p->loss_scale : (t.prec == NPT_FP16 ? 16384.0f : 1.0f);
  t.master_prec = p ? (int)p->master_prec : NPT_FP32;
  t.path = p ? (int)p->path : NPT_TRAIN_AUTO;
}

static int train_check(npt_ctx* c, const TrainConfig& t) {
  if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
  if (!c->env_w) return fail(c, NPT_E_NO_ENV, "no environment map to train on");
  if (t.batch == 0 || t.batch % 2048 != 0 || t.batch > (1u << 22))
    return fail(c, NPT_E_INVALID_ARG, "batch must be a positive multiple of 2048, <= 2^22");
  if (t.prec != NPT_FP32 && t.prec != NPT_FP16 && t.prec != NPT_BF16)
    return fail(c, NPT_E_INVALID_ARG, "grad_prec must be FP32, FP16 or BF16");
  if (t.master_prec != NPT_FP32 && t.master_prec != NPT_FP16)
    return fail(c, NPT_E_INVALID_ARG, "master_prec must be FP32 or FP16");
  if (t.path != NPT_TRAIN_AUTO && t.path != NPT_TRAIN_LAYERED)
    return fail(c, NPT_E_INVALID_ARG, "path must be NPT_TRAIN_AUTO or NPT_TRAIN_LAYERED");
  return NPT_OK;
}

static TrainTargets train_targets(npt_ctx* c) {
  TrainTargets tt;
  tt.map = c->d_env.as<float4>();
  tt.w = c->env_w;
  tt.h = c->env_h;
  tt.master = c->d_master.as<float>();
  tt.m = c->d_adam_m.as<float>();
  tt.v = c->d_adam_v.as<float>();
  return tt;
}

extern "C" int npt_nif_train(npt_ctx* c, const npt_train_params* p, npt_train_stats* out, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    TrainConfig t;
    train_defaults(c, p, t);
    int r = train_check(c, t);
    if (r) return r;
    r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t steps = (uint32_t)((t.samples + t.batch - 1) / t.batch);
    TrainTargets tt = train_targets(c);
    float first = 0.0f, last = 0.0f, ms = 0.0f;
    HIP_TRY(c, hipEventRecord(c->ev0, s));
    hipError_t e = train_run(c->train, t, tt, c->adam_step, steps, &first, &last, s);
    HIP_TRY(c, e);
    HIP_TRY(c, hipEventRecord(c->ev1, s));
    HIP_TRY(c, hipEventSynchronize(c->ev1));
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->adam_step += steps;
    r = repack_nif(c, s);
    if (r) return r;
    HIP_TRY(c, hipStreamSynchronize(s));
    if (out) {
      out->steps = steps;
      out->step_total = c->adam_step;
      out->first_loss = first;
      out->last_loss = last;
      out->ms = ms;
    }
    return ok(c);
  });
}

extern "C" int npt_nif_train_grad(npt_ctx* c, const npt_train_params* p, uint32_t step, float* d_grad,
                                  float* d_loss, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!d_grad || !d_loss) return fail(c, NPT_E_INVALID_ARG, "null output");
    TrainConfig t;
    train_defaults(c, p, t);
    int r = train_check(c, t);
    if (r) return r;
    r = need_device(c);
    if (r) return r;
    HIP_TRY(c, train_gradient(c->train, t, train_targets(c), step, d_grad, d_loss, (hipStream_t)stream));
    return ok(c);
  });
}

extern "C" int npt_nif_eval_grid(npt_ctx* c, uint32_t gw, uint32_t gh, float* out2, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!out2 || gw == 0 || gh == 0 || (uint64_t)gw * gh > (1ull << 26)) return fail(c, NPT_E_INVALID_ARG, "bad grid");
    if (!c->have_nif) return fail(c, NPT_E_STATE, "no NIF uploaded");
    if (!c->env_w) return fail(c, NPT_E_NO_ENV, "no environment map");
    int r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    float res[2] = {0, 0};
    if (c->nif_layered)
      HIP_TRY(c, grid_eval(c->train, c->nif_prec, 0, c->d_frags.p, c->d_master.as<float>(), c->nif_cm,
                           train_targets(c), gw, gh, c->num_cus, res, s, &c->layered, &c->nif_shape));
    else
      HIP_TRY(c, grid_eval(c->train, c->nif_prec, c->nif_arch, c->d_frags.p, c->d_bias.as<float>(), c->nif_cm,
                           train_targets(c), gw, gh, c->num_cus, res, s));
    out2[0] = res[0];
    out2[1] = res[1];
    return ok(c);
  });
}

extern "C" int npt_env_query(npt_ctx* c, int mode, const float* d_dirs, uint64_t n, float* d_rgb, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!d_dirs || !d_rgb || n == 0) return fail(c, NPT_E_INVALID_ARG, "bad query buffers");
    int r = need_device(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    if (mode == NPT_ENV_MAP) {
      if (!c->env_w) return fail(c, NPT_E_NO_ENV, "no environment map");
      HIP_TRY(c, launch_env_query_map(c->d_env.as<float4>(), (int)c->env_w, (int)c->env_h, d_dirs, n, d_rgb, s));
    } else if (mode == NPT_ENV_NIF) {
      if (!c->have_nif) return fail(c, NPT_E_NO_ENV, "no NIF uploaded");
      if (c->nif_layered) {
        LayeredIO io{};
        io.source = kLayeredDirs;
        io.dirs = d_dirs;
        io.out = d_rgb;
        io.n = n;
        HIP_TRY(c, nif_layered(c->layered, c->nif_prec, c->nif_shape, c->d_frags.p, c->d_master.as<float>(), c->nif_cm,
                               io, s));
      } else {
        HIP_TRY(c, launch_nif_dirs(c->nif_arch, c->nif_prec, c->d_frags.p, c->d_bias.as<float>(), c->nif_cm,
                                   d_dirs, n, d_rgb, c->num_cus, s));
      }
    } else {
      return fail(c, NPT_E_INVALID_ARG, "unknown env mode");
    }
    return ok(c);
  });
}

// ===========================================================================
// rendering
// ===========================================================================
static int render_checks(npt_ctx* c, uint32_t W, uint32_t H) {
  if (c->tris.empty() && c->spheres.empty() && c->instances.empty())
    return fail(c, NPT_E_NO_SCENE, "no geometry uploaded");
  if (!c->bvh_built) return fail(c, NPT_E_STATE, "npt_build_bvh not called after the last scene change");
  if (!c->have_camera) return fail(c, NPT_E_STATE, "no camera set");
  if (W == 0 || H == 0) return fail(c, NPT_E_INVALID_ARG, "zero image size");
  if ((uint64_t)W * H >= (1ull << 31)) return fail(c, NPT_E_INVALID_ARG, "image too large");
  return NPT_OK;
}

// argument and state checks shared by the render entry points
static int render_args(npt_ctx* c, uint32_t W, uint32_t H, uint32_t spp, uint32_t max_depth, const float* d_out) {
  if (!d_out) return fail(c, NPT_E_INVALID_ARG, "null output buffer");
  if (spp == 0 || max_depth == 0 || max_depth > NPT_MAX_DEPTH)
    return fail(c, NPT_E_INVALID_ARG, "spp must be > 0 and max_depth in 1..64");
  if (W == 0 || H == 0 || (uint64_t)W * H * spp >= (1ull << 40))
    return fail(c, NPT_E_INVALID_ARG, "W*H*spp must be in (0, 2^40)");
  if (c->host_only) return fail(c, NPT_E_NO_DEVICE, "host-only context cannot render");
  int r = render_checks(c, W, H);
  if (r) return r;
  if (c->env_mode == NPT_ENV_MAP && !c->env_w) return fail(c, NPT_E_NO_ENV, "env mode MAP without a map");
  if (c->env_mode == NPT_ENV_NIF && !c->have_nif) return fail(c, NPT_E_NO_ENV, "env mode NIF without weights");
  return need_device(c);
}

// device buffers of one render: the path pool (slots = pixels x samples per
// pass; two ray queues, the environment queue, path radiance and hit
// records, 16 bytes per slot each), the accumulator, the queue counters and
// the per-depth statistics
struct RenderBufs {
  float4 *qa_o, *qa_d, *qa_b, *qb_o, *qb_d, *qb_b, *env_d, *env_b, *L, *hits, *accum;
  uint32_t* cnt;
  unsigned long long* stats;
  uint32_t* order = nullptr;  // trace order of sorted secondary rays (sort_rays), else null
};
constexpr int kPoolStreams = 10;  // float4 streams per path slot

// The passes over samples [s_begin, s_end) of every pixel (samples_per_pass
// samples each) on the given buffers.  Each pixel's radiance is added to
// b.accum in sample order, which is cleared first when s_begin == 0; with
// d_out, the mean over samples [0, s_end) is written there.  With `timing`,
// HIP events around every kernel launch.
static int render_passes(npt_ctx* c, uint32_t W, uint32_t H, uint64_t s_begin, uint64_t s_end, uint32_t max_depth,
                         uint64_t seed, float* d_out, hipStream_t s, const RenderBufs& b, uint64_t sp, bool timing,
                         unsigned long long* visit_cnt) {
  const uint64_t pixels = (uint64_t)W * H;
  c->trace_events.clear();
  c->shade_events.clear();
  c->env_events.clear();
  c->env_depths.clear();
  auto event_pair = [&](std::vector<hipEvent_t>& v) -> hipError_t {
    // events are pooled per context and reused across renders
    const size_t need = c->trace_events.size() + c->shade_events.size() + c->env_events.size() + 2;
    while (c->event_pool.size() < need) {
      hipEvent_t e;
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      c->event_pool.push_back(e);
    }
    v.push_back(c->event_pool[need - 2]);
    v.push_back(c->event_pool[need - 1]);
    return hipSuccess;
  };

  const SceneView sv = scene_view(c);
  const CameraView cam = camera_view(c->camera, W, H);
  RayQueue qa{b.qa_o, b.qa_d, b.qa_b};
  RayQueue qbq{b.qb_o, b.qb_d, b.qb_b};
  EnvQueue eq{b.env_d, b.env_b};
  float4* L = b.L;
  uint32_t* cnt = b.cnt;

  uint32_t passes = 0;
  for (uint64_t s0 = s_begin; s0 < s_end; s0 += sp) {
    PassView pv;
    pv.width = W;
    pv.height = H;
    pv.pixels = (uint32_t)pixels;
    pv.sample0 = (uint32_t)s0;
    pv.samples = (uint32_t)std::min<uint64_t>(sp, s_end - s0);
    pv.max_depth = max_depth;
    pv.rr_start = c->opt.rr_start ? c->opt.rr_start : 3;
    pv.key0 = (uint32_t)seed;
    pv.key1 = (uint32_t)(seed >> 32);
    const uint64_t n = pixels * pv.samples;
    HIP_TRY(c, launch_pass_init(cnt, (uint32_t)n, s));
    HIP_TRY(c, launch_generate(cam, pv, qa, L, s));
    RayQueue in = qa, out = qbq;
    for (uint32_t k = 1; k <= max_depth; ++k) {
      if (timing) {
        HIP_TRY(c, event_pair(c->trace_events));
        HIP_TRY(c, hipEventRecord(c->trace_events[c->trace_events.size() - 2], s));
      }
      const bool sorted = b.order && k >= 2;
      if (sorted) HIP_TRY(c, launch_sort_chunks(in, cnt, k, n, c->bvh.lo, c->bvh.hi, b.order, s));
      HIP_TRY(c, launch_extend(c->stack_depth, sv, k, n, in, b.hits, cnt, visit_cnt, sorted ? b.order : nullptr,
                               c->num_cus, s));
      if (timing) {
        HIP_TRY(c, hipEventRecord(c->trace_events.back(), s));
        HIP_TRY(c, event_pair(c->shade_events));
        HIP_TRY(c, hipEventRecord(c->shade_events[c->shade_events.size() - 2], s));
      }
      HIP_TRY(c, launch_shade(sv, pv, k, n, in, b.hits, out, eq, L, cnt, c->num_cus, s));
      if (timing) HIP_TRY(c, hipEventRecord(c->shade_events.back(), s));
      if (c->env_mode != NPT_ENV_NONE) {  // NONE: escaped paths carry no radiance
        if (timing) {
          HIP_TRY(c, event_pair(c->env_events));
          c->env_depths.push_back(k);
          HIP_TRY(c, hipEventRecord(c->env_events[c->env_events.size() - 2], s));
        }
        if (c->env_mode == NPT_ENV_MAP) {
          HIP_TRY(c, launch_env_lookup(c->d_env.as<float4>(), (int)c->env_w, (int)c->env_h, eq, L, cnt, k, n,
                                       c->num_cus, s));
        } else if (c->nif_layered) {
          LayeredIO io{};
          io.source = kLayeredQueue;
          io.env = eq;
          io.L = L;
          io.cnt = cnt;
          io.depth = k;
          HIP_TRY(c, nif_layered(c->layered, c->nif_prec, c->nif_shape, c->d_frags.p, c->d_master.as<float>(),
                                 c->nif_cm, io, s));
        } else {
          HIP_TRY(c, launch_nif_queue(c->nif_arch, c->nif_prec, c->d_frags.p, c->d_bias.as<float>(), c->nif_cm, eq, L,
                                      cnt, k, n, c->num_cus, s));
        }
        if (timing) HIP_TRY(c, hipEventRecord(c->env_events.back(), s));
      }
      std::swap(in, out);
    }
    HIP_TRY(c, launch_accumulate(L, b.accum, pv, s0 == 0, s));
    HIP_TRY(c, launch_stats_add(cnt, b.stats, s));
    ++passes;
  }
  if (d_out) HIP_TRY(c, launch_finalize(b.accum, d_out, (uint32_t)pixels, 1.0f / (float)s_end, s));
  c->stats = npt_stats{};
  c->stats.paths = pixels * (s_end - s_begin);
  c->stats.passes = passes;
  c->stats.samples_per_pass = (uint32_t)sp;
  return NPT_OK;
}

// A render of samples [s_begin, s_end) on the context's path pool, adding to
// `accum` (the context's accumulator when null); the mean over [0, s_end) goes
// to d_out when it is given.
static int render_pooled(npt_ctx* c, uint32_t W, uint32_t H, uint64_t s_begin, uint64_t s_end, uint32_t max_depth,
                         uint64_t seed, float4* accum, float* d_out, hipStream_t s) {
  const uint64_t pixels = (uint64_t)W * H;
  // default pool: 2^27 paths in flight (a whole 1080p x 64 spp frame in one
  // pass; 160 B of queues per path = 21.5 GB of the 288 GB of HBM).  One pass
  // instead of two halves the launches per frame and with them the tails in
  // which a launch's last rays run on a nearly empty GPU: 2.6 % more path
  // samples/s on the large-BVH frame.  Only the queues a render needs are
  // allocated.
  const uint64_t pool = c->opt.pool_paths ? c->opt.pool_paths : (1ull << 27);
  uint64_t sp = c->opt.samples_per_pass ? c->opt.samples_per_pass : std::max<uint64_t>(1, pool / pixels);
  sp = std::min<uint64_t>(sp, s_end - s_begin);
  while (sp > 1 && pixels * sp >= (1ull << 31)) --sp;
  const uint64_t slots = pixels * sp;
  const size_t qb = slots * sizeof(float4);
  DevBuf* qbufs[kPoolStreams] = {&c->qa_o, &c->qa_d, &c->qa_b, &c->qb_o, &c->qb_d, &c->qb_b, &c->env_d, &c->env_b,
                                 &c->d_L, &c->d_hits};
  for (DevBuf* b : qbufs) HIP_TRY(c, b->ensure(qb));
  if (!accum) {
    HIP_TRY(c, c->d_accum.ensure(pixels * sizeof(float4)));
    accum = c->d_accum.as<float4>();
  }
  HIP_TRY(c, c->d_cnt.ensure(kCntWords * sizeof(uint32_t)));
  HIP_TRY(c, c->d_stats.ensure(4 * NPT_MAX_DEPTH * sizeof(unsigned long long)));
  RenderBufs b{c->qa_o.as<float4>(), c->qa_d.as<float4>(), c->qa_b.as<float4>(), c->qb_o.as<float4>(),
               c->qb_d.as<float4>(), c->qb_b.as<float4>(), c->env_d.as<float4>(), c->env_b.as<float4>(),
               c->d_L.as<float4>(), c->d_hits.as<float4>(), accum, c->d_cnt.as<uint32_t>(),
               c->d_stats.as<unsigned long long>()};
  if (c->opt.sort_rays) {
    HIP_TRY(c, c->d_order.ensure(slots * sizeof(uint32_t)));
    b.order = c->d_order.as<uint32_t>();
  }
  unsigned long long* visit_cnt = c->opt.count_visits ? b.stats + 2 * NPT_MAX_DEPTH : nullptr;
  HIP_TRY(c, launch_stats_clear(b.stats, s));
  HIP_TRY(c, hipEventRecord(c->ev0, s));
  const int r = render_passes(c, W, H, s_begin, s_end, max_depth, seed, d_out, s, b, sp, c->opt.kernel_timing != 0,
                              visit_cnt);
  if (r) return r;
  HIP_TRY(c, hipEventRecord(c->ev1, s));
  c->timing_pending = true;
  return ok(c);
}

extern "C" int npt_render(npt_ctx* c, uint32_t W, uint32_t H, uint32_t spp, uint32_t max_depth, uint64_t seed,
                          float* d_out, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    const int r = render_args(c, W, H, spp, max_depth, d_out);
    if (r) return r;
    return render_pooled(c, W, H, 0, spp, max_depth, seed, nullptr, d_out, (hipStream_t)stream);
  });
}

extern "C" int npt_render_samples(npt_ctx* c, uint32_t W, uint32_t H, uint32_t sample0, uint32_t samples,
                                  uint32_t max_depth, uint64_t seed, float* d_sum, float* d_out, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!d_sum) return fail(c, NPT_E_INVALID_ARG, "null running-sum buffer");
    if (reinterpret_cast<uintptr_t>(d_sum) % sizeof(float4))
      return fail(c, NPT_E_INVALID_ARG, "running-sum buffer must be 16-byte aligned");
    if ((uint64_t)sample0 + samples > 0xFFFFFFFFull)
      return fail(c, NPT_E_INVALID_ARG, "sample indices must stay below 2^32");
    // the output is optional here: render_args checks the rest
    const int r = render_args(c, W, H, samples, max_depth, d_out ? d_out : d_sum);
    if (r) return r;
    return render_pooled(c, W, H, sample0, (uint64_t)sample0 + samples, max_depth, seed,
                         reinterpret_cast<float4*>(d_sum), d_out, (hipStream_t)stream);
  });
}

// Byte layout of the fixed scratch for a render of `pixels` pixels with `sp`
// samples per pass: counters, statistics, accumulator, then the ten pool
// streams, each 256-byte aligned.  Returns the bytes used.
static uint64_t noalloc_layout(uint64_t pixels, uint64_t sp, uint64_t off[4 + kPoolStreams]) {
  auto up = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  uint64_t o = 0;
  off[0] = o;  // counters
  o = up(o + kCntWords * sizeof(uint32_t));
  off[1] = o;  // statistics
  o = up(o + 4 * NPT_MAX_DEPTH * sizeof(unsigned long long));
  off[2] = o;  // accumulator
  o = up(o + pixels * sizeof(float4));
  for (int i = 0; i < kPoolStreams; ++i) {
    off[3 + i] = o;
    o = up(o + pixels * sp * sizeof(float4));
  }
  off[3 + kPoolStreams] = o;
  return o;
}

extern "C" int npt_render_noalloc(npt_ctx* c, uint32_t W, uint32_t H, uint32_t spp, uint32_t max_depth,
                                  uint64_t seed, float* d_out, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    int r = render_args(c, W, H, spp, max_depth, d_out);
    if (r) return r;
    if (!c->noalloc_scratch)
      return fail(c, NPT_E_HIP, std::string("no fixed scratch on this device: ") + hipGetErrorString(c->noalloc_status));
    if (c->env_mode == NPT_ENV_NIF && c->nif_layered)
      return fail(c, NPT_E_UNSUPPORTED, "the layer-serial NIF allocates its activations; use a resident shape");
    const uint64_t pixels = (uint64_t)W * H;
    uint64_t off[4 + kPoolStreams];
    if (noalloc_layout(pixels, 1, off) > NPT_NOALLOC_SCRATCH_BYTES)
      return fail(c, NPT_E_INVALID_ARG, "image too large for the fixed render scratch (about 176 bytes per pixel "
                                        "of NPT_NOALLOC_SCRATCH_BYTES)");
    // as many samples per pass as fit (at most the requested option)
    uint64_t sp = 1;
    const uint64_t sp_max = std::min<uint64_t>(spp, c->opt.samples_per_pass ? c->opt.samples_per_pass : spp);
    while (sp < sp_max && pixels * (sp + 1) < (1ull << 31) &&
           noalloc_layout(pixels, sp + 1, off) <= NPT_NOALLOC_SCRATCH_BYTES)
      ++sp;
    noalloc_layout(pixels, sp, off);
    unsigned char* base = static_cast<unsigned char*>(c->noalloc_scratch);
    auto f4 = [&](int i) { return reinterpret_cast<float4*>(base + off[3 + i]); };
    const RenderBufs b{f4(0), f4(1), f4(2), f4(3), f4(4), f4(5), f4(6), f4(7), f4(8), f4(9),
                       reinterpret_cast<float4*>(base + off[2]), reinterpret_cast<uint32_t*>(base + off[0]),
                       reinterpret_cast<unsigned long long*>(base + off[1])};
    HIP_TRY(c, launch_stats_clear(b.stats, (hipStream_t)stream));
    r = render_passes(c, W, H, 0, spp, max_depth, seed, d_out, (hipStream_t)stream, b, sp, false, nullptr);
    if (r) return r;
    c->timing_pending = false;  // no events: the statistics hold paths and passes only
    return ok(c);
  });
}

extern "C" int npt_trace_primary(npt_ctx* c, uint32_t W, uint32_t H, uint32_t sample, uint64_t seed, uint32_t* d_prim,
                                 uint32_t* d_inst, float* d_t, float* d_normal, void* stream) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (c->host_only) return fail(c, NPT_E_NO_DEVICE, "host-only context");
    int r = render_checks(c, W, H);
    if (r) return r;
    r = need_device(c);
    if (r) return r;
    PassView pv{};
    pv.width = W;
    pv.height = H;
    pv.pixels = W * H;
    pv.sample0 = sample;
    pv.samples = 1;
    pv.key0 = (uint32_t)seed;
    pv.key1 = (uint32_t)(seed >> 32);
    HIP_TRY(c, launch_trace_primary(c->stack_depth, scene_view(c), camera_view(c->camera, W, H), pv, d_prim, d_inst,
                                    d_t, d_normal, c->num_cus, (hipStream_t)stream));
    return ok(c);
  });
}

extern "C" int npt_get_stats(npt_ctx* c, npt_stats* out) {
  return guarded(c, [&]() -> int {
    if (!c) return NPT_E_INVALID_ARG;
    if (!out) return fail(c, NPT_E_INVALID_ARG, "null stats");
    if (c->timing_pending) {
      int r = need_device(c);
      if (r) return r;
      HIP_TRY(c, hipEventSynchronize(c->ev1));
      float ms = 0;
      HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
      c->stats.ms_total = ms;
      std::vector<unsigned long long> h(4 * NPT_MAX_DEPTH);
      HIP_TRY(c, hipMemcpy(h.data(), c->d_stats.p, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
      c->stats.env_queries = 0;
      for (int k = 0; k < NPT_MAX_DEPTH; ++k) {
        c->stats.rays[k] = h[k];
        c->stats.escaped[k] = h[NPT_MAX_DEPTH + k];
        c->stats.env_queries += h[NPT_MAX_DEPTH + k];
        c->stats.node_visits[k] = h[2 * NPT_MAX_DEPTH + k];
        c->stats.prim_tests[k] = h[3 * NPT_MAX_DEPTH + k];
      }
      float sum = 0.0f;
      for (size_t i = 0; i + 1 < c->trace_events.size(); i += 2) {
        HIP_TRY(c, hipEventElapsedTime(&ms, c->trace_events[i], c->trace_events[i + 1]));
        sum += ms;
      }
      c->stats.ms_trace = sum;
      c->stats.trace_launches = (uint32_t)(c->trace_events.size() / 2);
      sum = 0.0f;
      for (size_t i = 0; i + 1 < c->shade_events.size(); i += 2) {
        HIP_TRY(c, hipEventElapsedTime(&ms, c->shade_events[i], c->shade_events[i + 1]));
        sum += ms;
      }
      c->stats.ms_shade = sum;
      c->stats.shade_launches = (uint32_t)(c->shade_events.size() / 2);
      sum = 0.0f;
      for (int k = 0; k < NPT_MAX_DEPTH; ++k) c->stats.ms_env_depth[k] = 0.0f;
      for (size_t i = 0; i + 1 < c->env_events.size(); i += 2) {
        HIP_TRY(c, hipEventElapsedTime(&ms, c->env_events[i], c->env_events[i + 1]));
        sum += ms;
        const uint32_t k = c->env_depths[i / 2];
        if (k >= 1 && k <= NPT_MAX_DEPTH) c->stats.ms_env_depth[k - 1] += ms;
      }
      c->stats.ms_env = sum;
      c->stats.env_launches = (uint32_t)(c->env_events.size() / 2);
      c->timing_pending = false;
    }
    *out = c->stats;
    return ok(c);
  });
}
