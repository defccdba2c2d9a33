// npt_kernels.h -- host-side launchers of the library's kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "npt_shared.h"

namespace npt {

// k_render.hip
hipError_t launch_pass_init(uint32_t* cnt, uint32_t paths, hipStream_t s);
hipError_t launch_generate(const CameraView& cam, const PassView& pv, const RayQueue& q, float4* L,
                           hipStream_t s);
hipError_t launch_extend(int stack_depth, const SceneView& sc, uint32_t depth, uint64_t max_rays,
                         const RayQueue& in, float4* hits, uint32_t* cnt, unsigned long long* visit_cnt,
                         const uint32_t* order, int num_cus, hipStream_t s);
// every chunk of 1024 queued rays of `depth` sorted into a trace order
// (k_extend's `order`); lo / hi: scene bounds
hipError_t launch_sort_chunks(const RayQueue& in, const uint32_t* cnt, uint32_t depth, uint64_t max_rays,
                              const float lo[3], const float hi[3], uint32_t* order, hipStream_t s);
hipError_t launch_shade(const SceneView& sc, const PassView& pv, uint32_t depth, uint64_t max_rays,
                        const RayQueue& in, const float4* hits, const RayQueue& out, const EnvQueue& env,
                        float4* L, uint32_t* cnt, int num_cus, hipStream_t s);
int trace_stack_size(uint32_t entries);
hipError_t launch_env_lookup(const float4* map, int W, int H, const EnvQueue& env, float4* L,
                             const uint32_t* cnt, uint32_t depth, uint64_t max_rays, int num_cus,
                             hipStream_t s);
hipError_t launch_env_query_map(const float4* map, int W, int H, const float* dirs, uint64_t n, float* rgb,
                                hipStream_t s);
hipError_t launch_accumulate(const float4* L, float4* accum, const PassView& pv, int first_pass,
                             hipStream_t s);
hipError_t launch_finalize(const float4* accum, float* out, uint32_t pixels, float inv_spp, hipStream_t s);
hipError_t launch_trace_primary(int stack_depth, const SceneView& sc, const CameraView& cam,
                                const PassView& pv, uint32_t* prim, uint32_t* inst, float* t, float* normal,
                                int num_cus, hipStream_t s);

// k_scratch.hip: the device address of the fixed scratch array of
// npt_render_noalloc (NPT_NOALLOC_SCRATCH_BYTES) on `device`, which must be
// the current device; looked up on the first call per device
hipError_t noalloc_scratch_ptr(int device, void** ptr);

// k_nif.hip (arch: nif::resident_arch index of the network shape)
size_t nif_packed_bytes(int arch, int prec);
hipError_t launch_nif_pack(int arch, int prec, const float* master, void* frags, float* bias, hipStream_t s);
hipError_t launch_nif_dequant(int arch, int prec, const float* master, const float* bias, float* out, int n,
                              hipStream_t s);
size_t nif_bias_bytes(int arch);
hipError_t launch_nif_queue(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                            const EnvQueue& env, float4* L, const uint32_t* cnt, uint32_t depth, uint64_t max_rays,
                            int num_cus, hipStream_t s);
hipError_t launch_nif_dirs(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                           const float* dirs, uint64_t n, float* rgb, int num_cus, hipStream_t s);
hipError_t launch_nif_grid(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                           uint32_t gw, uint32_t gh, float* zout, int num_cus, hipStream_t s);

}  // namespace npt
