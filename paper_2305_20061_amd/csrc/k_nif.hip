// k_nif.hip -- HDR-NIF inference on MFMA (Sec. 3.2 network, Sec. 3.3 batched
// queries of escaped rays) and the weight packing it reads.
//
// One workgroup per CU keeps the whole packed network in LDS (FP16/BF16:
// 94 KB); each wave pushes 32-ray column tiles through all layers with
// activations held in registers (see npt_nif_layout.h).  FP32 operands
// (v_mfma_f32_32x32x2f32) keep the 4 hidden 96x96 layers in LDS and read the
// first and last layer from L2.
#include <hip/hip_runtime.h>

#include "npt.h"
#include "npt_device.h"
#include "npt_kernels.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"
#include "npt_shared.h"

namespace npt {
using namespace nif;

template <int P>
__host__ __device__ constexpr int lds_frag_offset(int l) {
  using G = Geometry<Prec<P>::KPL>;
  int o = 0;
  for (int i = 0; i < l; ++i)
    if (Prec<P>::kResident[i]) o += G::frags(i);
  return o;
}

template <int P>
size_t nif_lds_bytes() {
  return (size_t)lds_frag_offset<P>(kLayers + 1) * 64 * sizeof(typename Prec<P>::Frag) +
         kBiasFloats * sizeof(float);
}

// ---------------------------------------------------------------------------
// packing: master FP32 parameters -> MFMA fragments + bias table
// ---------------------------------------------------------------------------
template <int P>
__global__ void k_nif_pack(const float* master, typename Prec<P>::Elem* frags, float* bias) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL>;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = tid; i < G::kElems; i += gridDim.x * blockDim.x) {
    const int q = i / (64 * KPL);
    const int lane = (i / KPL) % 64;
    const int e = i % KPL;
    int l = 0;
    while (l < kLayers && q >= G::frag_offset(l + 1)) ++l;
    const int local = q - G::frag_offset(l);
    const int nkb = l == 0 ? G::kKBFeat : G::kKBHidden;
    const int mb = local / nkb, kb = local % nkb;
    const int row = 32 * mb + lane % 32;
    const int col = input_index<KPL>(l, kb, lane / 32, e);
    const float w = row < layer_out(l) ? master[w_offset(l) + row * layer_in(l) + col] : 0.0f;
    frags[i] = Prec<P>::cvt(w);
  }
  for (int j = tid; j < kBiasFloats; j += gridDim.x * blockDim.x) {
    float b = 0.0f;
    if (j < kLayers * kHidden) b = master[b_offset(j / kHidden) + j % kHidden];
    else if (j - kLayers * kHidden < kOut) b = master[b_offset(kLayers) + (j - kLayers * kHidden)];
    bias[j] = b;
  }
}

// the weights the kernel multiplies, back in FP32 (npt_nif_get_dequantized)
template <int P>
__global__ void k_nif_dequant(const float* master, float* out, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = (float)Prec<P>::cvt(master[i]);
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
// 8 waves (two per SIMD) x one 32-ray tile per wave measured fastest: the
// second wave hides MFMA/LDS latency; more tiles per wave spill registers.
#ifndef NPT_NIF_WAVES
#define NPT_NIF_WAVES 8
#endif
#ifndef NPT_NIF_TILES
#define NPT_NIF_TILES 1  // 32-ray column tiles per wave for FP16/BF16 operands
#endif
constexpr int kNifWaves = NPT_NIF_WAVES;
constexpr int kNifBlock = 64 * kNifWaves;

enum : int { kSrcQueue = 0, kSrcDirs = 1, kSrcGrid = 2 };

struct NifIO {
  int source;            // kSrc*
  EnvQueue env;          // kSrcQueue
  float4* L;
  const uint32_t* cnt;
  uint32_t depth;
  const float* dirs;     // kSrcDirs: [n][3]
  float* out;            // kSrcDirs: radiance [n][3]; kSrcGrid: log-space RGB [n][3]
  uint64_t n;            // kSrcDirs / kSrcGrid count
  uint32_t gw, gh;       // kSrcGrid
};

template <int P, bool kAccurateSin>
__device__ __forceinline__ float feature(int f, float u, float v) {
  const int blk = f >> 4;
  const float arg = blk < 2 ? u : v;
  const float ph = frac_product((float)frequency(f & 15), arg);
  if (kAccurateSin) {
    float s, c;
    sincos_turns(ph, s, c);
    return (blk & 1) ? c : s;
  }
  return (blk & 1) ? __builtin_amdgcn_cosf(ph) : __builtin_amdgcn_sinf(ph);
}

// one dense layer + ReLU over NT 32-ray column tiles: x (K-blocks of the
// layer input) -> x (K-blocks of the next layer), weights fr, biases lb
template <int P, int NT, int NKB>
__device__ __forceinline__ void dense_relu(const typename Prec<P>::Frag* fr, const float* lb, int lane, int h,
                                           typename Prec<P>::Frag (&x)[NT][Geometry<Prec<P>::KPL>::kKBHidden]) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL>;
  using Frag = typename Prec<P>::Frag;
  f32x16 acc[NT][kMB];
#pragma unroll
  for (int mb = 0; mb < kMB; ++mb) {
    f32x16 b;
#pragma unroll
    for (int r = 0; r < 16; ++r) b[r] = lb[acc_row(mb, h, r)];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][mb] = b;
  }
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) {
      const Frag a = fr[(mb * NKB + kb) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][mb] = Prec<P>::mma(a, x[t][kb], acc[t][mb]);
    }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int kb = 0; kb < G::kKBHidden; ++kb) {
      const int mb = kb / G::kKBPerMB, r0 = (kb % G::kKBPerMB) * KPL;
      if constexpr (KPL == 1) {
        x[t][kb] = fmaxf(acc[t][mb][r0], 0.0f);
      } else {
#pragma unroll
        for (int e = 0; e < KPL; ++e) x[t][kb][e] = Prec<P>::cvt(fmaxf(acc[t][mb][r0 + e], 0.0f));
      }
    }
}

template <int P>
__global__ __launch_bounds__(kNifBlock, 1) void k_nif_infer(const typename Prec<P>::Frag* gfrags,
                                                            const float* gbias, NifIO io) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL>;
  using Frag = typename Prec<P>::Frag;
  constexpr bool kAccurate = (P == NPT_FP32);
  constexpr int NT = (P == NPT_FP32) ? 1 : NPT_NIF_TILES;  // 32-ray column tiles per wave
  constexpr int kRays = 32 * NT;
  extern __shared__ float4 smem4[];
  Frag* lfrags = reinterpret_cast<Frag*>(smem4);
  float* lbias = reinterpret_cast<float*>(lfrags + (size_t)lds_frag_offset<P>(kLayers + 1) * 64);
  uint64_t n;
  if (io.source == kSrcQueue) n = io.cnt[kCntEnv + io.depth];
  else n = io.n;
  // workgroups without a tile leave before staging the weights
  if ((uint64_t)blockIdx.x * kNifWaves * kRays >= n) return;

  // stage the resident layers and the biases
  for (int l = 0; l <= kLayers; ++l) {
    if (!Prec<P>::kResident[l]) continue;
    const Frag* src = gfrags + (size_t)G::frag_offset(l) * 64;
    Frag* dst = lfrags + (size_t)lds_frag_offset<P>(l) * 64;
    for (int i = threadIdx.x; i < G::frags(l) * 64; i += kNifBlock) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < kBiasFloats; i += kNifBlock) lbias[i] = gbias[i];
  __syncthreads();

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int h = lane / 32, col = lane % 32;
  const uint64_t waves_total = (uint64_t)gridDim.x * kNifWaves;

  for (uint64_t tile = (uint64_t)blockIdx.x * kNifWaves + wave; tile * kRays < n; tile += waves_total) {
    float u[NT], v[NT], bx[NT], by[NT], bz[NT];
    uint32_t slot[NT];
    bool valid[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const uint64_t idx = tile * kRays + t * 32 + col;
      valid[t] = idx < n;
      u[t] = 0.5f; v[t] = 0.5f; bx[t] = by[t] = bz[t] = 0.0f; slot[t] = 0;
      if (valid[t]) {
        if (io.source == kSrcGrid) {
          const uint32_t gx = (uint32_t)(idx % io.gw), gy = (uint32_t)(idx / io.gw);
          u[t] = ((float)gx + 0.5f) / (float)io.gw;
          v[t] = ((float)gy + 0.5f) / (float)io.gh;
        } else {
          V3 d;
          if (io.source == kSrcQueue) {
            const float4 ed = io.env.d[idx], eb = io.env.b[idx];
            d = V3{ed.x, ed.y, ed.z};
            slot[t] = __float_as_uint(ed.w);
            bx[t] = eb.x; by[t] = eb.y; bz[t] = eb.z;
          } else {
            d = V3{io.dirs[3 * idx], io.dirs[3 * idx + 1], io.dirs[3 * idx + 2]};
          }
          direction_to_uv(d, u[t], v[t]);
        }
      }
    }

    // layer-0 operands: Fourier features
    Frag x[NT][G::kKBHidden];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int kb = 0; kb < G::kKBFeat; ++kb) {
        if constexpr (KPL == 1) {
          x[t][kb] = feature<P, kAccurate>(input_index<KPL>(0, kb, h, 0), u[t], v[t]);
        } else {
#pragma unroll
          for (int e = 0; e < KPL; ++e)
            x[t][kb][e] = Prec<P>::cvt(feature<P, kAccurate>(input_index<KPL>(0, kb, h, e), u[t], v[t]));
        }
      }

    // hidden layers: layer 0 (64 -> 96), then 1..4 (96 -> 96, all in LDS)
    if constexpr (Prec<P>::kResident[0])
      dense_relu<P, NT, G::kKBFeat>(lfrags + (size_t)lds_frag_offset<P>(0) * 64, lbias, lane, h, x);
    else
      dense_relu<P, NT, G::kKBFeat>(gfrags + (size_t)G::frag_offset(0) * 64, lbias, lane, h, x);
#pragma unroll 1
    for (int l = 1; l < kLayers; ++l)
      dense_relu<P, NT, G::kKBHidden>(lfrags + (size_t)lds_frag_offset<P>(l) * 64, lbias + l * kHidden, lane, h, x);

    // output layer (rows 0..2 of one padded M-block) and the colour matrix
    const Frag* fr;
    if constexpr (Prec<P>::kResident[kLayers]) fr = lfrags + (size_t)lds_frag_offset<P>(kLayers) * 64;
    else fr = gfrags + (size_t)G::frag_offset(kLayers) * 64;
    f32x16 o[NT];
    {
      f32x16 b;
#pragma unroll
      for (int r = 0; r < 16; ++r) b[r] = lbias[kLayers * kHidden + acc_row(0, h, r)];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] = b;
    }
#pragma unroll
    for (int kb = 0; kb < G::kKBHidden; ++kb) {
      const Frag a = fr[kb * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] = Prec<P>::mma(a, x[t][kb], o[t]);
    }
    if (h == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (!valid[t]) continue;
        const float Y = o[t][0], U = o[t][1], V = o[t][2];
        // YUV -> RGB (BT.601 analogue), in log space
        const float zr = Y + 1.13983f * V;
        const float zg = (Y - 0.39465f * U) - 0.58060f * V;
        const float zb = Y + 2.03211f * U;
        const uint64_t idx = tile * kRays + t * 32 + col;
        if (io.source == kSrcGrid) {
          io.out[3 * idx] = zr;
          io.out[3 * idx + 1] = zg;
          io.out[3 * idx + 2] = zb;
          continue;
        }
        const float cr = fmaxf(expm1f(zr), 0.0f), cg = fmaxf(expm1f(zg), 0.0f), cb = fmaxf(expm1f(zb), 0.0f);
        if (io.source == kSrcDirs) {
          io.out[3 * idx] = cr;
          io.out[3 * idx + 1] = cg;
          io.out[3 * idx + 2] = cb;
        } else {
          float4 l = io.L[slot[t]];
          l.x += bx[t] * cr;
          l.y += by[t] * cg;
          l.z += bz[t] * cb;
          io.L[slot[t]] = l;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t nif_packed_bytes(int prec) {
  switch (prec) {
    case NPT_FP32: return (size_t)Geometry<1>::kElems * sizeof(float);
    case NPT_FP16: return (size_t)Geometry<8>::kElems * 2;
    case NPT_BF16: return (size_t)Geometry<8>::kElems * 2;
    default: return 0;
  }
}

hipError_t launch_nif_pack(int prec, const float* master, void* frags, float* bias, hipStream_t s) {
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_nif_pack<NPT_FP32>, dim3(64), dim3(256), 0, s, master, (float*)frags, bias); break;
    case NPT_FP16: hipLaunchKernelGGL(k_nif_pack<NPT_FP16>, dim3(64), dim3(256), 0, s, master, (_Float16*)frags, bias); break;
    case NPT_BF16: hipLaunchKernelGGL(k_nif_pack<NPT_BF16>, dim3(64), dim3(256), 0, s, master, (__bf16*)frags, bias); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nif_dequant(int prec, const float* master, float* out, int n, hipStream_t s) {
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_nif_dequant<NPT_FP32>, dim3(64), dim3(256), 0, s, master, out, n); break;
    case NPT_FP16: hipLaunchKernelGGL(k_nif_dequant<NPT_FP16>, dim3(64), dim3(256), 0, s, master, out, n); break;
    case NPT_BF16: hipLaunchKernelGGL(k_nif_dequant<NPT_BF16>, dim3(64), dim3(256), 0, s, master, out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_infer_p(const void* frags, const float* bias, const NifIO& io, int grid, hipStream_t s) {
  const size_t lds = nif_lds_bytes<P>();
  hipError_t e = hipFuncSetAttribute((const void*)k_nif_infer<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nif_infer<P>, dim3(grid), dim3(kNifBlock), lds, s,
                     (const typename Prec<P>::Frag*)frags, bias, io);
  return hipGetLastError();
}

static hipError_t launch_infer(int prec, const void* frags, const float* bias, const NifIO& io, int grid,
                               hipStream_t s) {
  switch (prec) {
    case NPT_FP32: return launch_infer_p<NPT_FP32>(frags, bias, io, grid, s);
    case NPT_FP16: return launch_infer_p<NPT_FP16>(frags, bias, io, grid, s);
    case NPT_BF16: return launch_infer_p<NPT_BF16>(frags, bias, io, grid, s);
    default: return hipErrorInvalidValue;
  }
}

static int nif_grid(uint64_t n, int num_cus) {
  const uint64_t tiles = (n + 255) / 256;
  return (int)(tiles < 1 ? 1 : (tiles > (uint64_t)num_cus ? num_cus : tiles));
}

hipError_t launch_nif_queue(int prec, const void* frags, const float* bias, const EnvQueue& env, float4* L,
                            const uint32_t* cnt, uint32_t depth, uint64_t max_rays, int num_cus, hipStream_t s) {
  NifIO io{};
  io.source = kSrcQueue;
  io.env = env;
  io.L = L;
  io.cnt = cnt;
  io.depth = depth;
  return launch_infer(prec, frags, bias, io, nif_grid(max_rays, num_cus), s);
}

hipError_t launch_nif_dirs(int prec, const void* frags, const float* bias, const float* dirs, uint64_t n,
                           float* rgb, int num_cus, hipStream_t s) {
  NifIO io{};
  io.source = kSrcDirs;
  io.dirs = dirs;
  io.out = rgb;
  io.n = n;
  return launch_infer(prec, frags, bias, io, nif_grid(n, num_cus), s);
}

hipError_t launch_nif_grid(int prec, const void* frags, const float* bias, uint32_t gw, uint32_t gh,
                           float* zout, int num_cus, hipStream_t s) {
  NifIO io{};
  io.source = kSrcGrid;
  io.gw = gw;
  io.gh = gh;
  io.n = (uint64_t)gw * gh;
  io.out = zout;
  return launch_infer(prec, frags, bias, io, nif_grid(io.n, num_cus), s);
}

}  // namespace npt
