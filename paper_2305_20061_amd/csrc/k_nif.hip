// k_nif.hip -- HDR-NIF inference on MFMA (Sec. 3.2 network, Sec. 3.3 batched
// queries of escaped rays) and the weight packing it reads.
//
// One workgroup per CU keeps the whole packed network in LDS (FP16/BF16:
// 94 KB); each wave pushes 32-ray column tiles through all layers with
// activations held in registers (see npt_nif_layout.h).  FP32 operands
// (v_mfma_f32_32x32x2f32) keep the 4 hidden 96x96 layers in LDS and read the
// first and last layer from L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "npt.h"
#include "npt_device.h"
#include "npt_kernels.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"
#include "npt_shared.h"

namespace npt {
using namespace nif;

// Bytes of layer l's weight fragments, and their offsets in the packed
// buffer (all layers) and in LDS (the resident layers).
template <int P>
__host__ __device__ constexpr size_t layer_bytes(int l) {
  if (P == NPT_FP8 && fp8_layer(l)) return (size_t)kFp8LayerBytes;
  return (size_t)Geometry<Prec<P>::KPL>::frags(l) * 64 * sizeof(typename Prec<P>::Frag);
}

template <int P>
__host__ __device__ constexpr size_t global_offset(int l) {
  size_t o = 0;
  for (int i = 0; i < l; ++i) o += layer_bytes<P>(i);
  return o;
}

template <int P>
__host__ __device__ constexpr size_t lds_offset(int l) {
  size_t o = 0;
  for (int i = 0; i < l; ++i)
    if (Prec<P>::kResident[i]) o += layer_bytes<P>(i);
  return o;
}

template <int P>
size_t nif_lds_bytes() {
  return lds_offset<P>(kLayers + 1) + (kBiasFloats + kScaleWords) * sizeof(float);
}

// ---------------------------------------------------------------------------
// packing: master FP32 parameters -> MFMA fragments + bias table
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fill_bias(const float* master, float* bias, int tid, int stride) {
  for (int j = tid; j < kBiasFloats; j += stride) {
    float b = 0.0f;
    if (j < kLayers * kHidden) b = master[b_offset(j / kHidden) + j % kHidden];
    else if (j - kLayers * kHidden < kOut) b = master[b_offset(kLayers) + (j - kLayers * kHidden)];
    bias[j] = b;
  }
}

// FP16/BF16/FP32 fragment element i (over all layers) of the packed buffer
template <int KPL>
__device__ __forceinline__ float packed_weight(const float* master, int i) {
  using G = Geometry<KPL>;
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
  return row < layer_out(l) ? master[w_offset(l) + row * layer_in(l) + col] : 0.0f;
}

template <int P>
__global__ void k_nif_pack(const float* master, typename Prec<P>::Elem* frags, float* bias) {
  constexpr int KPL = Prec<P>::KPL;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = tid; i < Geometry<KPL>::kElems; i += gridDim.x * blockDim.x)
    frags[i] = Prec<P>::cvt(packed_weight<KPL>(master, i));
  fill_bias(master, bias, tid, gridDim.x * blockDim.x);
  for (int j = tid; j < kScaleWords; j += gridDim.x * blockDim.x) reinterpret_cast<int*>(bias + kBiasFloats)[j] = 0;
}

// FP8 weight scale: the largest s with m * 2^s <= 448 (0 for m = 0)
__device__ __forceinline__ int fp8_scale_exp(float m) {
  if (!(m > 0.0f)) return 0;
  int e;
  (void)frexpf(m, &e);  // m in [2^(e-1), 2^e)
  int s = 9 - e;
  if (ldexpf(m, s) > 448.0f) s -= 1;
  return s;
}

// FP8 mode: one workgroup of 256 per layer.  Layers 1..4 become E4M3
// fragments of W * 2^s (s from the layer's largest |w|, stored after the
// bias table); layers 0 and 5 FP16 fragments as in FP16 mode.
__global__ __launch_bounds__(256) void k_nif_pack_fp8(const float* master, uint8_t* packed, float* bias) {
  const int l = blockIdx.x;
  __shared__ float red[256];
  int* scales = reinterpret_cast<int*>(bias + kBiasFloats);
  if (fp8_layer(l)) {
    float m = 0.0f;
    for (int i = threadIdx.x; i < kHidden * kHidden; i += 256) m = fmaxf(m, fabsf(master[w_offset(l) + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
      __syncthreads();
    }
    const int s = fp8_scale_exp(red[0]);
    if (threadIdx.x == 0) scales[l] = s;
    int* dst = reinterpret_cast<int*>(packed + global_offset<NPT_FP8>(l));
    // dword wd: fragment q = (M-block, K-block), lane, bytes 4 (wd % 8) .. +3
    for (int wd = threadIdx.x; wd < kFp8LayerBytes / 4; wd += 256) {
      const int q = wd / (64 * 8), lane = (wd / 8) % 64, e0 = (wd % 8) * 4;
      const int mb = q / kKB8, kb = q % kKB8;
      const int row = 32 * mb + lane % 32;
      float v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int col = input_index_fp8(kb, lane / 32, e0 + k);
        v[k] = col < 0 ? 0.0f : ldexpf(master[w_offset(l) + row * kHidden + col], s);
      }
      dst[wd] = pack_e4m3<true>(v[2], v[3], pack_e4m3<false>(v[0], v[1], 0));
    }
  } else {
    using G = Geometry<8>;
    _Float16* dst = reinterpret_cast<_Float16*>(packed + global_offset<NPT_FP8>(l));
    const int base = G::frag_offset(l) * 64 * 8;
    for (int i = threadIdx.x; i < G::frags(l) * 64 * 8; i += 256) dst[i] = (_Float16)packed_weight<8>(master, base + i);
    if (threadIdx.x == 0) scales[l] = 0;
  }
  if (l == 0) {
    fill_bias(master, bias, threadIdx.x, 256);
    for (int j = kLayers + 1 + threadIdx.x; j < kScaleWords; j += 256) scales[j] = 0;
  }
}

// the values the kernel multiplies, back in FP32 (npt_nif_get_dequantized):
// weights rounded as packed, biases unchanged (they are added in FP32)
template <int P>
__global__ void k_nif_dequant(const float* master, const float* bias_tab, float* out, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int l = 0;
    while (l < kLayers && i >= w_offset(l + 1)) ++l;
    const float w = master[i];
    if (i >= b_offset(l)) {
      out[i] = w;
    } else if (P == NPT_FP8 && fp8_layer(l)) {
      const int s = reinterpret_cast<const int*>(bias_tab + kBiasFloats)[l];
      out[i] = ldexpf(__builtin_amdgcn_cvt_f32_fp8(pack_e4m3<false>(ldexpf(w, s), 0.0f, 0), 0), -s);
    } else {
      out[i] = (float)Prec<P>::cvt(w);
    }
  }
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
  ColourMatrix cm;       // network output -> log-space RGB
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

// bias-initialised accumulators of one layer over NT 32-ray column tiles
template <int NT>
__device__ __forceinline__ void init_acc(const float* lb, int h, f32x16 (&acc)[NT][kMB]) {
#pragma unroll
  for (int mb = 0; mb < kMB; ++mb) {
    f32x16 b;
#pragma unroll
    for (int r = 0; r < 16; ++r) b[r] = lb[acc_row(mb, h, r)];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][mb] = b;
  }
}

// acc += W x for Prec<P> operands: x holds the layer input as NKB K-blocks
template <int P, int NT, int NKB>
__device__ __forceinline__ void mma_layer(const typename Prec<P>::Frag* fr, int lane,
                                          const typename Prec<P>::Frag (&x)[NT][Geometry<Prec<P>::KPL>::kKBHidden],
                                          f32x16 (&acc)[NT][kMB]) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) {
      const typename Prec<P>::Frag a = fr[(mb * NKB + kb) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][mb] = Prec<P>::mma(a, x[t][kb], acc[t][mb]);
    }
}

// ReLU of the accumulators into the Prec<P> K-blocks of the next layer
template <int P, int NT>
__device__ __forceinline__ void relu_to_frags(const f32x16 (&acc)[NT][kMB],
                                              typename Prec<P>::Frag (&x)[NT][Geometry<Prec<P>::KPL>::kKBHidden]) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL>;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int kb = 0; kb < G::kKBHidden; ++kb) {
      const int mb = kb / G::kKBPerMB, r0 = (kb % G::kKBPerMB) * KPL;
      if constexpr (KPL == 1) {
        x[t][kb] = fmaxf(acc[t][mb][r0], 0.0f);
      } else if constexpr (std::is_same_v<typename Prec<P>::Elem, _Float16>) {
        // ReLU after the rounding, on packed halves (rounding is monotone
        // and keeps 0, so the result is the same)
        typename Prec<P>::Frag v;
#pragma unroll
        for (int e = 0; e < KPL; ++e) v[e] = (_Float16)acc[t][mb][r0 + e];
        x[t][kb] = __builtin_elementwise_max(v, typename Prec<P>::Frag{});
      } else {
#pragma unroll
        for (int e = 0; e < KPL; ++e) x[t][kb][e] = Prec<P>::cvt(fmaxf(acc[t][mb][r0 + e], 0.0f));
      }
    }
}

// one dense layer + ReLU: x (K-blocks of the layer input) -> x (K-blocks of
// the next layer), weights fr, biases lb
template <int P, int NT, int NKB>
__device__ __forceinline__ void dense_relu(const typename Prec<P>::Frag* fr, const float* lb, int lane, int h,
                                           typename Prec<P>::Frag (&x)[NT][Geometry<Prec<P>::KPL>::kKBHidden]) {
  f32x16 acc[NT][kMB];
  init_acc<NT>(lb, h, acc);
  mma_layer<P, NT, NKB>(fr, lane, x, acc);
  relu_to_frags<P, NT>(acc, x);
}

// FP8 hidden-to-hidden layer: acc += 2^-s (W 2^s) x with E4M3 operands
template <int NT>
__device__ __forceinline__ void mma_layer_e4m3(const i32x8* fr, int lane, int scale_a, const i32x8 (&x)[NT][kKB8],
                                               f32x16 (&acc)[NT][kMB]) {
#pragma unroll
  for (int kb = 0; kb < kKB8; ++kb)
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) {
      const i32x8 a = fr[(mb * kKB8 + kb) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][mb] = mma_e4m3(a, x[t][kb], acc[t][mb], scale_a);
    }
}

__device__ __forceinline__ float relu448(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 448.0f); }

__device__ __forceinline__ int pack4_e4m3(const f32x16& a, int r) {
  return pack_e4m3<true>(relu448(a[r + 2]), relu448(a[r + 3]), pack_e4m3<false>(relu448(a[r]), relu448(a[r + 1]), 0));
}

// ReLU of the accumulators, saturated at 448, into the two E4M3 K-blocks of
// the next layer (byte e of K-block 0: M-block e / 16, register e % 16;
// K-block 1: M-block 2, then zero padding)
template <int NT>
__device__ __forceinline__ void relu_to_e4m3(const f32x16 (&acc)[NT][kMB], i32x8 (&x)[NT][kKB8]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int d = 0; d < 8; ++d) x[t][0][d] = pack4_e4m3(acc[t][d / 4], 4 * (d % 4));
#pragma unroll
    for (int d = 0; d < 4; ++d) x[t][1][d] = pack4_e4m3(acc[t][2], 4 * d);
#pragma unroll
    for (int d = 4; d < 8; ++d) x[t][1][d] = 0;
  }
}

template <int P>
__global__ __launch_bounds__(kNifBlock, 1) void k_nif_infer(const uint8_t* gpack, const float* gbias, NifIO io) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL>;
  using Frag = typename Prec<P>::Frag;
  constexpr bool kAccurate = (P == NPT_FP32);
  constexpr int NT = (P == NPT_FP32) ? 1 : NPT_NIF_TILES;  // 32-ray column tiles per wave
  constexpr int kRays = 32 * NT;
  extern __shared__ float4 smem4[];
  uint8_t* lds = reinterpret_cast<uint8_t*>(smem4);
  float* lbias = reinterpret_cast<float*>(lds + lds_offset<P>(kLayers + 1));
  const int* lscale = reinterpret_cast<const int*>(lbias + kBiasFloats);
  uint64_t n;
  if (io.source == kSrcQueue) n = io.cnt[kCntEnv + io.depth];
  else n = io.n;
  // workgroups without a tile leave before staging the weights
  if ((uint64_t)blockIdx.x * kNifWaves * kRays >= n) return;

  // stage the resident layers, the biases and the FP8 scale exponents
#pragma unroll
  for (int l = 0; l <= kLayers; ++l) {
    if (!Prec<P>::kResident[l]) continue;
    const uint4* src = reinterpret_cast<const uint4*>(gpack + global_offset<P>(l));
    uint4* dst = reinterpret_cast<uint4*>(lds + lds_offset<P>(l));
    for (int i = threadIdx.x; i < (int)(layer_bytes<P>(l) / 16); i += kNifBlock) dst[i] = src[i];
  }
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gbias);
    uint32_t* dst = reinterpret_cast<uint32_t*>(lbias);
    for (int i = threadIdx.x; i < kBiasFloats + kScaleWords; i += kNifBlock) dst[i] = src[i];
  }
  __syncthreads();
  // weights of layer l: from LDS when resident, else from the packed buffer
  auto frags = [&](int l) -> const Frag* {
    return Prec<P>::kResident[l] ? reinterpret_cast<const Frag*>(lds + lds_offset<P>(l))
                                 : reinterpret_cast<const Frag*>(gpack + global_offset<P>(l));
  };

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

    if constexpr (P == NPT_FP8) {
      // layer 0 on FP16 operands, layers 1..4 on E4M3, FP16 input to the output layer
      f32x16 acc[NT][kMB];
      i32x8 x8[NT][kKB8];
      init_acc<NT>(lbias, h, acc);
      mma_layer<P, NT, G::kKBFeat>(frags(0), lane, x, acc);
      relu_to_e4m3<NT>(acc, x8);
#pragma unroll 1
      for (int l = 1; l < kLayers; ++l) {
        init_acc<NT>(lbias + l * kHidden, h, acc);
        mma_layer_e4m3<NT>(reinterpret_cast<const i32x8*>(lds + lds_offset<P>(l)), lane, 127 - lscale[l], x8, acc);
        if (l + 1 < kLayers) relu_to_e4m3<NT>(acc, x8);
      }
      relu_to_frags<P, NT>(acc, x);
    } else {
      // layer 0 (64 -> 96), then 1..4 (96 -> 96, all in LDS)
      dense_relu<P, NT, G::kKBFeat>(frags(0), lbias, lane, h, x);
#pragma unroll 1
      for (int l = 1; l < kLayers; ++l) dense_relu<P, NT, G::kKBHidden>(frags(l), lbias + l * kHidden, lane, h, x);
    }

    // output layer (rows 0..2 of one padded M-block) and the colour matrix
    const Frag* fr = frags(kLayers);
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
        // the fixed colour matrix, in log space
        const float* m = io.cm.m;
        const float y0 = o[t][0], y1 = o[t][1], y2 = o[t][2];
        const float zr = fmaf(m[2], y2, fmaf(m[1], y1, m[0] * y0));
        const float zg = fmaf(m[5], y2, fmaf(m[4], y1, m[3] * y0));
        const float zb = fmaf(m[8], y2, fmaf(m[7], y1, m[6] * y0));
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
    case NPT_FP32: return global_offset<NPT_FP32>(kLayers + 1);
    case NPT_FP16: return global_offset<NPT_FP16>(kLayers + 1);
    case NPT_BF16: return global_offset<NPT_BF16>(kLayers + 1);
    case NPT_FP8: return global_offset<NPT_FP8>(kLayers + 1);
    default: return 0;
  }
}

size_t nif_bias_bytes() { return (kBiasFloats + kScaleWords) * sizeof(float); }

hipError_t launch_nif_pack(int prec, const float* master, void* frags, float* bias, hipStream_t s) {
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_nif_pack<NPT_FP32>, dim3(64), dim3(256), 0, s, master, (float*)frags, bias); break;
    case NPT_FP16: hipLaunchKernelGGL(k_nif_pack<NPT_FP16>, dim3(64), dim3(256), 0, s, master, (_Float16*)frags, bias); break;
    case NPT_BF16: hipLaunchKernelGGL(k_nif_pack<NPT_BF16>, dim3(64), dim3(256), 0, s, master, (__bf16*)frags, bias); break;
    case NPT_FP8: hipLaunchKernelGGL(k_nif_pack_fp8, dim3(kLayers + 1), dim3(256), 0, s, master, (uint8_t*)frags, bias); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nif_dequant(int prec, const float* master, const float* bias, float* out, int n, hipStream_t s) {
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_nif_dequant<NPT_FP32>, dim3(64), dim3(256), 0, s, master, bias, out, n); break;
    case NPT_FP16: hipLaunchKernelGGL(k_nif_dequant<NPT_FP16>, dim3(64), dim3(256), 0, s, master, bias, out, n); break;
    case NPT_BF16: hipLaunchKernelGGL(k_nif_dequant<NPT_BF16>, dim3(64), dim3(256), 0, s, master, bias, out, n); break;
    case NPT_FP8: hipLaunchKernelGGL(k_nif_dequant<NPT_FP8>, dim3(64), dim3(256), 0, s, master, bias, out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_infer_p(const void* frags, const float* bias, const NifIO& io, int grid, hipStream_t s) {
  const size_t lds = nif_lds_bytes<P>();
  hipError_t e = hipFuncSetAttribute((const void*)k_nif_infer<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nif_infer<P>, dim3(grid), dim3(kNifBlock), lds, s, (const uint8_t*)frags, bias, io);
  return hipGetLastError();
}

static hipError_t launch_infer(int prec, const void* frags, const float* bias, const NifIO& io, int grid,
                               hipStream_t s) {
  switch (prec) {
    case NPT_FP32: return launch_infer_p<NPT_FP32>(frags, bias, io, grid, s);
    case NPT_FP16: return launch_infer_p<NPT_FP16>(frags, bias, io, grid, s);
    case NPT_BF16: return launch_infer_p<NPT_BF16>(frags, bias, io, grid, s);
    case NPT_FP8: return launch_infer_p<NPT_FP8>(frags, bias, io, grid, s);
    default: return hipErrorInvalidValue;
  }
}

static int nif_grid(uint64_t n, int num_cus) {
  const uint64_t tiles = (n + 255) / 256;
  return (int)(tiles < 1 ? 1 : (tiles > (uint64_t)num_cus ? num_cus : tiles));
}

hipError_t launch_nif_queue(int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                            const EnvQueue& env, float4* L, const uint32_t* cnt, uint32_t depth, uint64_t max_rays,
                            int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcQueue;
  io.env = env;
  io.L = L;
  io.cnt = cnt;
  io.depth = depth;
  return launch_infer(prec, frags, bias, io, nif_grid(max_rays, num_cus), s);
}

hipError_t launch_nif_dirs(int prec, const void* frags, const float* bias, const ColourMatrix& cm, const float* dirs,
                           uint64_t n, float* rgb, int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcDirs;
  io.dirs = dirs;
  io.out = rgb;
  io.n = n;
  return launch_infer(prec, frags, bias, io, nif_grid(n, num_cus), s);
}

hipError_t launch_nif_grid(int prec, const void* frags, const float* bias, const ColourMatrix& cm, uint32_t gw,
                           uint32_t gh, float* zout, int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcGrid;
  io.gw = gw;
  io.gh = gh;
  io.n = (uint64_t)gw * gh;
  io.out = zout;
  return launch_infer(prec, frags, bias, io, nif_grid(io.n, num_cus), s);
}

}  // namespace npt
