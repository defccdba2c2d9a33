// k_nif.hip -- HDR-NIF inference on MFMA (Sec. 3.2 network, Sec. 3.3 batched
// queries of escaped rays) and the weight packing it reads.
//
// One workgroup per CU keeps the packed network in LDS (the 16/96/5 network
// in FP16/BF16: 87 KB; the paper's H128 skip network with 40-d features:
// 108 KB); each wave pushes 32-ray column tiles through all layers with
// activations held in registers (see npt_nif_layout.h).  Layers that do not
// fit (FP32 operands on v_mfma_f32_32x32x2f32, larger networks) are read
// from L2.  Built for the shapes listed in npt_nif_layout.h.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "npt.h"
#include "npt_device.h"
#include "npt_kernels.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"
#include "npt_nif_mma.h"
#include "npt_shared.h"

namespace npt {
using namespace nif;

// LDS of one workgroup (gfx950: 160 KiB per CU)
constexpr size_t kLdsBudget = 160 * 1024;

// Packed buffer of one network at precision P: every layer's weight
// fragments (E4M3 for the FP8 hidden-to-hidden layers), and which of them the
// inference kernel keeps in LDS.
template <int P, class A>
struct Pack {
  using G = Geometry<Prec<P>::KPL, A>;
  static constexpr int L = A::kLayers;
  __host__ __device__ static constexpr size_t layer_bytes(int l) {
    if (P == NPT_FP8 && Fp8<A>::layer(l)) return (size_t)Fp8<A>::layer_bytes(l);
    return (size_t)G::elems(l) * sizeof(typename Prec<P>::Elem);
  }
  __host__ __device__ static constexpr size_t global_offset(int l) {
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += layer_bytes(i);
    return o;
  }
  static constexpr size_t kBiasBytes = (size_t)(A::kBiasFloats + kScaleWords) * sizeof(float);
  // residency: the hidden layers first, then the first layer, then the
  // output layer, each while it still fits beside the bias table
  __host__ __device__ static constexpr bool resident(int l) {
    size_t used = kBiasBytes;
    for (int j = 0; j <= L; ++j) {
      const int i = j < L - 1 ? j + 1 : j == L - 1 ? 0 : L;
      const bool fits = used + layer_bytes(i) <= kLdsBudget;
      if (fits) used += layer_bytes(i);
      if (i == l) return fits;
    }
    return false;
  }
  __host__ __device__ static constexpr size_t lds_offset(int l) {
    size_t o = 0;
    for (int i = 0; i < l; ++i)
      if (resident(i)) o += layer_bytes(i);
    return o;
  }
  __host__ __device__ static constexpr bool hidden_resident() {
    for (int l = 1; l < L; ++l)
      if (!resident(l)) return false;
    return true;
  }
  static constexpr size_t kLdsBytes = lds_offset(L + 1) + kBiasBytes;
  static_assert(kLdsBytes <= kLdsBudget, "LDS budget");
};

// ---------------------------------------------------------------------------
// packing: master FP32 parameters -> MFMA fragments + bias table
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void fill_bias(const float* master, float* bias, int tid, int stride) {
  constexpr int H = A::kHidden, L = A::kLayers;
  for (int j = tid; j < A::kBiasFloats; j += stride) {
    float b = 0.0f;
    if (j < L * H) {
      if (j % H < A::layer_out(j / H)) b = master[A::b_offset(j / H) + j % H];
    } else if (j - L * H < kOut) {
      b = master[A::b_offset(L) + (j - L * H)];
    }
    bias[j] = b;
  }
}

// element j of layer l's packed fragments (FP16/BF16/FP32 layouts)
template <int KPL, class A>
__device__ __forceinline__ float packed_weight(const float* master, int l, int j) {
  using G = Geometry<KPL, A>;
  const int e = j % KPL;
  int row, kb, h;
  if (l == A::kLayers) {  // compact output layer: [kb][h][row 0..2][e]
    row = (j / KPL) % 3;
    h = (j / (3 * KPL)) % 2;
    kb = j / (6 * KPL);
  } else {  // [mb][kb][lane][e]
    const int lane = (j / KPL) % 64;
    const int q = j / (64 * KPL);
    const int nkb = G::kb_in(l);
    row = 32 * (q / nkb) + lane % 32;
    kb = q % nkb;
    h = lane / 32;
  }
  const int col = input_index<KPL, A>(l, kb, h, e);
  return col < 0 || row >= A::layer_out(l) ? 0.0f : master[A::w_offset(l) + row * A::layer_in(l) + col];
}

template <int P, class A>
__global__ void k_nif_pack(const float* master, typename Prec<P>::Elem* frags, float* bias) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL, A>;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = tid; i < G::kElems; i += gridDim.x * blockDim.x) {
    int l = 0;
    while (l < A::kLayers && i >= G::elem_offset(l + 1)) ++l;
    frags[i] = Prec<P>::cvt(packed_weight<KPL, A>(master, l, i - G::elem_offset(l)));
  }
  fill_bias<A>(master, bias, tid, gridDim.x * blockDim.x);
  for (int j = tid; j < kScaleWords; j += gridDim.x * blockDim.x) reinterpret_cast<int*>(bias + A::kBiasFloats)[j] = 0;
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

// FP8 mode: one workgroup of 256 per layer.  The hidden-to-hidden layers
// become E4M3 fragments of W * 2^s (s from the layer's largest |w|, stored
// after the bias table); the first and output layers FP16 fragments as in
// FP16 mode.
template <class A>
__global__ __launch_bounds__(256) void k_nif_pack_fp8(const float* master, uint8_t* packed, float* bias) {
  using K = Pack<NPT_FP8, A>;
  const int l = blockIdx.x;
  __shared__ float red[256];
  int* scales = reinterpret_cast<int*>(bias + A::kBiasFloats);
  if (Fp8<A>::layer(l)) {
    const int nin = A::layer_in(l), nout = A::layer_out(l), nw = nout * nin;
    float m = 0.0f;
    for (int i = threadIdx.x; i < nw; i += 256) m = fmaxf(m, fabsf(master[A::w_offset(l) + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
      __syncthreads();
    }
    const int s = fp8_scale_exp(red[0]);
    if (threadIdx.x == 0) scales[l] = s;
    int* dst = reinterpret_cast<int*>(packed + K::global_offset(l));
    const int nkb = Fp8<A>::kb_in(l);
    // dword wd: fragment q = (M-block, K-block), half (bytes 0-15 / 16-31 of
    // the lane's 32), lane, bytes 4 (wd % 4) .. +3 of the half: each half is
    // read with a 16-byte lane stride, free of LDS bank conflicts
    for (int wd = threadIdx.x; wd < Fp8<A>::layer_bytes(l) / 4; wd += 256) {
      const int q = wd / (2 * 64 * 4), half = (wd / (64 * 4)) % 2, lane = (wd / 4) % 64;
      const int e0 = half * 16 + (wd % 4) * 4;
      const int mb = q / nkb, kb = q % nkb;
      const int row = 32 * mb + lane % 32;
      float v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int col = Fp8<A>::input_index(l, kb, lane / 32, e0 + k);
        v[k] = col < 0 || row >= nout ? 0.0f : ldexpf(master[A::w_offset(l) + row * nin + col], s);
      }
      dst[wd] = pack_e4m3<true>(v[2], v[3], pack_e4m3<false>(v[0], v[1], 0));
    }
  } else {
    _Float16* dst = reinterpret_cast<_Float16*>(packed + K::global_offset(l));
    for (int j = threadIdx.x; j < Geometry<8, A>::elems(l); j += 256)
      dst[j] = (_Float16)packed_weight<8, A>(master, l, j);
    if (threadIdx.x == 0) scales[l] = 0;
  }
  if (l == 0) {
    fill_bias<A>(master, bias, threadIdx.x, 256);
    for (int j = A::kLayers + 1 + threadIdx.x; j < kScaleWords; j += 256) scales[j] = 0;
  }
}

// the values the kernel multiplies, back in FP32 (npt_nif_get_dequantized):
// weights rounded as packed, biases unchanged (they are added in FP32)
template <int P, class A>
__global__ void k_nif_dequant(const float* master, const float* bias_tab, float* out, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int l = 0;
    while (l < A::kLayers && i >= A::w_offset(l + 1)) ++l;
    const float w = master[i];
    if (i >= A::b_offset(l)) {
      out[i] = w;
    } else if (P == NPT_FP8 && Fp8<A>::layer(l)) {
      const int s = reinterpret_cast<const int*>(bias_tab + A::kBiasFloats)[l];
      out[i] = ldexpf(__builtin_amdgcn_cvt_f32_fp8(pack_e4m3<false>(ldexpf(w, s), 0.0f, 0), 0), -s);
    } else {
      out[i] = (float)Prec<P>::cvt(w);
    }
  }
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
// Waves per workgroup (one workgroup per CU).  The FP8 kernel for networks
// 65 to 96 wide fits in 128 registers once its first- and output-layer
// operands are read inside the tile loop, so NPT_NIF_WAVES_FP8 waves (four
// per SIMD) take turns at the MFMA and VALU work of their tiles: the 16/96/5
// network's queries take 10 % less time than with two waves per SIMD (4-5 %
// less with three; two tiles per wave at two waves per SIMD gain nothing).  The others
// need more registers (the 64-wide FP8 kernel would spill at four waves per
// SIMD; FP16 with one tile per wave at four waves per SIMD is no faster than
// two tiles at two) and run two waves per SIMD, the second one hiding MFMA /
// LDS latency.
#ifndef NPT_NIF_WAVES_FP8
#define NPT_NIF_WAVES_FP8 16
#endif
template <int P, class A>
constexpr int nif_waves() {
  return P == NPT_FP8 && A::kHidden > 64 && A::kHidden <= 96 ? NPT_NIF_WAVES_FP8 : 8;
}
static_assert(NPT_NIF_WAVES_FP8 % 4 == 0 && NPT_NIF_WAVES_FP8 >= 4 && NPT_NIF_WAVES_FP8 <= 16,
              "whole waves per SIMD, at most 1024 threads");

// 32-ray column tiles per wave: two for FP16 / BF16 operands on networks 65
// to 96 wide (each weight fragment read from LDS feeds two MFMAs: 16/96/5
// queries 12-13 % faster, and the same results bit for bit), else one (E4M3
// hidden layers already read half the LDS bytes per MFMA and gain nothing;
// a 64-wide network loses 4 %; 128-wide tiles do not fit twice in registers).
template <int P, class A>
constexpr int nif_tiles() {
  return (P == NPT_FP16 || P == NPT_BF16) && A::kHidden > 64 && A::kHidden <= 96 ? 2 : 1;
}

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

// FP8 layer: acc += 2^-s (W 2^s) x over E4M3 K-blocks KB0 .. KB0+NKB-1 of a
// layer with NKBIN K-blocks, first NMB M-blocks.  A fragment's 32 bytes per
// lane are stored as two halves of 16, each [lane]-contiguous.
template <class A, int NT, int NKB, int NKBIN, int KB0, int NMB = A::kMB, int NX>
__device__ __forceinline__ void mma_layer_e4m3(const i32x8* fr, int lane, int scale_a, const i32x8 (&x)[NT][NX],
                                               f32x16 (&acc)[NT][A::kMB]) {
  const int4* f4 = reinterpret_cast<const int4*>(fr);
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
      const int q = mb * NKBIN + KB0 + kb;
      const int4 lo = f4[(2 * q) * 64 + lane], hi = f4[(2 * q + 1) * 64 + lane];
      const i32x8 a = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][mb] = mma_e4m3(a, x[t][kb], acc[t][mb], scale_a);
    }
}

__device__ __forceinline__ float relu448(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 448.0f); }

// four E4M3 bytes of ReLU'd accumulators; the low conversion's other half
// is overwritten by the high one, so the word it starts from is any register
// (here the first value's bits: no zeroing instruction)
__device__ __forceinline__ int pack4_e4m3(const f32x16& a, int r) {
  const float v0 = relu448(a[r]);
  return pack_e4m3<true>(relu448(a[r + 2]), relu448(a[r + 3]),
                         pack_e4m3<false>(v0, relu448(a[r + 1]), __float_as_int(v0)));
}

// ReLU of the accumulators (the first NMB M-blocks), saturated at 448, into
// the E4M3 K-blocks of the next layer (byte e of K-block kb: M-block
// 2kb + e / 16, register e % 16; zero bytes past M-block NMB - 1)
template <class A, int NT, int NMB = A::kMB>
__device__ __forceinline__ void relu_to_e4m3(const f32x16 (&acc)[NT][A::kMB], i32x8 (&x)[NT][Fp8<A>::kKBHidden]) {
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int kb = 0; kb < (NMB + 1) / 2; ++kb)
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int mb = 2 * kb + d / 4;
        x[t][kb][d] = mb < NMB ? pack4_e4m3(acc[t][mb], 4 * (d % 4)) : 0;
      }
}

template <int P, class A>
__global__ __launch_bounds__((64 * nif_waves<P, A>()), 1) void k_nif_infer(const uint8_t* gpack, const float* gbias,
                                                                           NifIO io) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL, A>;
  using K = Pack<P, A>;
  using Frag = typename Prec<P>::Frag;
  constexpr int L = A::kLayers, H = A::kHidden, MB = A::kMB;
  constexpr bool kAccurate = (P == NPT_FP32);
  constexpr int NT = nif_tiles<P, A>();
  constexpr int kRays = 32 * NT;
  constexpr int kNifWaves = nif_waves<P, A>(), kNifBlock = 64 * kNifWaves;
  extern __shared__ float4 smem4[];
  uint8_t* lds = reinterpret_cast<uint8_t*>(smem4);
  float* lbias = reinterpret_cast<float*>(lds + K::lds_offset(L + 1));
  const int* lscale = reinterpret_cast<const int*>(lbias + A::kBiasFloats);
  uint64_t n;
  if (io.source == kSrcQueue) n = io.cnt[kCntEnv + io.depth];
  else n = io.n;
  // workgroups without a tile leave before staging the weights
  if ((uint64_t)blockIdx.x * kNifWaves * kRays >= n) return;

  // stage the resident layers, the biases and the FP8 scale exponents
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    if (!K::resident(l)) continue;
    const uint4* src = reinterpret_cast<const uint4*>(gpack + K::global_offset(l));
    uint4* dst = reinterpret_cast<uint4*>(lds + K::lds_offset(l));
    for (int i = threadIdx.x; i < (int)(K::layer_bytes(l) / 16); i += kNifBlock) dst[i] = src[i];
  }
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gbias);
    uint32_t* dst = reinterpret_cast<uint32_t*>(lbias);
    for (int i = threadIdx.x; i < A::kBiasFloats + kScaleWords; i += kNifBlock) dst[i] = src[i];
  }
  __syncthreads();
  // weights of the first and output layers (compile-time residency) ...
  const Frag* fr_first = reinterpret_cast<const Frag*>(K::resident(0) ? lds + K::lds_offset(0)
                                                                       : gpack + K::global_offset(0));
  const Frag* fr_out = reinterpret_cast<const Frag*>(K::resident(L) ? lds + K::lds_offset(L)
                                                                     : gpack + K::global_offset(L));
  // ... and of hidden layer l = 1..L-1 (wave-uniform l)
  auto hidden = [&](int l) -> const uint8_t* {
    if constexpr (K::hidden_resident()) {
      uint32_t off = 0;
#pragma unroll
      for (int i = 1; i < L; ++i)
        if (i == l) off = (uint32_t)K::lds_offset(i);
      return lds + off;
    } else {
      const uint8_t* p = gpack;
#pragma unroll
      for (int i = 1; i < L; ++i)
        if (i == l) p = K::resident(i) ? lds + K::lds_offset(i) : gpack + K::global_offset(i);
      return p;
    }
  };

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int h = lane / 32, col = lane % 32;
  const uint64_t waves_total = (uint64_t)gridDim.x * kNifWaves;

  for (uint64_t tile = (uint64_t)blockIdx.x * kNifWaves + wave; tile * kRays < n; tile += waves_total) {
    // Wider networks, two tiles per wave and more than two waves per SIMD:
    // an offset of 0 that the compiler cannot see through (tiles stay far
    // below 2^62) keeps the first- and output-layer operands inside the tile
    // loop; hoisted out of it, they would not fit in the registers and
    // would spill.
    const int z = (H > 96 || NT > 1 || kNifWaves > 8) ? (int)(tile >> 62) : 0;
    const Frag* fr0 = fr_first + z;
    const Frag* fro = fr_out + z;
    const float* lb0 = lbias + 4 * z;  // (4 z keeps its 16-byte alignment visible)
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

    // Fourier features: the first layer's operands, kept for a skip layer
    Frag xf[NT][G::kKBFeat];
    [[maybe_unused]] i32x8 x8f[NT][1];  // FP8 skip layer: the features in E4M3
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int kb = 0; kb < G::kKBFeat; ++kb) {
        if constexpr (KPL == 1) {
          xf[t][kb] = feature<A, kAccurate>(kb * G::kKB, kb * G::kKB + 1, h, u[t], v[t]);
        } else {
          float fv[KPL];
#pragma unroll
          for (int e = 0; e < KPL; ++e) {
            fv[e] = feature<A, kAccurate>(kb * G::kKB + e, kb * G::kKB + KPL + e, h, u[t], v[t]);
            xf[t][kb][e] = Prec<P>::cvt(fv[e]);
          }
          if constexpr (P == NPT_FP8 && A::kSkip != 0) {
            // byte 8 kb + e of the feature K-block, straight from FP32
            x8f[t][0][2 * kb] = pack_e4m3<true>(fv[2], fv[3], pack_e4m3<false>(fv[0], fv[1], 0));
            x8f[t][0][2 * kb + 1] = pack_e4m3<true>(fv[6], fv[7], pack_e4m3<false>(fv[4], fv[5], 0));
          }
        }
      }
    if constexpr (P == NPT_FP8 && A::kSkip != 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int d = 2 * G::kKBFeat; d < 8; ++d) x8f[t][0][d] = 0;
    }

    // With a skip-concat, layer S - 1 computes only the M-blocks of its
    // H - 4 NF outputs, and layer S reads only the K-blocks they fill (the
    // weights of padding rows and columns are zero) followed by the features.
    constexpr int S = A::kSkip, MBN = A::kMBNarrow;
    constexpr int MB0 = A::mb_out(0);
    Frag x[NT][G::kKBHidden];
    f32x16 acc[NT][MB];
    init_acc<NT, A, MB0>(lb0, h, acc);
    mma_layer<P, A, NT, G::kKBFeat, G::kKBFeat, 0, MB0>(fr0, lane, xf, acc);
    if constexpr (P == NPT_FP8) {
      // the first layer on FP16 operands, the hidden-to-hidden layers on
      // E4M3, FP16 input to the output layer
      constexpr int NKB8 = Fp8<A>::kKBHidden, NKB8N = Fp8<A>::kKBNarrow;
      i32x8 x8[NT][NKB8];
      relu_to_e4m3<A, NT, MB0>(acc, x8);
#pragma unroll 1
      for (int l = 1; l < L; ++l) {
        const i32x8* fr = reinterpret_cast<const i32x8*>(hidden(l));
        const int sa = 127 - lscale[l];
        if (S != 0 && l + 1 == S) {
          init_acc<NT, A, MBN>(lbias + l * H, h, acc);
          mma_layer_e4m3<A, NT, NKB8, NKB8, 0, MBN>(fr, lane, sa, x8, acc);
          relu_to_e4m3<A, NT, MBN>(acc, x8);
          continue;
        }
        init_acc<NT, A>(lbias + l * H, h, acc);
        if (S != 0 && l == S) {
          mma_layer_e4m3<A, NT, NKB8N, NKB8N + 1, 0>(fr, lane, sa, x8, acc);
          mma_layer_e4m3<A, NT, 1, NKB8N + 1, NKB8N>(fr, lane, sa, x8f, acc);
        } else {
          mma_layer_e4m3<A, NT, NKB8, NKB8, 0>(fr, lane, sa, x8, acc);
        }
        if (l + 1 < L) relu_to_e4m3<A, NT>(acc, x8);
      }
      relu_to_frags<P, A, NT>(acc, x);
    } else {
      relu_to_frags<P, A, NT, (S == 1 ? G::kKBNarrow : G::kKBHidden)>(acc, x);
#pragma unroll 1
      for (int l = 1; l < L; ++l) {
        const Frag* fr = reinterpret_cast<const Frag*>(hidden(l));
        if (S != 0 && l + 1 == S) {
          init_acc<NT, A, MBN>(lbias + l * H, h, acc);
          mma_layer<P, A, NT, G::kKBHidden, G::kKBHidden, 0, MBN>(fr, lane, x, acc);
          relu_to_frags<P, A, NT, G::kKBNarrow>(acc, x);
          continue;
        }
        init_acc<NT, A>(lbias + l * H, h, acc);
        if (S != 0 && l == S) {
          constexpr int NKBIN = G::kKBNarrow + G::kKBFeat;
          mma_layer<P, A, NT, G::kKBNarrow, NKBIN, 0>(fr, lane, x, acc);
          mma_layer<P, A, NT, G::kKBFeat, NKBIN, G::kKBNarrow>(fr, lane, xf, acc);
        } else {
          mma_layer<P, A, NT, G::kKBHidden, G::kKBHidden, 0>(fr, lane, x, acc);
        }
        relu_to_frags<P, A, NT>(acc, x);
      }
    }

    // output layer: its 3 rows from the compact fragments, zero A rows for
    // the other 29; then the colour matrix
    f32x16 o[NT];
    {
      f32x16 b;
#pragma unroll
      for (int r = 0; r < 16; ++r) b[r] = lb0[L * H + acc_row(0, h, r)];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] = b;
    }
    const bool real_row = col < kOut;
    const int orow = real_row ? col : 0;
#pragma unroll
    for (int kb = 0; kb < G::kKBHidden; ++kb) {
      Frag a = fro[(kb * 2 + h) * 3 + orow];
      if (!real_row) a = Frag{};
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
// host launchers: network shape by index (resident_arch), precision by code
// ---------------------------------------------------------------------------
template <class F>
static auto with_arch(int arch, F&& f) {
  switch (arch) {
    case 1: return f(ArchH128Skip40{});
    case 2: return f(ArchH128Skip64{});
    case 3: return f(ArchH64{});
    default: return f(ArchDefault{});
  }
}

template <int P>
using PrecTag = std::integral_constant<int, P>;

static bool prec_ok(int prec) { return prec >= NPT_FP32 && prec <= NPT_FP8; }
static bool arch_ok(int arch) { return arch >= 0 && arch < kNumArch; }

template <class F>
static auto with_prec(int prec, F&& f) {
  switch (prec) {
    case NPT_FP16: return f(PrecTag<NPT_FP16>{});
    case NPT_BF16: return f(PrecTag<NPT_BF16>{});
    case NPT_FP8: return f(PrecTag<NPT_FP8>{});
    default: return f(PrecTag<NPT_FP32>{});
  }
}

size_t nif_packed_bytes(int arch, int prec) {
  if (!arch_ok(arch) || !prec_ok(prec)) return 0;
  return with_arch(arch, [&](auto a) {
    using A = decltype(a);
    return with_prec(prec, [&](auto p) { return Pack<decltype(p)::value, A>::global_offset(A::kLayers + 1); });
  });
}

size_t nif_bias_bytes(int arch) {
  if (!arch_ok(arch)) return 0;
  return with_arch(arch, [&](auto a) { return (size_t)(decltype(a)::kBiasFloats + kScaleWords) * sizeof(float); });
}

hipError_t launch_nif_pack(int arch, int prec, const float* master, void* frags, float* bias, hipStream_t s) {
  if (!arch_ok(arch) || !prec_ok(prec)) return hipErrorInvalidValue;
  return with_arch(arch, [&](auto a) {
    using A = decltype(a);
    switch (prec) {
      case NPT_FP32: hipLaunchKernelGGL((k_nif_pack<NPT_FP32, A>), dim3(64), dim3(256), 0, s, master, (float*)frags, bias); break;
      case NPT_FP16: hipLaunchKernelGGL((k_nif_pack<NPT_FP16, A>), dim3(64), dim3(256), 0, s, master, (_Float16*)frags, bias); break;
      case NPT_BF16: hipLaunchKernelGGL((k_nif_pack<NPT_BF16, A>), dim3(64), dim3(256), 0, s, master, (__bf16*)frags, bias); break;
      default: hipLaunchKernelGGL((k_nif_pack_fp8<A>), dim3(A::kLayers + 1), dim3(256), 0, s, master, (uint8_t*)frags, bias); break;
    }
    return hipGetLastError();
  });
}

hipError_t launch_nif_dequant(int arch, int prec, const float* master, const float* bias, float* out, int n,
                              hipStream_t s) {
  if (!arch_ok(arch) || !prec_ok(prec)) return hipErrorInvalidValue;
  return with_arch(arch, [&](auto a) {
    using A = decltype(a);
    return with_prec(prec, [&](auto p) {
      hipLaunchKernelGGL((k_nif_dequant<decltype(p)::value, A>), dim3(64), dim3(256), 0, s, master, bias, out, n);
      return hipGetLastError();
    });
  });
}

// one workgroup per CU at most, and no more than the tiles of n_max rays need
static hipError_t launch_infer(int arch, int prec, const void* frags, const float* bias, const NifIO& io,
                               uint64_t n_max, int num_cus, hipStream_t s) {
  if (!arch_ok(arch) || !prec_ok(prec)) return hipErrorInvalidValue;
  return with_arch(arch, [&](auto a) {
    using A = decltype(a);
    return with_prec(prec, [&](auto p) {
      constexpr int P = decltype(p)::value;
      const size_t lds = Pack<P, A>::kLdsBytes;
      hipError_t e = hipFuncSetAttribute((const void*)k_nif_infer<P, A>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      const uint64_t rays = (uint64_t)32 * nif_waves<P, A>() * nif_tiles<P, A>();  // per workgroup round
      const uint64_t need = (n_max + rays - 1) / rays;
      const int grid = (int)(need < 1 ? 1 : (need < (uint64_t)num_cus ? need : (uint64_t)num_cus));
      hipLaunchKernelGGL((k_nif_infer<P, A>), dim3(grid), dim3(64 * nif_waves<P, A>()), lds, s,
                         (const uint8_t*)frags, bias, io);
      return hipGetLastError();
    });
  });
}

hipError_t launch_nif_queue(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                            const EnvQueue& env, float4* L, const uint32_t* cnt, uint32_t depth, uint64_t max_rays,
                            int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcQueue;
  io.env = env;
  io.L = L;
  io.cnt = cnt;
  io.depth = depth;
  return launch_infer(arch, prec, frags, bias, io, max_rays, num_cus, s);
}

hipError_t launch_nif_dirs(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                           const float* dirs, uint64_t n, float* rgb, int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcDirs;
  io.dirs = dirs;
  io.out = rgb;
  io.n = n;
  return launch_infer(arch, prec, frags, bias, io, n, num_cus, s);
}

hipError_t launch_nif_grid(int arch, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                           uint32_t gw, uint32_t gh, float* zout, int num_cus, hipStream_t s) {
  NifIO io{};
  io.cm = cm;
  io.source = kSrcGrid;
  io.gw = gw;
  io.gh = gh;
  io.n = (uint64_t)gw * gh;
  io.out = zout;
  return launch_infer(arch, prec, frags, bias, io, io.n, num_cus, s);
}

}  // namespace npt
