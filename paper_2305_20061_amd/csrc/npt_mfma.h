// npt_mfma.h -- MFMA operand types of the NIF kernels (gfx950).
//   FP32: v_mfma_f32_32x32x2_f32   (1 element per lane per K-block)
//   FP16: v_mfma_f32_32x32x16_f16  (8 elements per lane per K-block)
//   BF16: v_mfma_f32_32x32x16_bf16 (8 elements per lane per K-block)
//   FP8:  the first and output layers as FP16; the hidden-to-hidden layers
//         on v_mfma_scale_f32_32x32x64_f8f6f4 with OCP E4M3 operands (32
//         bytes per lane per K-block of 64)
#pragma once
#include <hip/hip_runtime.h>

#include "npt.h"

namespace npt {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int P>
struct Prec;

template <>
struct Prec<NPT_FP32> {
  static constexpr int KPL = 1;
  using Elem = float;
  using Frag = float;
  static __device__ __forceinline__ f32x16 mma(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Elem cvt(float x) { return x; }
};

template <>
struct Prec<NPT_FP16> {
  static constexpr int KPL = 8;
  using Elem = _Float16;
  using Frag = f16x8;
  static __device__ __forceinline__ f32x16 mma(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Elem cvt(float x) { return (_Float16)x; }
};

template <>
struct Prec<NPT_BF16> {
  static constexpr int KPL = 8;
  using Elem = __bf16;
  using Frag = bf16x8;
  static __device__ __forceinline__ f32x16 mma(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Elem cvt(float x) { return (__bf16)x; }
};

// FP8 mode: FP16 operands for the first and output layers ...
template <>
struct Prec<NPT_FP8> : Prec<NPT_FP16> {};

// ... and E4M3 x E4M3 for the hidden-to-hidden layers.  Lane i + 32h of A
// (rows) and lane j + 32h of B (columns) meet byte by byte; the products are
// scaled by 2^(scale_a - 127) (E8M0 exponent of the A operand; B unscaled)
// and accumulated in FP32.
__device__ __forceinline__ f32x16 mma_e4m3(i32x8 a, i32x8 b, f32x16 c, int scale_a) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, scale_a, 0, 127);
}

// Two values to E4M3 (round to nearest even) in the low or high half of
// `word`; inputs must lie in [-448, 448].
template <bool kHigh>
__device__ __forceinline__ int pack_e4m3(float a, float b, int word) {
  return __builtin_amdgcn_cvt_pk_fp8_f32(a, b, word, kHigh);
}

}  // namespace npt
