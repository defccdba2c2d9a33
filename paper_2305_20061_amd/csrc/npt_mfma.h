// npt_mfma.h -- MFMA operand types of the NIF kernels (gfx950).
//   FP32: v_mfma_f32_32x32x2_f32   (1 element per lane per K-block)
//   FP16: v_mfma_f32_32x32x16_f16  (8 elements per lane per K-block)
//   BF16: v_mfma_f32_32x32x16_bf16 (8 elements per lane per K-block)
#pragma once
#include <hip/hip_runtime.h>

#include "npt.h"

namespace npt {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
  // inference: which layers live in LDS (FP32 weights do not all fit)
  static constexpr bool kResident[6] = {false, true, true, true, true, false};
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
  static constexpr bool kResident[6] = {true, true, true, true, true, true};
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
  static constexpr bool kResident[6] = {true, true, true, true, true, true};
};

}  // namespace npt
