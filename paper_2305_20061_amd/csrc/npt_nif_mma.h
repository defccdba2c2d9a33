// npt_nif_mma.h -- register-resident MLP building blocks shared by the
// HDR-NIF inference kernel and the fused training kernel: Fourier features
// straight into MFMA operand fragments, bias-initialised accumulators, one
// layer's MFMAs with weight fragments read from memory (LDS or global), and
// the ReLU that turns a layer's accumulators into the next layer's operands
// (register layout in npt_nif_layout.h).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "npt_device.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"

namespace npt {
namespace nif {

// Fourier feature f (natural order: sin u, cos u, sin v, cos v blocks of NF
// frequencies each; 0 for the padding past the last one) for lane half h,
// which feeds feature f0 (h = 0) or f1 (h = 1): both are compile-time
// constants once the K-block loops unroll, so the frequency, the argument and
// sin / cos become selects between constants
template <class A, bool kAccurateSin>
__device__ __forceinline__ float feature(int f0, int f1, int h, float u, float v) {
  constexpr int NF = A::kFreq;
  const int b0 = f0 / NF, b1 = f1 / NF;
  const float q0 = (float)frequency(f0 - b0 * NF), q1 = (float)frequency(f1 - b1 * NF);
  const bool hi = h != 0;
  const int blk = hi ? b1 : b0;
  const float q = hi ? q1 : q0, x = blk < 2 ? u : v;
  float r;
  if (kAccurateSin) {
    float s, c;
    sincos_turns(frac_product(q, x), s, c);
    r = (blk & 1) ? c : s;
    return (hi ? f1 : f0) < A::kFeat ? r : 0.0f;
  }
  // The hardware sin / cos reduce their argument (in turns) themselves, so
  // the phase needs no wrap into [0, 1): the fraction of the product plus the
  // product's rounding error (recovered with an FMA) lies within an ulp of it.
  const float p = q * x;
  const float ph = __builtin_amdgcn_fractf(p) + __builtin_fmaf(q, x, -p);
  if ((b0 & 1) == (b1 & 1)) {
    r = (b0 & 1) ? __builtin_amdgcn_cosf(ph) : __builtin_amdgcn_sinf(ph);
  } else {
    r = (blk & 1) ? __builtin_amdgcn_cosf(ph) : __builtin_amdgcn_sinf(ph);
  }
  return (hi ? f1 : f0) < A::kFeat ? r : 0.0f;
}

// bias-initialised accumulators (the first NMB M-blocks) of one layer over
// NT 32-ray column tiles
template <int NT, class A, int NMB = A::kMB>
__device__ __forceinline__ void init_acc(const float* lb, int h, f32x16 (&acc)[NT][A::kMB]) {
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb) {
    f32x16 b;
#pragma unroll
    for (int r = 0; r < 16; ++r) b[r] = lb[acc_row(mb, h, r)];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][mb] = b;
  }
}

// acc += W[:, K-blocks KB0 .. KB0+NKB-1] x for Prec<P> operands over the
// first NMB M-blocks; the layer's fragments are [mb][NKBIN][lane]
template <int P, class A, int NT, int NKB, int NKBIN, int KB0, int NMB = A::kMB, int NX>
__device__ __forceinline__ void mma_layer(const typename Prec<P>::Frag* fr, int lane,
                                          const typename Prec<P>::Frag (&x)[NT][NX], f32x16 (&acc)[NT][A::kMB]) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
      const typename Prec<P>::Frag a = fr[(mb * NKBIN + KB0 + kb) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][mb] = Prec<P>::mma(a, x[t][kb], acc[t][mb]);
    }
}

// ReLU of the accumulators into the first NKBX Prec<P> K-blocks of the next
// layer
template <int P, class A, int NT, int NKBX = Geometry<Prec<P>::KPL, A>::kKBHidden>
__device__ __forceinline__ void relu_to_frags(
    const f32x16 (&acc)[NT][A::kMB],
    typename Prec<P>::Frag (&x)[NT][Geometry<Prec<P>::KPL, A>::kKBHidden]) {
  constexpr int KPL = Prec<P>::KPL;
  using G = Geometry<KPL, A>;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int kb = 0; kb < NKBX; ++kb) {
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

}  // namespace nif
}  // namespace npt
