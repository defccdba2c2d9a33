// npt_nif_layout.h -- register/LDS layout of the HDR-NIF MLP on MFMA
// (shared by the inference, packing and training kernels of the library).
//
// Network (Sec. 3.2): 4*NF Fourier features -> L x [dense H + ReLU] -> dense
// 3 -> fixed colour matrix -> expm1; with a skip layer S (Sec. 3.2, the
// paper's own architecture) hidden layer S takes [h ; features], where h is
// the output of layer S - 1, narrowed to H - 4 NF units so that the
// concatenation is H wide.
//
// MFMA 32x32xK (K = 2 for FP32 operands, 16 for FP16/BF16): lane l holds,
// per K-block, KPL = K/2 consecutive k of row/column l % 32 in lane half
// h = l / 32.  The 32x32 FP32 accumulator gives lane l the rows
// 8*(r/4) + 4*h + (r%4), r = 0..15, of column l % 32.
//
// A layer's reduction order is free, so the next layer takes its K-block
// kb directly from accumulator registers: kb -> (M-block mb, registers
// r0..r0+KPL-1); the host-side packing permutes that layer's weight columns
// to match.  Activations therefore stay in registers between layers.
#pragma once
#include <stdint.h>

namespace npt {
namespace nif {

constexpr int kMaxFreq = 16;
constexpr int kOut = 3;
// FP8 weight-scale exponents stored after the bias table (one per layer)
constexpr int kScaleWords = 16;

// Frequencies round(2^((k+1)/2)), k = 0..15.
__host__ __device__ constexpr int frequency(int k) {
  return k == 0 ? 1 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 4 : k == 4 ? 6 : k == 5 ? 8 : k == 6 ? 11
       : k == 7 ? 16 : k == 8 ? 23 : k == 9 ? 32 : k == 10 ? 45 : k == 11 ? 64 : k == 12 ? 91
       : k == 13 ? 128 : k == 14 ? 181 : 256;
}

// Output row held in accumulator register r of lane half h, M-block mb.
__host__ __device__ constexpr int acc_row(int mb, int h, int r) { return 32 * mb + 8 * (r / 4) + 4 * h + (r % 4); }

// One network shape: H hidden units, L hidden layers, skip layer S (0: none),
// NF frequencies.  Parameters are [W_0, b_0, ..., W_L, b_L], W_l row-major
// [out][in].
template <int H, int L, int S, int NF>
struct Arch {
  static_assert(H >= 32 && H % 32 == 0, "hidden width is a multiple of 32");
  static_assert(L >= 1 && L + 1 <= kScaleWords, "layer count");
  static_assert(S == 0 || (S >= 1 && S < L), "skip layer is a hidden layer after the first");
  static_assert(NF >= 1 && NF <= kMaxFreq, "frequency count");
  static_assert(S == 0 || 4 * NF < H, "the layer before a skip-concat keeps some outputs");
  static constexpr int kHidden = H, kLayers = L, kSkip = S, kFreq = NF;
  static constexpr int kFeat = 4 * NF;
  static constexpr int kMB = H / 32;  // M-blocks of a hidden layer
  // outputs of the layer before the skip layer, and its M-blocks
  static constexpr int kNarrow = S != 0 ? H - kFeat : H;
  static constexpr int kMBNarrow = (kNarrow + 31) / 32;
  static constexpr int kBiasFloats = L * H + 32;  // bias table: L x H (zero past a layer's outputs), then 32
  __host__ __device__ static constexpr bool is_skip(int l) { return S != 0 && l == S; }
  __host__ __device__ static constexpr bool is_narrow(int l) { return S != 0 && l + 1 == S; }
  __host__ __device__ static constexpr int layer_in(int l) { return l == 0 ? kFeat : H; }
  __host__ __device__ static constexpr int layer_out(int l) { return l == L ? kOut : is_narrow(l) ? kNarrow : H; }
  // M-blocks a hidden layer computes
  __host__ __device__ static constexpr int mb_out(int l) { return is_narrow(l) ? kMBNarrow : kMB; }
  __host__ __device__ static constexpr int w_offset(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += layer_out(i) * layer_in(i) + layer_out(i);
    return o;
  }
  __host__ __device__ static constexpr int b_offset(int l) { return w_offset(l) + layer_out(l) * layer_in(l); }
  __host__ __device__ static constexpr int params() { return w_offset(L + 1); }
};

// Per-precision MFMA geometry: KPL elements per lane per K-block.  The output
// layer is packed compactly: only its 3 real rows, [kb][h][row] fragments.
template <int KPL, class A>
struct Geometry {
  static constexpr int kKB = 2 * KPL;                           // K per MFMA
  static constexpr int kKBPerMB = 16 / KPL;                     // K-blocks from one 32-row M-block
  static constexpr int kKBFeat = (A::kFeat + kKB - 1) / kKB;    // K-blocks of the features (zero padded)
  static constexpr int kKBHidden = A::kHidden / kKB;            // K-blocks of a hidden activation
  static constexpr int kKBNarrow = A::kMBNarrow * kKBPerMB;     // ... of the narrowed layer's output
  __host__ __device__ static constexpr int kb_in(int l) {
    return l == 0 ? kKBFeat : A::is_skip(l) ? kKBNarrow + kKBFeat : kKBHidden;
  }
  // fragments (64 lanes x KPL elements) of layer l; the output layer's
  // 2 * 3 * kb_in compact fragments of KPL elements count as a fraction
  __host__ __device__ static constexpr int elems(int l) {
    return l == A::kLayers ? kb_in(l) * 2 * 3 * KPL : A::mb_out(l) * kb_in(l) * 64 * KPL;
  }
  __host__ __device__ static constexpr int elem_offset(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += elems(i);
    return o;
  }
  static constexpr int kElems = elem_offset(A::kLayers + 1);
};

// Input index (column of W_l) fed by element e of lane half h in K-block kb,
// or -1 for zero padding.  Features (layer 0, and the K-blocks of a skip
// layer after its hidden input) come in natural order; a skip layer's hidden
// K-blocks hold the narrowed layer's outputs (columns 0 .. kNarrow - 1, rows
// past them padding) and its features columns kNarrow ...
template <int KPL, class A>
__host__ __device__ constexpr int input_index(int l, int kb, int h, int e) {
  using G = Geometry<KPL, A>;
  if (l == 0 || (A::is_skip(l) && kb >= G::kKBNarrow)) {
    const int f = (l == 0 ? kb : kb - G::kKBNarrow) * G::kKB + h * KPL + e;
    return f >= A::kFeat ? -1 : l == 0 ? f : A::kNarrow + f;
  }
  const int mb = kb / G::kKBPerMB;
  const int r = (kb % G::kKBPerMB) * KPL + e;
  const int row = acc_row(mb, h, r);
  return A::is_skip(l) && row >= A::kNarrow ? -1 : row;
}

// FP8 hidden-to-hidden layers (1..L-1) on MFMA 32x32x64: 32 E4M3 values per
// lane per K-block.  Hidden K-block kb holds M-blocks 2kb and 2kb + 1 of the
// previous layer's accumulator (byte e -> M-block 2kb + e / 16, register
// e % 16; zero bytes past the last M-block).  A skip layer has one more
// K-block with the features, in the order in which the FP16 K-blocks of
// layer 0 hold them (byte e -> FP16 K-block e / 8, element e % 8).
template <class A>
struct Fp8 {
  static constexpr int kKBHidden = (A::kMB + 1) / 2;
  static constexpr int kKBNarrow = (A::kMBNarrow + 1) / 2;  // K-blocks of the narrowed layer's output
  __host__ __device__ static constexpr bool layer(int l) { return l >= 1 && l < A::kLayers; }
  __host__ __device__ static constexpr int kb_in(int l) { return A::is_skip(l) ? kKBNarrow + 1 : kKBHidden; }
  __host__ __device__ static constexpr int layer_bytes(int l) { return A::mb_out(l) * kb_in(l) * 64 * 32; }
  __host__ __device__ static constexpr int input_index(int l, int kb, int h, int e) {
    const bool skip = A::is_skip(l);
    if (kb < (skip ? kKBNarrow : kKBHidden)) {
      const int mb = 2 * kb + e / 16;
      if (mb >= (skip ? A::kMBNarrow : A::kMB)) return -1;
      const int row = acc_row(mb, h, e % 16);
      return skip && row >= A::kNarrow ? -1 : row;
    }
    const int kb16 = e / 8;
    const int f = kb16 * 16 + h * 8 + e % 8;
    return (kb16 < Geometry<8, A>::kKBFeat && f < A::kFeat) ? A::kNarrow + f : -1;
  }
};

// Shapes with an LDS-resident inference kernel (any other shape runs on the
// layer-serial GEMM path): the default 16/96/5 network, the paper's network
// (40-d features, H128, four dense-ReLU layers the second of which is
// narrowed to 88 outputs and followed by the features: with the linear output
// layer, five trainable layers and 97.7 KiB in FP16), the same with 64-d
// features, and the small H64 L2 network of the model-size study.
using ArchDefault = Arch<96, 5, 0, 16>;
using ArchH128Skip40 = Arch<128, 4, 2, 10>;
using ArchH128Skip64 = Arch<128, 4, 2, 16>;
using ArchH64 = Arch<64, 2, 0, 16>;
constexpr int kNumArch = 4;

// index of the LDS-resident shape (0 = the default), or -1
inline int resident_arch(int hidden, int layers, int skip, int n_freq) {
  auto is = [&](int H, int L, int S, int NF) { return hidden == H && layers == L && skip == S && n_freq == NF; };
  if (is(96, 5, 0, 16)) return 0;
  if (is(128, 4, 2, 10)) return 1;
  if (is(128, 4, 2, 16)) return 2;
  if (is(64, 2, 0, 16)) return 3;
  return -1;
}

}  // namespace nif
}  // namespace npt
