// npt_nif_layout.h -- register/LDS layout of the HDR-NIF MLP on MFMA
// (shared by the inference, packing and training kernels of the library).
//
// Network (Sec. 3.2): 64 Fourier features -> 5 x [dense 96 + ReLU] -> dense 3
// (YUV) -> fixed YUV->RGB matrix -> expm1.
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

constexpr int kFreq = 16;
constexpr int kFeat = 64;
constexpr int kHidden = 96;
constexpr int kLayers = 5;            // hidden layers
constexpr int kOut = 3;
constexpr int kMB = kHidden / 32;     // M-blocks of a hidden layer
constexpr int kParams = kFeat * kHidden + kHidden + (kLayers - 1) * (kHidden * kHidden + kHidden) +
                        kOut * kHidden + kOut;  // 43,779

// Frequencies round(2^((k+1)/2)), k = 0..15.
__host__ __device__ constexpr int frequency(int k) {
  return k == 0 ? 1 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 4 : k == 4 ? 6 : k == 5 ? 8 : k == 6 ? 11
       : k == 7 ? 16 : k == 8 ? 23 : k == 9 ? 32 : k == 10 ? 45 : k == 11 ? 64 : k == 12 ? 91
       : k == 13 ? 128 : k == 14 ? 181 : 256;
}

// Offsets of W_l and b_l (l = 0..5) in the flat parameter vector.
__host__ __device__ constexpr int layer_in(int l) { return l == 0 ? kFeat : kHidden; }
__host__ __device__ constexpr int layer_out(int l) { return l == kLayers ? kOut : kHidden; }
__host__ __device__ constexpr int w_offset(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += layer_out(i) * layer_in(i) + layer_out(i);
  return o;
}
__host__ __device__ constexpr int b_offset(int l) { return w_offset(l) + layer_out(l) * layer_in(l); }

// Per-precision MFMA geometry: KPL elements per lane per K-block.
template <int KPL>
struct Geometry {
  static constexpr int kKB = 2 * KPL;              // K per MFMA
  static constexpr int kRegsPerKB = KPL;           // accumulator registers feeding one K-block
  static constexpr int kKBPerMB = 16 / KPL;        // K-blocks from one 32-row M-block
  static constexpr int kKBFeat = kFeat / kKB;      // K-blocks of layer 0
  static constexpr int kKBHidden = kHidden / kKB;  // K-blocks of layers 1..5
  // fragments (64 lanes x KPL elements) per layer
  __host__ __device__ static constexpr int frags(int l) {
    return (l == kLayers ? 1 : kMB) * (l == 0 ? kKBFeat : kKBHidden);
  }
  __host__ __device__ static constexpr int frag_offset(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += frags(i);
    return o;
  }
  static constexpr int kFragsTotal = frag_offset(kLayers + 1);
  static constexpr int kElems = kFragsTotal * 64 * KPL;
};

// Input index (column of W_l) fed by element e of lane half h in K-block kb.
template <int KPL>
__host__ __device__ constexpr int input_index(int l, int kb, int h, int e) {
  if (l == 0) return kb * 2 * KPL + h * KPL + e;  // features in natural order
  const int mb = kb / Geometry<KPL>::kKBPerMB;
  const int r = (kb % Geometry<KPL>::kKBPerMB) * KPL + e;
  return 32 * mb + 8 * (r / 4) + 4 * h + (r % 4);
}

// Output row held in accumulator register r of lane half h, M-block mb.
__host__ __device__ constexpr int acc_row(int mb, int h, int r) { return 32 * mb + 8 * (r / 4) + 4 * h + (r % 4); }

// Bias table in LDS: 5 hidden layers x 96, then 32 for the output layer.
// In device memory it is followed by kScaleWords words: the FP8 weight scale
// exponent s of each layer (used by layers 1..4 in FP8 mode).
constexpr int kBiasFloats = kLayers * kHidden + 32;
constexpr int kScaleWords = 8;

// FP8 hidden-to-hidden layers (1..4) on MFMA 32x32x64: 32 E4M3 values per
// lane per K-block; the 96 inputs pad to two K-blocks.  K-block 0 holds
// M-blocks 0 and 1 of the previous layer's accumulator (byte e -> M-block
// e / 16, register e % 16), K-block 1 M-block 2 (bytes 0..15) and 16 zero
// bytes.  Input index fed by byte e of lane half h, or -1 for padding:
constexpr int kKB8 = 2;
constexpr int kFp8Frags = kMB * kKB8;         // A fragments per FP8 layer
constexpr int kFp8LayerBytes = kFp8Frags * 64 * 32;
__host__ __device__ constexpr int input_index_fp8(int kb, int h, int e) {
  return kb == 0 ? acc_row(e / 16, h, e % 16) : (e < 16 ? acc_row(2, h, e) : -1);
}
__host__ __device__ constexpr bool fp8_layer(int l) { return l >= 1 && l < kLayers; }

}  // namespace nif
}  // namespace npt
