// k_train_fused.hip -- one HDR-NIF training step (Sec. 3.2.1) in two kernel
// launches, for the network shapes with an LDS-resident inference kernel and
// FP16 GEMM operands (BF16 conversions need more registers than one wave per
// SIMD holds here, and take the layer-by-layer path).
//
// k_train_fused: one workgroup of four waves per 128 samples, one 32-sample
// column tile per wave (one wave per SIMD: every layer's activations stay in
// registers).  Each wave draws its samples and targets, runs the
// forward pass with every layer's input kept in registers as MFMA operand
// fragments (the inference kernel's layout), takes the output layer, colour
// matrix, Huber loss and per-sample gradient on the VALU with FP32 weights,
// and runs the backward-data products on MFMA with transposed weight
// fragments.  A layer's weight gradient sums over samples, which sit across
// lanes in that layout; so per layer the four waves write the gradient at
// the layer's outputs and the layer's inputs, transposed, to LDS, and the
// workgroup forms dW = sum over its 128 samples on MFMA with the samples as
// the reduction dimension, and the bias gradients as row sums.  Each
// workgroup writes its sums (and loss) once.
//
// k_fused_update: the workgroups' sums in a fixed order (deterministic),
// then Adam on the FP32 master weights, which also rewrites both operand
// copies of each weight (forward and transposed fragments) and the head
// table (biases and the output layer, FP32) through position maps built on
// the host.
//
// Rounding points are those of the layer-by-layer path: features, weights
// and post-ReLU activations rounded to the operand format, FP32 sums, the
// output layer in FP32, the loss-scaled gradients at hidden-layer outputs
// rounded to the operand format after the ReLU mask.  The features' sin and
// cos come from the hardware instructions, as in FP16 inference (within an
// FP32 ulp of the accurate ones; the FP16 rounding of a feature moves
// rarely).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "npt.h"
#include "npt_device.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"
#include "npt_nif_mma.h"
#include "npt_train.h"

namespace npt {
using namespace nif;

constexpr int kFusedWaves = 4;
constexpr int kFusedBlock = 64 * kFusedWaves;
constexpr int kFusedSamples = 32 * kFusedWaves;  // samples per workgroup
constexpr int kFusedLd = kFusedSamples + 8;      // row stride (elements) of the transposed LDS operands
constexpr int kUpdateWaves = 8;

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// LDS and pack geometry of one shape (16-bit operands: 8 elements per lane
// per K-block of 16)
template <class A>
struct Fused {
  using G = Geometry<8, A>;
  static constexpr int L = A::kLayers, H = A::kHidden;
  static constexpr int kFeatRows = (A::kFeat + 31) / 32 * 32;
  static constexpr int kRowsIn = kFeatRows > H ? kFeatRows : H;  // rows of XT: a layer's inputs
  static constexpr int kRowsOut = H;                             // rows of GT: gradients at its outputs
  static constexpr size_t kGt = 0;
  static constexpr size_t kXt = kGt + (size_t)kRowsOut * kFusedLd * 2;
  static constexpr size_t kDy = kXt + (size_t)kRowsIn * kFusedLd * 2;  // [3][samples] FP32
  // head table (FP32, copied whole from global memory): the biases [L][H]
  // (zero past a layer's outputs), the output layer's 3 (and padding to 32),
  // the output layer's weights [3][H]; 1 KiB multiple
  static constexpr int kHeadFloats = L * H + 32 + kOut * H;
  static constexpr size_t kHeadBytes = ((size_t)kHeadFloats * 4 + 1023) / 1024 * 1024;
  static constexpr size_t kBias = kDy + (size_t)kOut * kFusedSamples * 4;
  static constexpr size_t kWout = kBias + (size_t)(L * H + 32) * 4;
  static constexpr size_t kRed = kBias + kHeadBytes;                     // per-wave loss
  // forward fragments: layers 0..L-1 as the inference kernel packs them
  static constexpr int kFElems = G::elem_offset(L);
  // transposed fragments of hidden layer l = 1..L-1: [mi][kb][lane][8],
  // mi over the M-blocks of layer l - 1's outputs (rows: layer l's hidden
  // inputs in natural order), kb over the K-blocks of layer l's outputs in
  // the accumulator order of its gradient
  __host__ __device__ static constexpr int t_kb(int l) { return 2 * A::mb_out(l); }
  __host__ __device__ static constexpr int t_elems(int l) {
    return l >= 1 && l < L ? A::mb_out(l - 1) * t_kb(l) * 64 * 8 : 0;
  }
  __host__ __device__ static constexpr int t_offset(int l) {
    int o = 0;
    for (int i = 1; i < l; ++i) o += t_elems(i);
    return o;
  }
  static constexpr int kTElems = t_offset(L);
  // two staging buffers for one layer's weight fragments (forward or
  // transposed): the next layer's are loaded while this one's are used
  __host__ __device__ static constexpr int stage_bytes() {
    int m = 0;
    for (int l = 0; l < L; ++l) {
      m = G::elems(l) * 2 > m ? G::elems(l) * 2 : m;
      m = t_elems(l) * 2 > m ? t_elems(l) * 2 : m;
    }
    return m;
  }
  static constexpr int kStageBytes = stage_bytes();
  // most weight-gradient tiles of one layer that one wave computes
  __host__ __device__ static constexpr int max_tiles() {
    int m = 0;
    for (int l = 0; l < L; ++l) {
      const int t = (A::mb_out(l) * ((A::layer_in(l) + 31) / 32) + kFusedWaves - 1) / kFusedWaves;
      m = t > m ? t : m;
    }
    return m;
  }
  static constexpr int kMaxTiles = max_tiles();
  static constexpr size_t kStage = (kRed + kFusedWaves * 4 + 15) / 16 * 16;
  static constexpr size_t kLdsBytes = kStage + 2 * (size_t)kStageBytes;
  static_assert(kLdsBytes <= 160 * 1024, "LDS budget");
  // 16-byte chunks of the staging copy per thread
};

// One layer's weight fragments (a multiple of 1 KiB) from global memory
// into an LDS staging buffer with the LDS-direct loads of gfx950
// (global_load_lds_dwordx4: lane i's 16 bytes land at the wave's LDS
// address + 16 i), 1 KiB per wave and instruction, no registers involved;
// stage_wait() (all of this wave's loads done) and a barrier publish them.
__device__ __forceinline__ void stage_issue(const uint8_t* src, uint8_t* dst, int bytes, int wave, int lane) {
  for (int c = wave; c < bytes / 1024; c += kFusedWaves)
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + c * 1024 + lane * 16),
                                     (__attribute__((address_space(3))) void*)(dst + c * 1024), 16, 0, 0);
}
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Position, among a wave's 32 slots of a transposed LDS row, of the wave's
// sample s: put_transposed() writes samples in the accumulator's row order
// (slot 16 g + 8 h + e holds sample 16 g + 8 (e / 4) + 4 h + e % 4), the same
// for every row, so sums over slots pair the same samples.
__device__ __forceinline__ int transposed_slot(int s) {
  return 16 * (s / 16) + 8 * ((s % 8) / 4) + 4 * ((s % 16) / 8) + s % 4;
}

// One or two K-block fragments of the wave's 32 samples (as an MFMA A
// operand: lane = sample, element = one of 16 positions along K) turned
// around by MFMAs against identity selections (idlo: position k -> column k,
// idhi: -> column 16 + k; exact), so that lane = column = one position and
// its registers = the 32 samples; each lane then writes its 16 samples as
// two 16-byte runs into row `row` (< 0: nothing) of an LDS [row][sample]
// array.  Sixteen-bit scattered writes would take eight times the LDS
// instructions.
template <int P>
__device__ __forceinline__ void put_transposed(const typename Prec<P>::Frag& fa, const typename Prec<P>::Frag* fb,
                                               const typename Prec<P>::Frag& idlo, const typename Prec<P>::Frag& idhi,
                                               typename Prec<P>::Elem* base, int row, int wave, int h) {
  using Frag = typename Prec<P>::Frag;
  f32x16 c = Prec<P>::mma(fa, idlo, f32x16{});
  if (fb) c = Prec<P>::mma(*fb, idhi, c);
  Frag r0, r1;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    r0[e] = Prec<P>::cvt(c[e]);
    r1[e] = Prec<P>::cvt(c[8 + e]);
  }
  if (row >= 0) {
    *reinterpret_cast<Frag*>(base + row * kFusedLd + wave * 32 + 8 * h) = r0;
    *reinterpret_cast<Frag*>(base + row * kFusedLd + wave * 32 + 16 + 8 * h) = r1;
  }
}

struct FusedStep {
  const void* fpack;
  const void* tpack;
  const float* head;  // head table (Fused<A>::kHeadBytes)
  const float4* map;
  uint32_t map_w, map_h;
  uint32_t key0, key1, step;
  float delta, loss_scale;
  ColourMatrix cm;
  float* partial;    // [workgroups][ld]: gradient sums (loss-scaled) of np parameters
  float* loss_part;  // [workgroups]: loss sums
  int64_t np, ld;    // ld: np rounded up to a multiple of 256
};

template <int P, class A>
__global__ __launch_bounds__(kFusedBlock, 1) void k_train_fused(FusedStep a) {
  using K = Fused<A>;
  using G = Geometry<8, A>;
  using Frag = typename Prec<P>::Frag;
  using Elem = typename Prec<P>::Elem;
  constexpr int L = A::kLayers, H = A::kHidden, MB = A::kMB;
  constexpr int KBH = G::kKBHidden, KBF = G::kKBFeat, KBN = G::kKBNarrow;
  constexpr int LD = kFusedLd, NS = kFusedSamples;
  extern __shared__ float4 smem4[];
  uint8_t* lds = reinterpret_cast<uint8_t*>(smem4);
  Elem* gt = reinterpret_cast<Elem*>(lds + K::kGt);
  Elem* xt = reinterpret_cast<Elem*>(lds + K::kXt);
  float* dyl = reinterpret_cast<float*>(lds + K::kDy);
  float* lbias = reinterpret_cast<float*>(lds + K::kBias);
  float* lwout = reinterpret_cast<float*>(lds + K::kWout);
  float* lred = reinterpret_cast<float*>(lds + K::kRed);
  uint8_t* stage[2] = {lds + K::kStage, lds + K::kStage + K::kStageBytes};
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, h = lane / 32, col = lane % 32;
  const int sl = wave * 32 + col;  // this lane's sample within the workgroup
  // identity selections for put_transposed
  typename Prec<P>::Frag idlo, idhi;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    idlo[e] = Prec<P>::cvt(8 * h + e == col ? 1.0f : 0.0f);
    idhi[e] = Prec<P>::cvt(8 * h + e == col - 16 ? 1.0f : 0.0f);
  }
  // row of the transposed block for this lane's column: position k of
  // K-block kb of a layer-l input (or of a hidden layer's outputs: l = L
  // reads them as the output layer's inputs)
  auto in_row = [&](int l, int kb, int k) { return input_index<8, A>(l, kb, k / 8, k % 8); };
  auto pair_row = [&](int l, int kba, int kbb, int nkb) {
    return col < 16 ? in_row(l, kba, col) : kbb < nkb ? in_row(l, kbb, col - 16) : -1;
  };
  float* part = a.partial + (size_t)blockIdx.x * (size_t)a.ld;

  // the head table (biases and the output layer in FP32) into LDS
  stage_issue(static_cast<const uint8_t*>(static_cast<const void*>(a.head)), lds + K::kBias, (int)K::kHeadBytes,
              wave, lane);

  // layer 0's forward fragments into the first staging buffer
  const uint8_t* fpb = static_cast<const uint8_t*>(a.fpack);
  const uint8_t* tpb = static_cast<const uint8_t*>(a.tpack);
  stage_issue(fpb, stage[0], G::elems(0) * 2, wave, lane);

  // the sample: (u, v) from the training stream, its target, its features
  const uint32_t bidx = blockIdx.x * NS + sl;
  const U4 rnd = philox(bidx, a.step, 0, kRngTrain, a.key0, a.key1);
  const float u = unit_float(rnd.x), v = unit_float(rnd.y);
  const float3 c3 = env_bilinear(a.map, (int)a.map_w, (int)a.map_h, u, v);
  const float tg[3] = {log1pf(c3.x), log1pf(c3.y), log1pf(c3.z)};
  Frag xf[1][KBF];
#pragma unroll
  for (int kb = 0; kb < KBF; ++kb)
#pragma unroll
    for (int e = 0; e < 8; ++e) xf[0][kb][e] = Prec<P>::cvt(feature<A, false>(kb * 16 + e, kb * 16 + 8 + e, h, u, v));
  stage_wait();
  __syncthreads();

  // forward: xh[l] = the output of hidden layer l (the hidden part of layer
  // l + 1's input), kept for the backward pass
  // (layer l's fragments in stage[l % 2]; the next layer's, or the last
  // hidden layer's transposed ones, are loaded meanwhile)
  Frag xh[L][1][KBH];
  f32x16 acc[1][MB];
  static_for<0, L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int nmb = A::mb_out(l);
    if constexpr (l + 1 < L) stage_issue(fpb + G::elem_offset(l + 1) * 2, stage[(l + 1) % 2], G::elems(l + 1) * 2, wave, lane);
    else if constexpr (L >= 2) stage_issue(tpb + K::t_offset(L - 1) * 2, stage[(l + 1) % 2], K::t_elems(L - 1) * 2, wave, lane);
    const Frag* fr = reinterpret_cast<const Frag*>(stage[l % 2]);
    init_acc<1, A, nmb>(lbias + l * H, h, acc);
    if constexpr (l == 0) {
      mma_layer<P, A, 1, KBF, KBF, 0, nmb>(fr, lane, xf, acc);
    } else if constexpr (A::is_skip(l)) {
      mma_layer<P, A, 1, KBN, KBN + KBF, 0, nmb>(fr, lane, xh[l - 1], acc);
      mma_layer<P, A, 1, KBF, KBN + KBF, KBN, nmb>(fr, lane, xf, acc);
    } else {
      mma_layer<P, A, 1, KBH, KBH, 0, nmb>(fr, lane, xh[l - 1], acc);
    }
    relu_to_frags<P, A, 1, 2 * nmb>(acc, xh[l]);
    stage_wait();
    __syncthreads();
  });

  // output layer (FP32 weights) over this lane's half of the last hidden
  // layer's outputs, summed with the other half's lane
  constexpr int KBL = 2 * A::mb_out(L - 1);
  // (registers 4q .. 4q + 3 of an M-block hold four consecutive rows: one
  // 16-byte LDS read per output and group of four)
  float y[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < KBL; ++kb)
#pragma unroll
    for (int e0 = 0; e0 < 8; e0 += 4) {
      const int row0 = acc_row(kb / 2, h, (kb % 2) * 8 + e0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float4 w = *reinterpret_cast<const float4*>(lwout + j * H + row0);
        const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) y[j] = fmaf(wv[e], (float)xh[L - 1][0][kb][e0 + e], y[j]);
      }
    }
#pragma unroll
  for (int j = 0; j < 3; ++j) y[j] = lbias[L * H + j] + (y[j] + __shfl_xor(y[j], 32));
  // colour matrix, Huber loss and its gradient (loss-scaled), back through
  // the colour matrix: dy = M^T g
  const float* m = a.cm.m;
  const float z[3] = {fmaf(m[2], y[2], fmaf(m[1], y[1], m[0] * y[0])),
                      fmaf(m[5], y[2], fmaf(m[4], y[1], m[3] * y[0])),
                      fmaf(m[8], y[2], fmaf(m[7], y[1], m[6] * y[0]))};
  float loss = 0.0f, g3[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float e = z[k] - tg[k];
    const float ae = fabsf(e);
    loss += ae <= a.delta ? 0.5f * e * e : a.delta * (ae - 0.5f * a.delta);
    g3[k] = (ae <= a.delta ? e : copysignf(a.delta, e)) * a.loss_scale;
  }
  const float dy0 = fmaf(m[6], g3[2], fmaf(m[3], g3[1], m[0] * g3[0]));
  const float dy1 = fmaf(m[7], g3[2], fmaf(m[4], g3[1], m[1] * g3[0]));
  const float dy2 = fmaf(m[8], g3[2], fmaf(m[5], g3[1], m[2] * g3[0]));
  // the workgroup's loss: lanes of half 0 carry one sample each
  float ls = h == 0 ? loss : 0.0f;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
  if (lane == 0) lred[wave] = ls;
  if (h == 0) {
    const int ds = wave * 32 + transposed_slot(col);
    dyl[ds] = dy0;
    dyl[NS + ds] = dy1;
    dyl[2 * NS + ds] = dy2;
  }
  // gradient at the last hidden layer's outputs (masked by its ReLU,
  // rounded), and that layer's outputs, transposed, for the output layer's
  // weight gradient
  Frag gc[1][KBH];
#pragma unroll
  for (int kb = 0; kb < KBL; ++kb)
#pragma unroll
    for (int e0 = 0; e0 < 8; e0 += 4) {
      const int row0 = acc_row(kb / 2, h, (kb % 2) * 8 + e0);
      const float4 w0 = *reinterpret_cast<const float4*>(lwout + row0);
      const float4 w1 = *reinterpret_cast<const float4*>(lwout + H + row0);
      const float4 w2 = *reinterpret_cast<const float4*>(lwout + 2 * H + row0);
      const float a0[4] = {w0.x, w0.y, w0.z, w0.w}, a1[4] = {w1.x, w1.y, w1.z, w1.w};
      const float a2[4] = {w2.x, w2.y, w2.z, w2.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float gv = fmaf(dy2, a2[e], fmaf(dy1, a1[e], dy0 * a0[e]));
        const Elem xe = xh[L - 1][0][kb][e0 + e];
        gc[0][kb][e0 + e] = xe > Elem{} ? Prec<P>::cvt(gv) : Elem{};
      }
    }
#pragma unroll
  for (int kb = 0; kb < KBL; kb += 2)
    put_transposed<P>(xh[L - 1][0][kb], kb + 1 < KBL ? &xh[L - 1][0][kb + 1] : nullptr, idlo, idhi, xt,
                      pair_row(L, kb, kb + 1, KBL), wave, h);
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int w = 0; w < kFusedWaves; ++w) s += lred[w];
    a.loss_part[blockIdx.x] = s;
  }
  // output layer: dW = sum over samples of dy x^T, db = sum of dy
  for (int idx = threadIdx.x; idx < kOut * H + kOut; idx += kFusedBlock) {
    const bool wgt = idx < kOut * H;
    const int j = wgt ? idx / H : idx - kOut * H, q = wgt ? idx % H : 0;
    const float4* d4 = reinterpret_cast<const float4*>(dyl + j * NS);
    const uint4* x4 = reinterpret_cast<const uint4*>(xt + q * LD);
    float s = 0.0f;
    for (int k = 0; k < NS / 8; ++k) {
      const float4 da = d4[2 * k], db = d4[2 * k + 1];
      const float dv[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
      if (wgt) {
        const uint4 xr = x4[k];
        const Elem* xe = reinterpret_cast<const Elem*>(&xr);
#pragma unroll
        for (int i = 0; i < 8; ++i) s = fmaf(dv[i], (float)xe[i], s);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) s += dv[i];
      }
    }
    part[(wgt ? A::w_offset(L) : A::b_offset(L)) + (wgt ? idx : j)] = s;
  }
  __syncthreads();

  // Weight-gradient tiles and bias sums of a layer are held in registers
  // and written out during the next layer's phase, after its first barrier:
  // a wait for the staging loads (which counts every outstanding memory
  // operation) then no longer waits for these stores as well.
  constexpr int KT = K::kMaxTiles;
  f32x16 keep[KT];
  float bkeep = 0.0f;
  auto flush = [&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int ntn = (A::layer_in(l) + 31) / 32, ntiles = A::mb_out(l) * ntn;
    constexpr int nin = A::layer_in(l), nout = A::layer_out(l);
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      const int tile = wave + i * kFusedWaves;
      const int mt = tile / ntn, in = 32 * (tile % ntn) + col;
      if (tile < ntiles && in < nin)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int out = acc_row(mt, h, r);
          if (out < nout) part[A::w_offset(l) + out * nin + in] = keep[i][r];
        }
    }
    const int row = kFusedBlock - 1 - (int)threadIdx.x;
    if (row < nout) part[A::b_offset(l) + row] = bkeep;
  };

  // hidden layers, last to first (layer l's transposed fragments in
  // stage[(2 L - 1 - l) % 2], the next layer's loaded meanwhile)
  static_for<0, L>([&](auto ic) {
    constexpr int l = L - 1 - decltype(ic)::value;
    constexpr int kbo = 2 * A::mb_out(l);  // K-blocks of the gradient at layer l's outputs
    constexpr int cur = (2 * L - 1 - l) % 2;
    if constexpr (l >= 2) stage_issue(tpb + K::t_offset(l - 1) * 2, stage[cur ^ 1], K::t_elems(l - 1) * 2, wave, lane);
    // the transposed operands of dW_l: gradient rows (layer l's outputs) and
    // input rows (natural column order of W_l)
    // (gradient K-block pairs hold the rows of one M-block of layer l's
    // outputs: the input rows of layer l + 1, or of the output layer)
#pragma unroll
    for (int kb = 0; kb < kbo; kb += 2)
      put_transposed<P>(gc[0][kb], &gc[0][kb + 1], idlo, idhi, gt, pair_row(L, kb, kb + 1, kbo), wave, h);
    if constexpr (l == 0) {
#pragma unroll
      for (int kb = 0; kb < KBF; kb += 2)
        put_transposed<P>(xf[0][kb], kb + 1 < KBF ? &xf[0][kb + 1] : nullptr, idlo, idhi, xt,
                          pair_row(0, kb, kb + 1, KBF), wave, h);
      // rows between the last feature and the tile edge
      constexpr int z0 = A::kFeat, nz = K::kFeatRows - z0;
      for (int i = threadIdx.x; i < nz * NS; i += kFusedBlock) xt[(z0 + i / NS) * LD + i % NS] = Elem{};
    } else if constexpr (A::is_skip(l)) {
#pragma unroll
      for (int kb = 0; kb < KBN; kb += 2)
        put_transposed<P>(xh[l - 1][0][kb], kb + 1 < KBN ? &xh[l - 1][0][kb + 1] : nullptr, idlo, idhi, xt,
                          pair_row(l, kb, kb + 1, KBN), wave, h);
#pragma unroll
      for (int kb = 0; kb < KBF; kb += 2)
        put_transposed<P>(xf[0][kb], kb + 1 < KBF ? &xf[0][kb + 1] : nullptr, idlo, idhi, xt,
                          pair_row(l, KBN + kb, KBN + kb + 1, KBN + KBF), wave, h);
    } else {
#pragma unroll
      for (int kb = 0; kb < KBH; kb += 2)
        put_transposed<P>(xh[l - 1][0][kb], &xh[l - 1][0][kb + 1], idlo, idhi, xt, pair_row(l, kb, kb + 1, KBH),
                          wave, h);
    }
    // backward data: the gradient at layer l - 1's outputs, W_l^T g masked
    // by their ReLU and rounded
    Frag gn[1][KBH];
    if constexpr (l >= 1) {
      constexpr int mbi = A::mb_out(l - 1);
      f32x16 accb[1][MB];
#pragma unroll
      for (int mi = 0; mi < mbi; ++mi) accb[0][mi] = f32x16{};
      mma_layer<P, A, 1, kbo, kbo, 0, mbi>(reinterpret_cast<const Frag*>(stage[cur]), lane, gc, accb);
#pragma unroll
      for (int kb = 0; kb < 2 * mbi; ++kb)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float gv = accb[0][kb / 2][(kb % 2) * 8 + e];
          gn[0][kb][e] = xh[l - 1][0][kb][e] > Elem{} ? Prec<P>::cvt(gv) : Elem{};
        }
    }
    stage_wait();
    __syncthreads();
    if constexpr (l + 1 < L) flush(std::integral_constant<int, l + 1>{});
    // dW_l = sum over the workgroup's samples of g x^T, 32 x 32 tiles on
    // MFMA with the samples as K; db_l = row sums of g
    constexpr int ntn = (A::layer_in(l) + 31) / 32, ntiles = A::mb_out(l) * ntn;
    // (the wave's tiles share each K-block step: independent accumulators
    // in flight one after another)
    constexpr int mytiles_max = (ntiles + kFusedWaves - 1) / kFusedWaves;
    const Elem* ga[mytiles_max];
    const Elem* xb[mytiles_max];
#pragma unroll
    for (int i = 0; i < mytiles_max; ++i) {
      const int tile = min(wave + i * kFusedWaves, ntiles - 1);  // a wave past the end repeats the last tile
      ga[i] = gt + (32 * (tile / ntn) + col) * LD + 8 * h;
      xb[i] = xt + (32 * (tile % ntn) + col) * LD + 8 * h;
      keep[i] = f32x16{};
    }
#pragma unroll 2
    for (int kb = 0; kb < NS / 16; ++kb)
#pragma unroll
      for (int i = 0; i < mytiles_max; ++i)
        keep[i] = Prec<P>::mma(*reinterpret_cast<const Frag*>(ga[i] + 16 * kb),
                               *reinterpret_cast<const Frag*>(xb[i] + 16 * kb), keep[i]);
    {
      const int row = kFusedBlock - 1 - (int)threadIdx.x;  // the last waves, which hold the fewest tiles
      if (row < A::layer_out(l)) {
        // pairs of FP16 values summed into FP32 by the dot-product unit
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        const h2 ones = {(_Float16)1.0f, (_Float16)1.0f};
        const h2* g2 = reinterpret_cast<const h2*>(gt + row * LD);
        float s = 0.0f;
#pragma unroll 8
        for (int k = 0; k < NS / 2; ++k) s = __builtin_amdgcn_fdot2(g2[k], ones, s, false);
        bkeep = s;
      }
    }
    __syncthreads();
    if constexpr (l >= 1) {
#pragma unroll
      for (int kb = 0; kb < KBH; ++kb) gc[0][kb] = gn[0][kb];
    }
  });
  flush(std::integral_constant<int, 0>{});
}

// Stochastic rounding to binary16 (FP16 master weights, Sec. 3.2.1; Gupta
// et al. 2015), as in the layer-by-layer path's Adam
__device__ __forceinline__ float fp16_round_stochastic(float x, float u) {
  const float ax = fabsf(x);
  if (ax == 0.0f || ax != ax) return x;
  if (ax >= 65504.0f) return copysignf(65504.0f, x);
  const int e = max(ilogbf(ax), -14);
  const float q = ldexpf(1.0f, e - 10);
  const float lo = floorf(ax / q) * q;
  return copysignf(u < (ax - lo) / q ? lo + q : lo, x);
}

struct FusedUpdate {
  const float* partial;    // [groups][ld]
  const float* loss_part;  // [groups]
  int groups;
  int64_t np, ld;
  float scale;           // 1 / (3 B loss_scale)
  float loss_norm;       // 1 / (3 B)
  float* loss_out;
  float* grad_out;       // gradient only (no update)
  // Adam (update)
  float* w;
  float* m;
  float* v;
  float lr, b1, b2, eps, c1, c2;
  uint32_t t, key0, key1;
  const int32_t* fmap;
  const int32_t* tmap;
  const int32_t* bmap;
  void* fpack;
  void* tpack;
  float* head;
};

// The workgroups' sums of 256 parameters: wave q adds groups q, q + 8, ...
// (16-byte loads, four parameters per lane) into eight interleaved running
// sums (group q + 8 i into sum i mod 8: eight loads in flight), the
// eight waves' sums are added in wave order; then per parameter the gradient
// (kUpdate false) or Adam (Kingma & Ba, Alg. 1) on the master weights and the
// rewrite of both operand copies.  Workgroup 0's first wave also sums the
// losses (lane i: groups i, i + 64, ...; then a fixed butterfly).
template <int P, bool kUpdate, bool kSR>
__global__ __launch_bounds__(64 * kUpdateWaves) void k_fused_update(FusedUpdate u) {
  using Elem = typename Prec<P>::Elem;
  constexpr int W = kUpdateWaves, R = 8;
  __shared__ float part[W][256];
  const int q = threadIdx.x >> 6, jj = threadIdx.x & 63;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  float4 sum[R];
#pragma unroll
  for (int i = 0; i < R; ++i) sum[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  auto row = [&](int k) { return *reinterpret_cast<const float4*>(u.partial + (size_t)k * u.ld + j0 + 4 * jj); };
  auto add = [](float4& a, const float4& x) {
    a.x += x.x;
    a.y += x.y;
    a.z += x.z;
    a.w += x.w;
  };
  if (j0 + 4 * jj < u.np) {
    int k = q;
    // all R loads of a round issued before any is used
    for (; k + (R - 1) * W < u.groups; k += R * W) {
      float4 x[R];
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = row(k + i * W);
#pragma unroll
      for (int i = 0; i < R; ++i) add(sum[i], x[i]);
    }
#pragma unroll
    for (int i = 0; i < R - 1; ++i)
      if (k + i * W < u.groups) add(sum[i], row(k + i * W));
  }
  float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  {
    const float4 a = sum[0], b = sum[1], c = sum[2], d = sum[3], e = sum[4], f = sum[5], g = sum[6], hh = sum[7];
    t.x = ((a.x + b.x) + (c.x + d.x)) + ((e.x + f.x) + (g.x + hh.x));
    t.y = ((a.y + b.y) + (c.y + d.y)) + ((e.y + f.y) + (g.y + hh.y));
    t.z = ((a.z + b.z) + (c.z + d.z)) + ((e.z + f.z) + (g.z + hh.z));
    t.w = ((a.w + b.w) + (c.w + d.w)) + ((e.w + f.w) + (g.w + hh.w));
  }
  part[q][4 * jj] = t.x;
  part[q][4 * jj + 1] = t.y;
  part[q][4 * jj + 2] = t.z;
  part[q][4 * jj + 3] = t.w;
  __syncthreads();
  const int64_t j = j0 + threadIdx.x;
  if (threadIdx.x < 256 && j < u.np) {
    float s = 0.0f;
    for (int w = 0; w < W; ++w) s += part[w][threadIdx.x];
    const float g = s * u.scale;
    if constexpr (!kUpdate) {
      u.grad_out[j] = g;
    } else {
      const float mj = u.b1 * u.m[j] + (1.0f - u.b1) * g;
      const float vj = u.b2 * u.v[j] + (1.0f - u.b2) * g * g;
      u.m[j] = mj;
      u.v[j] = vj;
      const float w0 = kSR ? (float)(_Float16)u.w[j] : u.w[j];
      float wj = w0 - u.lr * (mj / u.c1) / (sqrtf(vj / u.c2) + u.eps);
      if (kSR) wj = fp16_round_stochastic(wj, unit_float(philox((uint32_t)j, u.t, 0, kRngStochRound, u.key0, u.key1).x));
      u.w[j] = wj;
      const Elem we = Prec<P>::cvt(wj);
      if (u.fmap[j] >= 0) static_cast<Elem*>(u.fpack)[u.fmap[j]] = we;
      if (u.tmap[j] >= 0) static_cast<Elem*>(u.tpack)[u.tmap[j]] = we;
      if (u.bmap[j] >= 0) u.head[u.bmap[j]] = wj;
    }
  }
  if (blockIdx.x == 0 && q == 0 && u.loss_out) {
    float ls = 0.0f;
    for (int k = jj; k < u.groups; k += 64) ls += u.loss_part[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
    if (jj == 0) *u.loss_out = ls * u.loss_norm;
  }
}

// Operand copies of the master weights (zeros where no weight lands);
// kFp16Master first rounds the master itself to the nearest binary16.
template <int P>
__global__ __launch_bounds__(256) void k_fused_zero(void* p, int64_t n) {
  using Elem = typename Prec<P>::Elem;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    static_cast<Elem*>(p)[i] = Elem{};
}

template <int P, bool kFp16Master>
__global__ __launch_bounds__(256) void k_fused_pack(float* w, const int32_t* fmap, const int32_t* tmap,
                                                   const int32_t* bmap, void* fpack, void* tpack, float* head,
                                                   int64_t np) {
  using Elem = typename Prec<P>::Elem;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    float x = w[j];
    if (kFp16Master) {
      x = (float)(_Float16)x;
      w[j] = x;
    }
    const Elem xe = Prec<P>::cvt(x);
    if (fmap[j] >= 0) static_cast<Elem*>(fpack)[fmap[j]] = xe;
    if (tmap[j] >= 0) static_cast<Elem*>(tpack)[tmap[j]] = xe;
    if (bmap[j] >= 0) head[bmap[j]] = x;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Positions of every weight of layers 0..L-1 in the forward fragments, and of
// every hidden weight of layers 1..L-1 in the transposed fragments (-1:
// none); false if some weight would have no forward position.
template <class A>
static bool fused_maps(std::vector<int32_t>& fmap, std::vector<int32_t>& tmap, std::vector<int32_t>& bmap) {
  using K = Fused<A>;
  using G = Geometry<8, A>;
  constexpr int L = A::kLayers, H = A::kHidden;
  fmap.assign(A::params(), -1);
  tmap.assign(A::params(), -1);
  bmap.assign(A::params(), -1);
  for (int l = 0; l <= L; ++l)
    for (int r = 0; r < A::layer_out(l); ++r) bmap[A::b_offset(l) + r] = l < L ? l * H + r : L * H + r;
  for (int j = 0; j < kOut * H; ++j) bmap[A::w_offset(L) + j] = L * H + 32 + j;
  for (int l = 0; l < L; ++l) {
    const int nkb = G::kb_in(l);
    for (int i = 0; i < G::elems(l); ++i) {
      const int e = i % 8, lane = (i / 8) % 64, qq = i / 512;
      const int row = 32 * (qq / nkb) + lane % 32, kb = qq % nkb;
      const int c = input_index<8, A>(l, kb, lane / 32, e);
      if (c >= 0 && row < A::layer_out(l)) fmap[A::w_offset(l) + row * A::layer_in(l) + c] = G::elem_offset(l) + i;
    }
  }
  for (int l = 1; l < L; ++l) {
    const int kbn = K::t_kb(l);
    for (int i = 0; i < K::t_elems(l); ++i) {
      const int e = i % 8, lane = (i / 8) % 64, qq = i / 512;
      const int mi = qq / kbn, kb = qq % kbn;
      const int in = 32 * mi + lane % 32, out = acc_row(kb / 2, lane / 32, (kb % 2) * 8 + e);
      if (in < A::layer_out(l - 1) && out < A::layer_out(l))
        tmap[A::w_offset(l) + out * A::layer_in(l) + in] = K::t_offset(l) + i;
    }
  }
  for (int l = 0; l < L; ++l)
    for (int j = A::w_offset(l); j < A::b_offset(l); ++j)
      if (fmap[j] < 0) return false;
  return true;
}

static hipError_t grow(void** p, size_t* cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(p, need);
  if (e == hipSuccess) *cap = need;
  return e;
}

void FusedScratch::release() {
  void* all[] = {fpack, tpack, fmap, tmap, partial, loss, loss_part, bmap, head};
  for (void* p : all)
    if (p) (void)hipFree(p);
  fpack = tpack = nullptr;
  fmap = tmap = bmap = nullptr;
  partial = loss = loss_part = head = nullptr;
  for (size_t& b : bytes) b = 0;
  arch = -1;
}

bool fused_train_ok(const TrainConfig& c) {
  return c.path == 0 && c.prec == NPT_FP16 &&
         resident_arch(c.shape.hidden, c.shape.layers, c.shape.skip, c.shape.n_freq) >= 0 &&
         c.batch % kFusedSamples == 0;
}

template <int P, class A>
static hipError_t fused_run_pa(FusedScratch& s, int arch, const TrainConfig& c, const TrainTargets& t,
                               uint32_t step0, uint32_t steps, bool update, float* grad_out, float* loss_out,
                               hipStream_t st) {
  using K = Fused<A>;
  constexpr int64_t np = A::params();
  const int groups = (int)(c.batch / kFusedSamples);
  hipError_t e;
  if (s.arch != arch) {
    std::vector<int32_t> fm, tm, bm;
    if (!fused_maps<A>(fm, tm, bm)) return hipErrorInvalidValue;
    if ((e = grow((void**)&s.fmap, &s.bytes[2], np * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = grow((void**)&s.tmap, &s.bytes[3], np * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = grow((void**)&s.bmap, &s.bytes[7], np * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMemcpy(s.fmap, fm.data(), np * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(s.tmap, tm.data(), np * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(s.bmap, bm.data(), np * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
    s.arch = arch;
  }
  if ((e = grow(&s.fpack, &s.bytes[0], (size_t)K::kFElems * 2)) != hipSuccess) return e;
  if ((e = grow(&s.tpack, &s.bytes[1], (size_t)std::max(K::kTElems, 1) * 2)) != hipSuccess) return e;
  constexpr int64_t ld = (np + 255) / 256 * 256;
  if ((e = grow((void**)&s.partial, &s.bytes[4], (size_t)groups * ld * sizeof(float))) != hipSuccess) return e;
  if ((e = grow((void**)&s.loss, &s.bytes[5], (size_t)std::max(steps, 1u) * sizeof(float))) != hipSuccess) return e;
  if ((e = grow((void**)&s.loss_part, &s.bytes[6], (size_t)groups * sizeof(float))) != hipSuccess) return e;
  if ((e = grow((void**)&s.head, &s.bytes[8], K::kHeadBytes)) != hipSuccess) return e;

  // operand copies of the current master weights
  const bool fp16_master = update && c.master_prec == NPT_FP16;
  hipLaunchKernelGGL(k_fused_zero<P>, dim3(256), dim3(256), 0, st, s.fpack, (int64_t)K::kFElems);
  hipLaunchKernelGGL(k_fused_zero<P>, dim3(256), dim3(256), 0, st, s.tpack, (int64_t)K::kTElems);
  hipLaunchKernelGGL(k_fused_zero<NPT_FP32>, dim3(8), dim3(256), 0, st, static_cast<void*>(s.head),
                     (int64_t)(K::kHeadBytes / 4));
  const int pg = (int)std::min<int64_t>(4096, (np + 255) / 256);
  if (fp16_master)
    hipLaunchKernelGGL((k_fused_pack<P, true>), dim3(pg), dim3(256), 0, st, t.master, s.fmap, s.tmap, s.bmap,
                       s.fpack, s.tpack, s.head, np);
  else
    hipLaunchKernelGGL((k_fused_pack<P, false>), dim3(pg), dim3(256), 0, st, t.master, s.fmap, s.tmap, s.bmap,
                       s.fpack, s.tpack, s.head, np);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  FusedStep fs{};
  fs.fpack = s.fpack;
  fs.tpack = s.tpack;
  fs.head = s.head;
  fs.map = t.map;
  fs.map_w = t.w;
  fs.map_h = t.h;
  fs.key0 = (uint32_t)c.seed;
  fs.key1 = (uint32_t)(c.seed >> 32);
  fs.delta = c.delta;
  fs.loss_scale = c.loss_scale;
  fs.cm = c.cm;
  fs.partial = s.partial;
  fs.loss_part = s.loss_part;
  fs.np = np;
  fs.ld = ld;
  FusedUpdate fu{};
  fu.partial = s.partial;
  fu.loss_part = s.loss_part;
  fu.groups = groups;
  fu.np = np;
  fu.ld = ld;
  fu.scale = 1.0f / (3.0f * (float)c.batch * c.loss_scale);
  fu.loss_norm = 1.0f / (3.0f * (float)c.batch);
  fu.grad_out = grad_out;
  fu.w = t.master;
  fu.m = t.m;
  fu.v = t.v;
  fu.lr = c.lr;
  fu.b1 = c.beta1;
  fu.b2 = c.beta2;
  fu.eps = c.eps;
  fu.key0 = fs.key0;
  fu.key1 = fs.key1;
  fu.fmap = s.fmap;
  fu.tmap = s.tmap;
  fu.bmap = s.bmap;
  fu.head = s.head;
  fu.fpack = s.fpack;
  fu.tpack = s.tpack;
  const int ug = (int)((np + 255) / 256);
  for (uint32_t i = 0; i < steps; ++i) {
    const uint32_t step = step0 + i;
    fs.step = step;
    hipLaunchKernelGGL((k_train_fused<P, A>), dim3(groups), dim3(kFusedBlock), K::kLdsBytes, st, fs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!update) {
      fu.loss_out = loss_out;
      hipLaunchKernelGGL((k_fused_update<P, false, false>), dim3(ug), dim3(64 * kUpdateWaves), 0, st, fu);
    } else {
      const double tt = (double)step + 1.0;
      fu.c1 = (float)(1.0 - std::pow((double)c.beta1, tt));
      fu.c2 = (float)(1.0 - std::pow((double)c.beta2, tt));
      fu.t = step + 1;
      fu.loss_out = s.loss + i;
      if (fp16_master)
        hipLaunchKernelGGL((k_fused_update<P, true, true>), dim3(ug), dim3(64 * kUpdateWaves), 0, st, fu);
      else
        hipLaunchKernelGGL((k_fused_update<P, true, false>), dim3(ug), dim3(64 * kUpdateWaves), 0, st, fu);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
static hipError_t fused_run_p(FusedScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0,
                              uint32_t steps, bool update, float* grad_out, float* loss_out, hipStream_t st) {
  const int arch = resident_arch(c.shape.hidden, c.shape.layers, c.shape.skip, c.shape.n_freq);
  switch (arch) {
    case 0: return fused_run_pa<P, ArchDefault>(s, arch, c, t, step0, steps, update, grad_out, loss_out, st);
    case 1: return fused_run_pa<P, ArchH128Skip40>(s, arch, c, t, step0, steps, update, grad_out, loss_out, st);
    case 2: return fused_run_pa<P, ArchH128Skip64>(s, arch, c, t, step0, steps, update, grad_out, loss_out, st);
    case 3: return fused_run_pa<P, ArchH64>(s, arch, c, t, step0, steps, update, grad_out, loss_out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t fused_train(FusedScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0, uint32_t steps,
                       bool update, float* grad_out, float* loss_out, hipStream_t st) {
  if (!fused_train_ok(c)) return hipErrorInvalidValue;
  return fused_run_p<NPT_FP16>(s, c, t, step0, steps, update, grad_out, loss_out, st);
}

}  // namespace npt
