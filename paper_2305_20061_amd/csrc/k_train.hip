// k_train.hip -- on-device HDR-NIF training (Sec. 3.2.1): samples, forward
// and backward MFMA GEMMs, Huber head, split-K weight gradients reduced in a
// fixed order (deterministic), Adam on FP32 master weights, grid evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "npt.h"
#include "npt_device.h"
#include "npt_kernels.h"
#include "npt_mfma.h"
#include "npt_nif_layout.h"
#include "npt_train.h"

namespace npt {
using namespace nif;

// batch rows per split-K chunk of the weight gradients: 2048, halved down to
// 512 while a hidden-to-hidden layer's gradient would get fewer than 2048
// waves of 32 x 32 tiles (narrow networks); batches are multiples of 2048
constexpr int kChunkMax = 2048, kChunkMin = 512;
static int grad_chunk(const NifShape& sh, uint32_t B) {
  const int64_t tiles = (int64_t)(sh.hidden / 32) * (sh.hidden / 32);
  int chunk = kChunkMax;
  while (chunk > kChunkMin && tiles * (int64_t)(B / chunk) < 2048) chunk /= 2;
  return chunk;
}

// ---------------------------------------------------------------------------
// samples: (u, v) uniform from the TRAIN Philox stream; features; targets
// log1p(bilinear(map))
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_train_sample(TrainTargets t, uint32_t key0, uint32_t key1, uint32_t step,
                                                     uint32_t B, int nf, typename Prec<P>::Elem* X0, float* target) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const U4 r = philox(b, step, 0, kRngTrain, key0, key1);
    const float u = unit_float(r.x), v = unit_float(r.y);
    typename Prec<P>::Elem* x = X0 + (size_t)b * 4 * nf;
    for (int k = 0; k < nf; ++k) {
      const float f = (float)frequency(k);
      float su, cu, sv, cv;
      sincos_turns(frac_product(f, u), su, cu);
      sincos_turns(frac_product(f, v), sv, cv);
      x[k] = Prec<P>::cvt(su);
      x[nf + k] = Prec<P>::cvt(cu);
      x[2 * nf + k] = Prec<P>::cvt(sv);
      x[3 * nf + k] = Prec<P>::cvt(cv);
    }
    const float3 c = env_bilinear(t.map, (int)t.w, (int)t.h, u, v);
    target[3 * (size_t)b] = log1pf(c.x);
    target[3 * (size_t)b + 1] = log1pf(c.y);
    target[3 * (size_t)b + 2] = log1pf(c.z);
  }
}

// columns [col0, col0 + F) of rows of dst (row stride ld) := the F
// features of each row of X0 (the skip-concat input)
template <int P>
__global__ __launch_bounds__(256) void k_copy_features(const typename Prec<P>::Elem* X0, uint32_t rows, int F,
                                                      typename Prec<P>::Elem* dst, int ld, int col0) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < (uint64_t)rows * F;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = i / F, k = i % F;
    dst[r * ld + col0 + k] = X0[i];
  }
}

// ---------------------------------------------------------------------------
// GEMM on MFMA, one wave per 32x32 output tile, operands straight from
// global memory: C(m, n) = sum_k A(m, k) B(k, n), A(m,k) = A[m*a_sm + k*a_sk],
// B(k,n) = B[k*b_sk + n*b_sn].  AK / BK: the operand is contiguous along k.
// ---------------------------------------------------------------------------
struct GemmDesc {
  const void* A;
  int64_t a_sm, a_sk;
  const void* B;
  int64_t b_sk, b_sn;
  int M, N, K, k_chunk, splits;
  int mode;             // 0: relu(acc + bias[n]) -> C;  1: mask(m,n) > 0 ? acc : 0 -> C;  2: FP32 partial
  float* a_rowsum;      // mode 2, optional: per split, the sums of A's rows over the split's K
  const float* bias;
  const void* mask;
  int64_t mask_ld;
  void* C;
  int64_t ldc, c_split_stride;
};

template <int P, bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc g) {
  using Elem = typename Prec<P>::Elem;
  using Frag = typename Prec<P>::Frag;
  constexpr int KPL = Prec<P>::KPL;
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int mt = (g.M + 31) / 32, nt = (g.N + 31) / 32;  // the last row and column tiles may be partial
  if (wave >= mt * nt * g.splits) return;
  const int split = wave / (mt * nt), rem = wave % (mt * nt);
  const int m0 = (rem / nt) * 32, n0 = (rem % nt) * 32;
  const int h = lane / 32, c = lane % 32;
  const bool col_ok = n0 + c < g.N, row_ok = m0 + c < g.M;
  const int kbeg = split * g.k_chunk, kend = min(g.K, kbeg + g.k_chunk);
  const Elem* A = static_cast<const Elem*>(g.A);
  const Elem* B = static_cast<const Elem*>(g.B);
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const Elem zero = Prec<P>::cvt(0.0f);
  // the waves of the first column tile also sum their rows of A (wave-uniform),
  // as one more MFMA per K-block against a B of ones: every column of `rsum`
  // holds the row sums
  const bool rowsum = g.mode == 2 && g.a_rowsum != nullptr && n0 == 0;
  f32x16 rsum = acc;
  Frag ones;
  if constexpr (KPL == 1) {
    ones = 1.0f;
  } else {
#pragma unroll
    for (int e = 0; e < KPL; ++e) ones[e] = Prec<P>::cvt(1.0f);
  }
  // whole K-blocks with vector loads, then (K not a multiple of 2 KPL) one
  // K-block with element-wise, bounds-checked loads
  int k0 = kbeg;
  for (; k0 + 2 * KPL <= kend; k0 += 2 * KPL) {
    const int kk = k0 + h * KPL;
    Frag a, b;
    if constexpr (KPL == 1) {
      a = row_ok ? A[(int64_t)(m0 + c) * g.a_sm + (int64_t)kk * g.a_sk] : zero;
      b = col_ok ? B[(int64_t)kk * g.b_sk + (int64_t)(n0 + c) * g.b_sn] : zero;
    } else {
      if (!row_ok) {
#pragma unroll
        for (int e = 0; e < KPL; ++e) a[e] = zero;
      } else if constexpr (AK) {
        a = *reinterpret_cast<const Frag*>(A + (int64_t)(m0 + c) * g.a_sm + kk);
      } else {
#pragma unroll
        for (int e = 0; e < KPL; ++e) a[e] = A[(int64_t)(m0 + c) * g.a_sm + (int64_t)(kk + e) * g.a_sk];
      }

      if (!col_ok) {
#pragma unroll
        for (int e = 0; e < KPL; ++e) b[e] = zero;
      } else if constexpr (BK) {
        b = *reinterpret_cast<const Frag*>(B + (int64_t)(n0 + c) * g.b_sn + kk);
      } else {
#pragma unroll
        for (int e = 0; e < KPL; ++e) b[e] = B[(int64_t)(kk + e) * g.b_sk + (int64_t)(n0 + c) * g.b_sn];
      }
    }
    acc = Prec<P>::mma(a, b, acc);
    if (rowsum) rsum = Prec<P>::mma(a, ones, rsum);
  }
  if (k0 < kend) {
    const int kk = k0 + h * KPL;
    Frag a, b;
    if constexpr (KPL == 1) {
      a = (row_ok && kk < kend) ? A[(int64_t)(m0 + c) * g.a_sm + (int64_t)kk * g.a_sk] : zero;
      b = (col_ok && kk < kend) ? B[(int64_t)kk * g.b_sk + (int64_t)(n0 + c) * g.b_sn] : zero;
    } else {
#pragma unroll
      for (int e = 0; e < KPL; ++e) {
        const bool in = kk + e < kend;
        a[e] = (in && row_ok) ? A[(int64_t)(m0 + c) * g.a_sm + (int64_t)(kk + e) * g.a_sk] : zero;
        b[e] = (in && col_ok) ? B[(int64_t)(kk + e) * g.b_sk + (int64_t)(n0 + c) * g.b_sn] : zero;
      }
    }
    acc = Prec<P>::mma(a, b, acc);
    if (rowsum) rsum = Prec<P>::mma(a, ones, rsum);
  }
  if (rowsum && c == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (m0 + acc_row(0, h, r) < g.M) g.a_rowsum[(int64_t)split * g.c_split_stride + m0 + acc_row(0, h, r)] = rsum[r];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + acc_row(0, h, r), n = n0 + c;
    if (!col_ok || m >= g.M) continue;
    float val = acc[r];
    if (g.mode == 0) {
      val = fmaxf(val + g.bias[n], 0.0f);
      static_cast<Elem*>(g.C)[(int64_t)m * g.ldc + n] = Prec<P>::cvt(val);
    } else if (g.mode == 1) {
      const float mk = (float)static_cast<const Elem*>(g.mask)[(int64_t)m * g.mask_ld + n];
      static_cast<Elem*>(g.C)[(int64_t)m * g.ldc + n] = Prec<P>::cvt(mk > 0.0f ? val : 0.0f);
    } else {
      static_cast<float*>(g.C)[(int64_t)split * g.c_split_stride + (int64_t)m * g.ldc + n] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled GEMM for the forward layers of networks at least 64 wide (
// FP16 / BF16 operands, K a multiple of 32, A and B contiguous along K):
// 128 x 128 output tiles per 256-thread workgroup, each wave a 64 x 64
// quarter (2 x 2 MFMA tiles), K in steps of 32 staged through LDS; rows and
// columns beyond M and N are zero-filled on load and skipped on store.
// Epilogue: relu(acc + bias[n]) -> C (mode 0 of GemmDesc).
// ---------------------------------------------------------------------------
constexpr int kTileM = 128, kTileN = 128, kTileK = 32, kTileLd = kTileK + 8;  // LDS row: 40 elements

template <int P, bool AT, bool BT>
__global__ __launch_bounds__(256) void k_gemm_tiled(GemmDesc g) {
  using Elem = typename Prec<P>::Elem;
  using Frag = typename Prec<P>::Frag;
  static_assert(Prec<P>::KPL == 8, "16-bit operands");
  // the operand tiles; after the K loop, half of the output tile at a time
  __shared__ __align__(16) Elem smem[(kTileM + kTileN) * kTileLd];
  Elem* As = smem;
  Elem* Bs = smem + kTileM * kTileLd;
  const int nt = (g.N + kTileN - 1) / kTileN, tiles = ((g.M + kTileM - 1) / kTileM) * nt;
  const int split = blockIdx.x / tiles, tile = blockIdx.x % tiles;  // split-K chunk (mode 2), output tile
  const int m0 = (tile / nt) * kTileM, n0 = (tile % nt) * kTileN;
  const int kbeg = split * g.k_chunk, kend = min(g.K, kbeg + g.k_chunk);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const int h = lane / 32, c = lane % 32;
  const Elem* A = static_cast<const Elem*>(g.A);
  const Elem* B = static_cast<const Elem*>(g.B);
  // staging: thread t loads 16 consecutive k of row t / 2 of each tile
  const int lr = t >> 1, lk = (t & 1) * 16;
  const bool a_ok = m0 + lr < g.M, b_ok = n0 + lr < g.N;
  const Elem* a_src = A + (int64_t)(m0 + lr) * g.a_sm + lk;
  const Elem* b_src = B + (int64_t)(n0 + lr) * g.b_sn + lk;
  // AT / BT (A contiguous along m, B along n): thread t stages 8 consecutive
  // m (n) at one k for each of its two chunks c = t, t + 256 (k = c % 32,
  // m = 8 (c / 32) ..)
  const int bt_k = t % 32, bt_n0 = (t / 32) * 8, bt_n1 = bt_n0 + 64;
  // mode 2 with row sums: the waves of the first column tile also sum A's
  // rows over the chunk, as an MFMA against a B of ones
  const bool rowsum = g.mode == 2 && g.a_rowsum != nullptr && n0 == 0 && wn == 0;
  Frag ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = Prec<P>::cvt(1.0f);
  Frag zf;
#pragma unroll
  for (int e = 0; e < 8; ++e) zf[e] = Prec<P>::cvt(0.0f);
  f32x16 acc[2][2], rs[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) rs[i][r] = 0.0f;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  }
  for (int k0 = kbeg; k0 < kend; k0 += kTileK) {
    Frag a0, a1;
    if constexpr (AT) {
      const Elem* src = A + (int64_t)(k0 + bt_k) * g.a_sk + m0;
      a0 = m0 + bt_n0 < g.M ? *reinterpret_cast<const Frag*>(src + bt_n0) : zf;
      a1 = m0 + bt_n1 < g.M ? *reinterpret_cast<const Frag*>(src + bt_n1) : zf;
    } else {
      a0 = a_ok ? *reinterpret_cast<const Frag*>(a_src + k0) : zf;
      a1 = a_ok ? *reinterpret_cast<const Frag*>(a_src + k0 + 8) : zf;
    }
    Frag b0, b1;
    if constexpr (BT) {
      const Elem* src = B + (int64_t)(k0 + bt_k) * g.b_sk + n0;
      b0 = n0 + bt_n0 < g.N ? *reinterpret_cast<const Frag*>(src + bt_n0) : zf;
      b1 = n0 + bt_n1 < g.N ? *reinterpret_cast<const Frag*>(src + bt_n1) : zf;
    } else {
      b0 = b_ok ? *reinterpret_cast<const Frag*>(b_src + k0) : zf;
      b1 = b_ok ? *reinterpret_cast<const Frag*>(b_src + k0 + 8) : zf;
    }
    __syncthreads();  // the previous step's reads are done
    if constexpr (AT) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        As[(bt_n0 + e) * kTileLd + bt_k] = a0[e];
        As[(bt_n1 + e) * kTileLd + bt_k] = a1[e];
      }
    } else {
      *reinterpret_cast<Frag*>(&As[lr * kTileLd + lk]) = a0;
      *reinterpret_cast<Frag*>(&As[lr * kTileLd + lk + 8]) = a1;
    }
    if constexpr (BT) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        Bs[(bt_n0 + e) * kTileLd + bt_k] = b0[e];
        Bs[(bt_n1 + e) * kTileLd + bt_k] = b1[e];
      }
    } else {
      *reinterpret_cast<Frag*>(&Bs[lr * kTileLd + lk]) = b0;
      *reinterpret_cast<Frag*>(&Bs[lr * kTileLd + lk + 8]) = b1;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      Frag af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        af[i] = *reinterpret_cast<const Frag*>(&As[(wm + i * 32 + c) * kTileLd + kb * 16 + h * 8]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bf[j] = *reinterpret_cast<const Frag*>(&Bs[(wn + j * 32 + c) * kTileLd + kb * 16 + h * 8]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Prec<P>::mma(af[i], bf[j], acc[i][j]);
      if (rowsum) {
#pragma unroll
        for (int i = 0; i < 2; ++i) rs[i] = Prec<P>::mma(af[i], ones, rs[i]);
      }
    }
  }
  if (g.mode == 2) {
    // FP32 partial sums of this chunk, and the row sums of A (every column
    // of rs holds them: lanes 0 and 32 store)
    float* Cp = static_cast<float*>(g.C) + (int64_t)split * g.c_split_stride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn + j * 32 + c;
        if (n >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = m0 + wm + i * 32 + acc_row(0, h, r);
          if (m < g.M) Cp[(int64_t)m * g.ldc + n] = acc[i][j][r];
        }
      }
    if (rowsum && c == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = m0 + wm + i * 32 + acc_row(0, h, r);
          if (m < g.M) g.a_rowsum[(int64_t)split * g.c_split_stride + m] = rs[i][r];
        }
    }
    return;
  }
  Elem* C = static_cast<Elem*>(g.C);
  const Elem* mask = static_cast<const Elem*>(g.mask);
  if (g.ldc % 8 == 0 && g.N % 8 == 0 && reinterpret_cast<uintptr_t>(C) % 16 == 0 &&
      (g.mode == 0 || (g.mask_ld % 8 == 0 && reinterpret_cast<uintptr_t>(mask) % 16 == 0))) {
    // relu(acc + bias) (mode 0) or acc (mode 1) staged through LDS, 64 rows
    // at a time, then stored as 16-byte runs of 8 columns (mode 1 under the
    // ReLU mask, read as 16-byte runs too)
    constexpr int kCLd = kTileN + 8;
    static_assert(64 * kCLd <= (kTileM + kTileN) * kTileLd, "half tile fits the operand buffers");
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      __syncthreads();  // the operand tiles, or the previous half, are no longer read
      if ((wm >> 6) == half) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int nl = wn + j * 32 + c;
          const float bias = g.mode == 0 && n0 + nl < g.N ? g.bias[n0 + nl] : 0.0f;
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float v = acc[i][j][r] + bias;
              smem[(i * 32 + acc_row(0, h, r)) * kCLd + nl] = Prec<P>::cvt(g.mode == 0 ? fmaxf(v, 0.0f) : v);
            }
        }
      }
      __syncthreads();
      for (int q = t; q < 64 * (kTileN / 8); q += 256) {
        const int row = q / (kTileN / 8), col = (q % (kTileN / 8)) * 8;
        const int m = m0 + half * 64 + row, n = n0 + col;
        if (m < g.M && n < g.N) {
          Frag v = *reinterpret_cast<const Frag*>(&smem[row * kCLd + col]);
          if (g.mode == 1) {
            const Frag mk = *reinterpret_cast<const Frag*>(&mask[(int64_t)m * g.mask_ld + n]);
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (!((float)mk[e] > 0.0f)) v[e] = Prec<P>::cvt(0.0f);
          }
          *reinterpret_cast<Frag*>(&C[(int64_t)m * g.ldc + n]) = v;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 32 + c;
      if (n >= g.N) continue;
      const float bias = g.mode == 0 ? g.bias[n] : 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + i * 32 + acc_row(0, h, r);
        if (m >= g.M) continue;
        float v;
        if (g.mode == 0) {
          v = fmaxf(acc[i][j][r] + bias, 0.0f);
        } else {
          const float mk = (float)mask[(int64_t)m * g.mask_ld + n];
          v = mk > 0.0f ? acc[i][j][r] : 0.0f;
        }
        C[(int64_t)m * g.ldc + n] = Prec<P>::cvt(v);
      }
    }
}

// ---------------------------------------------------------------------------
// output layer, colour matrix, Huber loss and the per-sample gradient
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_train_head(const float* wout, int H, const typename Prec<P>::Elem* HL,
                                                   const float* target, float delta, float scale, uint32_t B,
                                                   ColourMatrix cm, float* dy_out, typename Prec<P>::Elem* dP,
                                                   float* loss_part) {
  extern __shared__ float w6[];  // output layer W [3][H], then b [3]
  __shared__ float red[256];
  for (int i = threadIdx.x; i < kOut * H + kOut; i += blockDim.x) w6[i] = wout[i];
  __syncthreads();
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  float loss = 0.0f;
  using Elem = typename Prec<P>::Elem;
  constexpr int V = 16 / sizeof(Elem);  // elements per 16-byte access (H is a multiple of 32)
  union Row {
    uint4 u;
    Elem e[V];
  };
  if (b < B) {
    const uint4* h4 = reinterpret_cast<const uint4*>(HL + (size_t)b * H);
    float y0 = w6[3 * H], y1 = w6[3 * H + 1], y2 = w6[3 * H + 2];
    for (int i0 = 0; i0 < H; i0 += V) {
      Row r;
      r.u = h4[i0 / V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        const float hv = (float)r.e[v];
        y0 += w6[i] * hv;
        y1 += w6[H + i] * hv;
        y2 += w6[2 * H + i] * hv;
      }
    }
    // the fixed colour matrix, in log space
    const float* m = cm.m;
    const float z[3] = {fmaf(m[2], y2, fmaf(m[1], y1, m[0] * y0)), fmaf(m[5], y2, fmaf(m[4], y1, m[3] * y0)),
                        fmaf(m[8], y2, fmaf(m[7], y1, m[6] * y0))};
    float g[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float e = z[k] - target[3 * (size_t)b + k];
      const float ae = fabsf(e);
      loss += ae <= delta ? 0.5f * e * e : delta * (ae - 0.5f * delta);
      g[k] = (ae <= delta ? e : copysignf(delta, e)) * scale;
    }
    // through the colour matrix: dy = M^T g
    const float d0 = fmaf(m[6], g[2], fmaf(m[3], g[1], m[0] * g[0]));
    const float d1 = fmaf(m[7], g[2], fmaf(m[4], g[1], m[1] * g[0]));
    const float d2 = fmaf(m[8], g[2], fmaf(m[5], g[1], m[2] * g[0]));
    dy_out[3 * (size_t)b] = d0;
    dy_out[3 * (size_t)b + 1] = d1;
    dy_out[3 * (size_t)b + 2] = d2;
    uint4* dp4 = reinterpret_cast<uint4*>(dP + (size_t)b * H);
    for (int i0 = 0; i0 < H; i0 += V) {
      Row r, o;
      r.u = h4[i0 / V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        const float gv = (d0 * w6[i] + d1 * w6[H + i]) + d2 * w6[2 * H + i];
        o.e[v] = Prec<P>::cvt((float)r.e[v] > 0.0f ? gv : 0.0f);
      }
      dp4[i0 / V] = o.u;
    }
  }
  red[threadIdx.x] = loss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Output-layer weight/bias gradients of one batch chunk.  Their batch
// reduction runs in two stages so that every CU takes part and the summation
// order stays fixed: runs of kRun rows are summed by separate workgroups into
// sub[run][j], then the runs of each chunk, in order, into the chunk's
// partial sums.  (Hidden-layer bias gradients are summed per chunk by the
// weight-gradient GEMM, which reads dP anyway.)
constexpr int kRun = 64;

// output layer: dW = dy^T HL and db = column sums of dy over one run
// (blockIdx.x: run; blockIdx.y: 320-wide slice of the 3 H + 3 gradients)
template <int P>
__global__ __launch_bounds__(320) void k_head_grad_runs(const float* dy, const typename Prec<P>::Elem* HL, int H,
                                                       float* sub) {
  const int heads = kOut * H + kOut;
  const int j = blockIdx.y * 320 + threadIdx.x;
  const uint32_t b0 = blockIdx.x * kRun;
  float s = 0.0f;
  if (j < kOut * H) {
    const int c = j / H, i = j % H;
    for (uint32_t b = b0; b < b0 + kRun; ++b) s += dy[3 * (size_t)b + c] * (float)HL[(size_t)b * H + i];
  } else if (j < heads) {
    const int c = j - kOut * H;
    for (uint32_t b = b0; b < b0 + kRun; ++b) s += dy[3 * (size_t)b + c];
  }
  if (j < heads) sub[(size_t)blockIdx.x * heads + j] = s;
}

// the runs of each chunk (runs of them), in run order, into
// partial[chunk][off + j]
__global__ __launch_bounds__(320) void k_chunk_sums(const float* sub, int width, int runs, float* partial,
                                                   int64_t off, int64_t np) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= width) return;
  float s = 0.0f;
  for (int r = 0; r < runs; ++r) s += sub[((size_t)blockIdx.x * runs + r) * width + j];
  partial[(size_t)blockIdx.x * np + off + j] = s;
}

// gradient = (sum of the chunk partials) * scale, in a fixed order: wave q
// of a workgroup sums chunks q, q + 8, ... of 64 parameters into four
// interleaved running sums (chunk q + 8i into sum i mod 4: independent loads
// in flight), then the eight waves' sums are added in wave order; loss of the
// step
constexpr int kReduceWaves = 8;
__global__ __launch_bounds__(64 * kReduceWaves) void k_reduce_grad(const float* partial, int splits, float scale,
                                                                  float* grad, const float* loss_part, int nloss,
                                                                  float loss_scale, float* loss_out, int64_t np) {
  __shared__ float part[kReduceWaves][64];
  const int q = threadIdx.x >> 6, jj = threadIdx.x & 63;
  for (int64_t j0 = (int64_t)blockIdx.x * 64; j0 < np; j0 += (int64_t)gridDim.x * 64) {
    const int64_t j = j0 + jj;
    constexpr int W = kReduceWaves;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    if (j < np)
      for (int k = q; k < splits; k += 4 * W) {
        s0 += partial[(size_t)k * np + j];
        if (k + W < splits) s1 += partial[(size_t)(k + W) * np + j];
        if (k + 2 * W < splits) s2 += partial[(size_t)(k + 2 * W) * np + j];
        if (k + 3 * W < splits) s3 += partial[(size_t)(k + 3 * W) * np + j];
      }
    part[q][jj] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (q == 0 && j < np) {
      float s = 0.0f;
      for (int w = 0; w < kReduceWaves; ++w) s += part[w][jj];
      grad[j] = s * scale;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) {
    float s = 0.0f;
    for (int k = 0; k < nloss; ++k) s += loss_part[k];
    *loss_out = s * loss_scale;
  }
}


// Stochastic rounding to binary16 (FP16 master weights, Sec. 3.2.1; Gupta
// et al. 2015): x between the binary16 magnitudes a (toward zero) and a + q
// (q their spacing: 2^(e-10) in the binade [2^e, 2^(e+1)), 2^-24 below
// 2^-14) goes to a + q when u < (|x| - a) / q.  Every step is exact in FP32:
// the scalings by q are powers of two, |x| - a is exact (a <= |x| < 2a or
// a = 0).  Magnitudes from 65504 up saturate.
__device__ __forceinline__ float fp16_stochastic(float x, float u) {
  const float ax = fabsf(x);
  if (ax == 0.0f || ax != ax) return x;
  if (ax >= 65504.0f) return copysignf(65504.0f, x);
  const int e = max(ilogbf(ax), -14);
  const float q = ldexpf(1.0f, e - 10);
  const float a = floorf(ax / q) * q;
  return copysignf(u < (ax - a) / q ? a + q : a, x);
}

// Adam (Kingma & Ba, Alg. 1) on the master weights; refreshes the
// operand-precision copy used by the next step's GEMMs.  kSR: binary16
// master weights (rounded to nearest on entry, a no-op after the first
// step) whose update is rounded stochastically with u from the Philox
// stream (parameter index, Adam step t, 0, kRngStochRound) under the seed.
template <int P, bool kSR>
__global__ __launch_bounds__(256) void k_adam(float* w, float* m, float* v, const float* g, float lr, float b1,
                                             float b2, float eps, float c1, float c2, uint32_t t, uint32_t key0,
                                             uint32_t key1, typename Prec<P>::Elem* wp, int64_t np) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float w0 = kSR ? (float)(_Float16)w[j] : w[j];
    float wj = w0 - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    if (kSR) wj = fp16_stochastic(wj, unit_float(philox((uint32_t)j, t, 0, kRngStochRound, key0, key1).x));
    w[j] = wj;
    wp[j] = Prec<P>::cvt(wj);
  }
}

// operand-precision copy of the master weights; kFp16Master first rounds the
// master itself to the nearest binary16
template <int P, bool kFp16Master>
__global__ __launch_bounds__(256) void k_convert(float* w, typename Prec<P>::Elem* wp, int64_t np) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    float x = w[j];
    if (kFp16Master) {
      x = (float)(_Float16)x;
      w[j] = x;
    }
    wp[j] = Prec<P>::cvt(x);
  }
}

// grid evaluation: squared log-error sums and the largest target per block
__global__ __launch_bounds__(256) void k_grid_err(const float* z, const float4* map, int W, int H, uint32_t gw,
                                                 uint32_t gh, float* part) {
  __shared__ float se[256], mx[256];
  float s = 0.0f, m = 0.0f;
  const uint64_t n = (uint64_t)gw * gh;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float u = ((float)(i % gw) + 0.5f) / (float)gw, v = ((float)(i / gw) + 0.5f) / (float)gh;
    const float3 c = env_bilinear(map, W, H, u, v);
    const float t[3] = {log1pf(c.x), log1pf(c.y), log1pf(c.z)};
    for (int k = 0; k < 3; ++k) {
      const float e = z[3 * i + k] - t[k];
      s += e * e;
      m = fmaxf(m, t[k]);
    }
  }
  se[threadIdx.x] = s;
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      se[threadIdx.x] += se[threadIdx.x + k];
      mx[threadIdx.x] = fmaxf(mx[threadIdx.x], mx[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = se[0];
    part[2 * blockIdx.x + 1] = mx[0];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void TrainScratch::release() {
  void* all[] = {act, dp, wp, target, dy, partial, sub, grad, loss_part, loss, zgrid, err_part};
  for (void* p : all)
    if (p) (void)hipFree(p);
  act = dp = wp = nullptr;
  target = dy = partial = sub = grad = loss_part = loss = zgrid = err_part = nullptr;
  for (size_t& b : bytes) b = 0;
  grid_cap = 0;
  fused.release();
}

static uint32_t elem_size(int prec) { return prec == NPT_FP32 ? 4u : 2u; }

// grows each scratch buffer to what a step of batch B, operand precision
// prec and shape sh needs (and the per-step loss record to `steps`)
static hipError_t ensure_scratch(TrainScratch& s, uint32_t B, int prec, uint32_t steps, const NifShape& sh) {
  const size_t es = elem_size(prec), np = (size_t)shape_params(sh), H = (size_t)sh.hidden;
  size_t act_cols = (size_t)shape_feat(sh);
  for (int l = 1; l <= sh.layers; ++l) act_cols += (size_t)shape_in(sh, l);
  const size_t need[10] = {(size_t)B * act_cols * es,
                           2 * (size_t)B * H * es,
                           np * 4,
                           (size_t)B * 3 * 4,
                           (size_t)B * 3 * 4,
                           ((size_t)B / grad_chunk(sh, B) + 1) * np * 4,
                           ((size_t)B / kRun + 1) * (3 * H + 3) * 4,
                           np * 4,
                           ((size_t)B / 256 + 1) * 4,
                           (size_t)std::max(steps, 1u) * 4};
  void** ptr[10] = {&s.act, &s.dp, &s.wp, (void**)&s.target, (void**)&s.dy, (void**)&s.partial, (void**)&s.sub,
                    (void**)&s.grad, (void**)&s.loss_part, (void**)&s.loss};
  for (int i = 0; i < 10; ++i) {
    if (need[i] <= s.bytes[i]) continue;
    if (*ptr[i]) (void)hipFree(*ptr[i]);
    *ptr[i] = nullptr;
    s.bytes[i] = 0;
    hipError_t e = hipMalloc(ptr[i], need[i]);
    if (e != hipSuccess) return e;
    s.bytes[i] = need[i];
  }
  return hipSuccess;
}

static int grid_for_params(int64_t np) { return (int)std::min<int64_t>(4096, (np + 255) / 256); }

// forward layers (mode 0, both operands contiguous along K) of networks at
// least 64 wide with 16-bit operands take the LDS-tiled kernel (a 96-wide
// layer leaves a quarter of its one 128-column tile idle and is still several
// times faster than one L2-fed wave per 32 x 32 tile)
// AT / BT: A contiguous along m / B contiguous along n (rows of 16-byte
// aligned runs); mode 2 (split-K FP32 partials) needs every chunk whole
template <int P, bool AT, bool BT>
static bool tiled_ok(const GemmDesc& g) {
  auto aligned = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  bool ok = Prec<P>::KPL == 8 && g.N >= 64 && aligned(g.A) && aligned(g.B);
  if (g.mode == 2) ok = ok && g.k_chunk % kTileK == 0 && g.K % g.k_chunk == 0 && g.splits == g.K / g.k_chunk;
  else ok = ok && (g.mode == 0 || g.mode == 1) && g.splits == 1 && g.K % kTileK == 0 && g.k_chunk == g.K;
  if (AT) ok = ok && g.a_sm == 1 && g.a_sk % 8 == 0 && g.M % 8 == 0;
  else ok = ok && g.a_sk == 1 && g.a_sm % 8 == 0;
  if (BT) ok = ok && g.b_sn == 1 && g.b_sk % 8 == 0 && g.N % 8 == 0;
  else ok = ok && g.b_sk == 1 && g.b_sn % 8 == 0;
  return ok;
}

template <int P, bool AK, bool BK>
static hipError_t gemm(const GemmDesc& g, hipStream_t st) {
  if constexpr (Prec<P>::KPL == 8) {
    if (tiled_ok<P, !AK, !BK>(g)) {
      const int tiles = ((g.M + kTileM - 1) / kTileM) * ((g.N + kTileN - 1) / kTileN);
      hipLaunchKernelGGL((k_gemm_tiled<P, !AK, !BK>), dim3(tiles * g.splits), dim3(256), 0, st, g);
      return hipGetLastError();
    }
  }
  const int waves = ((g.M + 31) / 32) * ((g.N + 31) / 32) * g.splits;
  hipLaunchKernelGGL((k_gemm<P, AK, BK>), dim3((waves + 3) / 4), dim3(256), 0, st, g);
  return hipGetLastError();
}

// One training step's loss and gradient (gradient of the mean loss) into
// s.grad / loss_out; weights in operand precision must be current in s.wp.
template <int P>
static hipError_t step_gradient(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step,
                                float* grad_out, float* loss_out, hipStream_t st) {
  using Elem = typename Prec<P>::Elem;
  const NifShape& sh = c.shape;
  const int H = sh.hidden, L = sh.layers;
  const int64_t np = shape_params(sh);
  const uint32_t B = c.batch;
  Elem* act = static_cast<Elem*>(s.act);
  std::vector<Elem*> acts(L + 1);
  acts[0] = act;
  for (int l = 1; l <= L; ++l) acts[l] = acts[l - 1] + (size_t)B * shape_in(sh, l - 1);
  Elem* dp[2] = {static_cast<Elem*>(s.dp), static_cast<Elem*>(s.dp) + (size_t)B * H};
  const Elem* wp = static_cast<const Elem*>(s.wp);
  hipError_t e;
  hipLaunchKernelGGL(k_train_sample<P>, dim3((B + 255) / 256), dim3(256), 0, st, t, (uint32_t)c.seed,
                     (uint32_t)(c.seed >> 32), step, B, sh.n_freq, acts[0], s.target);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (sh.skip != 0) {
    hipLaunchKernelGGL(k_copy_features<P>, dim3(4096), dim3(256), 0, st, acts[0], B, shape_feat(sh), acts[sh.skip],
                       shape_in(sh, sh.skip), shape_skip_col(sh));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int l = 0; l < L; ++l) {
    GemmDesc g{};
    g.A = acts[l];
    g.a_sm = shape_in(sh, l);
    g.a_sk = 1;
    g.B = wp + shape_w_offset(sh, l);
    g.b_sk = 1;
    g.b_sn = shape_in(sh, l);
    g.M = (int)B;
    g.N = shape_out(sh, l);
    g.K = shape_in(sh, l);
    g.k_chunk = g.K;
    g.splits = 1;
    g.mode = 0;
    g.bias = t.master + shape_b_offset(sh, l);
    g.C = acts[l + 1];
    g.ldc = shape_in(sh, l + 1);
    if ((e = gemm<P, true, true>(g, st)) != hipSuccess) return e;
  }
  const int nblk = (int)((B + 255) / 256);
  hipLaunchKernelGGL(k_train_head<P>, dim3(nblk), dim3(256), (size_t)(kOut * H + kOut) * sizeof(float), st,
                     t.master + shape_w_offset(sh, L), H, acts[L], s.target, c.delta, c.loss_scale, B, c.cm, s.dy,
                     dp[0], s.loss_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int chunk = grad_chunk(sh, B);
  const int splits = (int)(B / chunk);
  const int runs = (int)(B / kRun);
  const int heads = kOut * H + kOut;
  hipLaunchKernelGGL(k_head_grad_runs<P>, dim3(runs, (heads + 319) / 320), dim3(320), 0, st, s.dy, acts[L], H,
                     s.sub);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_chunk_sums, dim3(splits, (heads + 319) / 320), dim3(320), 0, st, s.sub, heads,
                     chunk / kRun, s.partial, shape_w_offset(sh, L), np);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int cur = 0;
  for (int l = L - 1; l >= 0; --l) {
    // dW_l = dP_l^T act_l and db_l, split over batch chunks (dP rows are
    // H apart; a narrowed layer uses the first shape_out(l) of them)
    GemmDesc g{};
    g.A = dp[cur];
    g.a_sm = 1;
    g.a_sk = H;
    g.B = acts[l];
    g.b_sk = shape_in(sh, l);
    g.b_sn = 1;
    g.M = shape_out(sh, l);
    g.N = shape_in(sh, l);
    g.K = (int)B;
    g.k_chunk = chunk;
    g.splits = splits;
    g.mode = 2;
    g.C = s.partial + shape_w_offset(sh, l);
    g.ldc = shape_in(sh, l);
    g.c_split_stride = np;
    g.a_rowsum = s.partial + shape_b_offset(sh, l);  // db_l: column sums of dP_l, per chunk
    if ((e = gemm<P, false, false>(g, st)) != hipSuccess) return e;
    if (l == 0) break;
    // dP_{l-1} = (dP_l W_l) masked by act_l > 0
    GemmDesc d{};
    d.A = dp[cur];
    d.a_sm = H;
    d.a_sk = 1;
    d.B = wp + shape_w_offset(sh, l);
    d.b_sk = shape_in(sh, l);
    d.b_sn = 1;
    d.M = (int)B;
    d.N = shape_out(sh, l - 1);  // the hidden part of layer l's input (not the features of a skip-concat)
    d.K = shape_out(sh, l);
    d.k_chunk = d.K;
    d.splits = 1;
    d.mode = 1;
    d.mask = acts[l];
    d.mask_ld = shape_in(sh, l);
    d.C = dp[cur ^ 1];
    d.ldc = H;
    if ((e = gemm<P, true, false>(d, st)) != hipSuccess) return e;
    cur ^= 1;
  }
  const float scale = 1.0f / (3.0f * (float)B * c.loss_scale);
  hipLaunchKernelGGL(k_reduce_grad, dim3((int)std::min<int64_t>(4096, (np + 63) / 64)), dim3(64 * kReduceWaves), 0, st,
                     s.partial, splits, scale, grad_out, s.loss_part, nblk, 1.0f / (3.0f * (float)B), loss_out, np);
  return hipGetLastError();
}

template <int P>
static hipError_t run_p(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0,
                        uint32_t steps, bool update, float* grad_out, float* loss_out, hipStream_t st) {
  using Elem = typename Prec<P>::Elem;
  const int64_t np = shape_params(c.shape);
  const int pg = grid_for_params(np);
  const bool fp16_master = update && c.master_prec == NPT_FP16;
  if (fp16_master)
    hipLaunchKernelGGL((k_convert<P, true>), dim3(pg), dim3(256), 0, st, t.master, static_cast<Elem*>(s.wp), np);
  else
    hipLaunchKernelGGL((k_convert<P, false>), dim3(pg), dim3(256), 0, st, t.master, static_cast<Elem*>(s.wp), np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (uint32_t i = 0; i < steps; ++i) {
    const uint32_t step = step0 + i;
    e = step_gradient<P>(s, c, t, step, update ? s.grad : grad_out, update ? s.loss + i : loss_out, st);
    if (e != hipSuccess) return e;
    if (!update) continue;
    const double tt = (double)step + 1.0;
    const float c1 = (float)(1.0 - std::pow((double)c.beta1, tt));
    const float c2 = (float)(1.0 - std::pow((double)c.beta2, tt));
    const uint32_t k0 = (uint32_t)c.seed, k1 = (uint32_t)(c.seed >> 32), tt1 = step + 1;
    if (fp16_master)
      hipLaunchKernelGGL((k_adam<P, true>), dim3(pg), dim3(256), 0, st, t.master, t.m, t.v, s.grad, c.lr, c.beta1,
                         c.beta2, c.eps, c1, c2, tt1, k0, k1, static_cast<Elem*>(s.wp), np);
    else
      hipLaunchKernelGGL((k_adam<P, false>), dim3(pg), dim3(256), 0, st, t.master, t.m, t.v, s.grad, c.lr, c.beta1,
                         c.beta2, c.eps, c1, c2, tt1, k0, k1, static_cast<Elem*>(s.wp), np);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t dispatch(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0,
                           uint32_t steps, bool update, float* grad_out, float* loss_out, hipStream_t st) {
  if (c.batch % kChunkMax != 0 || !shape_ok(c.shape)) return hipErrorInvalidValue;
  if (fused_train_ok(c)) return fused_train(s.fused, c, t, step0, steps, update, grad_out, loss_out, st);
  hipError_t e = ensure_scratch(s, c.batch, c.prec, update ? steps : 1, c.shape);
  if (e != hipSuccess) return e;
  switch (c.prec) {
    case NPT_FP32: return run_p<NPT_FP32>(s, c, t, step0, steps, update, grad_out, loss_out, st);
    case NPT_FP16: return run_p<NPT_FP16>(s, c, t, step0, steps, update, grad_out, loss_out, st);
    case NPT_BF16: return run_p<NPT_BF16>(s, c, t, step0, steps, update, grad_out, loss_out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t train_run(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0, uint32_t steps,
                     float* first_loss, float* last_loss, hipStream_t st) {
  hipError_t e = dispatch(s, c, t, step0, steps, true, nullptr, nullptr, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  std::vector<float> l(steps ? steps : 1, 0.0f);
  const float* rec = fused_train_ok(c) ? s.fused.loss : s.loss;
  if (steps && (e = hipMemcpy(l.data(), rec, steps * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
    return e;
  *first_loss = l.front();
  *last_loss = l[steps ? steps - 1 : 0];
  return hipSuccess;
}

hipError_t train_gradient(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step,
                          float* d_grad, float* d_loss, hipStream_t st) {
  return dispatch(s, c, t, step, 1, false, d_grad, d_loss, st);
}

// ---------------------------------------------------------------------------
// layer-serial inference (network shapes other than the LDS-resident default)
// ---------------------------------------------------------------------------
constexpr uint32_t kLayeredChunk = 1u << 20;  // rays per pass through the layers

__device__ __forceinline__ void layered_uv(const LayeredIO& io, uint64_t idx, float& u, float& v) {
  if (io.source == kLayeredGrid) {
    u = ((float)(uint32_t)(idx % io.gw) + 0.5f) / (float)io.gw;
    v = ((float)(uint32_t)(idx / io.gw) + 0.5f) / (float)io.gh;
    return;
  }
  V3 d;
  if (io.source == kLayeredQueue) {
    const float4 ed = io.env.d[idx];
    d = V3{ed.x, ed.y, ed.z};
  } else {
    d = V3{io.dirs[3 * idx], io.dirs[3 * idx + 1], io.dirs[3 * idx + 2]};
  }
  direction_to_uv(d, u, v);
}

// Fourier features of rows [base, base + rows) into X0 [rows][64]; rows past
// the n source entries are zero
template <int P>
__global__ __launch_bounds__(256) void k_layered_features(LayeredIO io, uint64_t n, uint64_t base, uint32_t rows,
                                                         int nf, typename Prec<P>::Elem* X0) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    typename Prec<P>::Elem* x = X0 + (size_t)r * 4 * nf;
    const uint64_t idx = base + r;
    if (idx >= n) {
      for (int k = 0; k < 4 * nf; ++k) x[k] = Prec<P>::cvt(0.0f);
      continue;
    }
    float u, v;
    layered_uv(io, idx, u, v);
    for (int k = 0; k < nf; ++k) {
      const float f = (float)frequency(k);
      float su, cu, sv, cv;
      sincos_turns(frac_product(f, u), su, cu);
      sincos_turns(frac_product(f, v), sv, cv);
      x[k] = Prec<P>::cvt(su);
      x[nf + k] = Prec<P>::cvt(cu);
      x[2 * nf + k] = Prec<P>::cvt(sv);
      x[3 * nf + k] = Prec<P>::cvt(cv);
    }
  }
}

// output layer (operand-precision weights, FP32 biases and sums), colour
// matrix, then by source: log-space RGB (grid), radiance (directions), or
// L[slot] += throughput * radiance (queue)
template <int P>
__global__ __launch_bounds__(256) void k_layered_head(const typename Prec<P>::Elem* wout, const float* bout, int H,
                                                     const typename Prec<P>::Elem* XL, ColourMatrix cm, LayeredIO io,
                                                     uint64_t n, uint64_t base, uint32_t rows) {
  extern __shared__ float w6[];  // [3][H] weights, then 3 biases
  for (int i = threadIdx.x; i < kOut * H; i += blockDim.x) w6[i] = (float)wout[i];
  if (threadIdx.x < kOut) w6[kOut * H + threadIdx.x] = bout[threadIdx.x];
  __syncthreads();
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    const uint64_t idx = base + r;
    if (idx >= n) continue;
    const typename Prec<P>::Elem* h = XL + (size_t)r * H;
    float y0 = w6[3 * H], y1 = w6[3 * H + 1], y2 = w6[3 * H + 2];
    for (int i = 0; i < H; ++i) {
      const float hv = (float)h[i];
      y0 = fmaf(w6[i], hv, y0);
      y1 = fmaf(w6[H + i], hv, y1);
      y2 = fmaf(w6[2 * H + i], hv, y2);
    }
    const float* m = cm.m;
    const float zr = fmaf(m[2], y2, fmaf(m[1], y1, m[0] * y0));
    const float zg = fmaf(m[5], y2, fmaf(m[4], y1, m[3] * y0));
    const float zb = fmaf(m[8], y2, fmaf(m[7], y1, m[6] * y0));
    if (io.source == kLayeredGrid) {
      io.out[3 * idx] = zr;
      io.out[3 * idx + 1] = zg;
      io.out[3 * idx + 2] = zb;
      continue;
    }
    const float cr = fmaxf(expm1f(zr), 0.0f), cg = fmaxf(expm1f(zg), 0.0f), cb = fmaxf(expm1f(zb), 0.0f);
    if (io.source == kLayeredDirs) {
      io.out[3 * idx] = cr;
      io.out[3 * idx + 1] = cg;
      io.out[3 * idx + 2] = cb;
    } else {
      const float4 ed = io.env.d[idx], eb = io.env.b[idx];
      const uint32_t slot = __float_as_uint(ed.w);
      float4 l = io.L[slot];
      l.x += eb.x * cr;
      l.y += eb.y * cg;
      l.z += eb.z * cb;
      io.L[slot] = l;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_params_convert(const float* w, typename Prec<P>::Elem* wp, int64_t np) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x)
    wp[j] = Prec<P>::cvt(w[j]);
}

template <int P>
__global__ __launch_bounds__(256) void k_params_dequant(NifShape sh, const float* master,
                                                       const typename Prec<P>::Elem* wp, float* out) {
  const int64_t np = shape_params(sh);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    bool bias = false;
    for (int l = 0; l <= sh.layers; ++l)
      bias |= j >= shape_b_offset(sh, l) && j < shape_b_offset(sh, l) + shape_out(sh, l);
    out[j] = bias ? master[j] : (float)wp[j];
  }
}

void LayeredScratch::release() {
  for (void*& p : x)
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
  cap = 0;
}

template <int P>
static hipError_t layered_p(LayeredScratch& ls, const NifShape& sh, const void* wpv, const float* master,
                            const ColourMatrix& cm, const LayeredIO& io, hipStream_t st) {
  using Elem = typename Prec<P>::Elem;
  const Elem* wp = static_cast<const Elem*>(wpv);
  const int H = sh.hidden, L = sh.layers;
  uint64_t n = io.n;
  hipError_t e;
  if (io.source == kLayeredQueue) {  // the queue length is known only on the device
    uint32_t c = 0;
    if ((e = hipMemcpyAsync(&c, io.cnt + kCntEnv + io.depth, sizeof(c), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    n = c;
  }
  if (n == 0) return hipSuccess;
  const size_t need = (size_t)kLayeredChunk * std::max(H, shape_feat(sh)) * sizeof(Elem);
  if (need > ls.cap) {
    ls.release();
    for (void*& p : ls.x)
      if ((e = hipMalloc(&p, need)) != hipSuccess) return e;
    ls.cap = need;
  }
  for (uint64_t base = 0; base < n; base += kLayeredChunk) {
    const uint32_t rows = (uint32_t)(((std::min<uint64_t>(kLayeredChunk, n - base)) + 31) / 32 * 32);
    // x[2]: the features (kept for a skip-concat); x[0] / x[1]: layer outputs
    // (rows hidden apart)
    Elem* x[3] = {static_cast<Elem*>(ls.x[0]), static_cast<Elem*>(ls.x[1]), static_cast<Elem*>(ls.x[2])};
    hipLaunchKernelGGL(k_layered_features<P>, dim3((rows + 255) / 256), dim3(256), 0, st, io, n, base, rows,
                       sh.n_freq, x[2]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cur = 2, nxt = 0;
    for (int l = 0; l < L; ++l) {
      GemmDesc g{};
      g.A = x[cur];
      g.a_sm = shape_in(sh, l);
      g.a_sk = 1;
      g.B = wp + shape_w_offset(sh, l);
      g.b_sk = 1;
      g.b_sn = shape_in(sh, l);
      g.M = (int)rows;
      g.N = shape_out(sh, l);
      g.K = shape_in(sh, l);
      g.k_chunk = g.K;
      g.splits = 1;
      g.mode = 0;
      g.bias = master + shape_b_offset(sh, l);
      g.C = x[nxt];
      g.ldc = shape_in(sh, l + 1);
      if ((e = gemm<P, true, true>(g, st)) != hipSuccess) return e;
      if (sh.skip != 0 && l + 1 == sh.skip) {
        hipLaunchKernelGGL(k_copy_features<P>, dim3(4096), dim3(256), 0, st, x[2], rows, shape_feat(sh), x[nxt],
                           shape_in(sh, l + 1), shape_skip_col(sh));
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      cur = nxt;
      nxt ^= 1;
    }
    hipLaunchKernelGGL(k_layered_head<P>, dim3((rows + 255) / 256), dim3(256), (size_t)(kOut * H + kOut) * 4, st,
                       wp + shape_w_offset(sh, L), master + shape_b_offset(sh, L), H, x[cur], cm, io, n, base, rows);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t nif_layered(LayeredScratch& ls, int prec, const NifShape& shape, const void* wp, const float* master,
                       const ColourMatrix& cm, const LayeredIO& io, hipStream_t st) {
  if (!shape_ok(shape)) return hipErrorInvalidValue;
  switch (prec) {
    case NPT_FP32: return layered_p<NPT_FP32>(ls, shape, wp, master, cm, io, st);
    case NPT_FP16: return layered_p<NPT_FP16>(ls, shape, wp, master, cm, io, st);
    case NPT_BF16: return layered_p<NPT_BF16>(ls, shape, wp, master, cm, io, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_params_convert(int prec, const float* master, void* wp, int64_t n, hipStream_t st) {
  const int g = grid_for_params(n);
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_params_convert<NPT_FP32>, dim3(g), dim3(256), 0, st, master, (float*)wp, n); break;
    case NPT_FP16: hipLaunchKernelGGL(k_params_convert<NPT_FP16>, dim3(g), dim3(256), 0, st, master, (_Float16*)wp, n); break;
    case NPT_BF16: hipLaunchKernelGGL(k_params_convert<NPT_BF16>, dim3(g), dim3(256), 0, st, master, (__bf16*)wp, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_params_dequant(int prec, const NifShape& shape, const float* master, const void* wp, float* out,
                                 hipStream_t st) {
  const int g = grid_for_params(shape_params(shape));
  switch (prec) {
    case NPT_FP32: hipLaunchKernelGGL(k_params_dequant<NPT_FP32>, dim3(g), dim3(256), 0, st, shape, master, (const float*)wp, out); break;
    case NPT_FP16: hipLaunchKernelGGL(k_params_dequant<NPT_FP16>, dim3(g), dim3(256), 0, st, shape, master, (const _Float16*)wp, out); break;
    case NPT_BF16: hipLaunchKernelGGL(k_params_dequant<NPT_BF16>, dim3(g), dim3(256), 0, st, shape, master, (const __bf16*)wp, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t grid_eval(TrainScratch& s, int prec, int arch, const void* frags, const float* bias,
                     const ColourMatrix& cm, const TrainTargets& t, uint32_t gw, uint32_t gh, int num_cus,
                     float out[2], hipStream_t st, LayeredScratch* layered, const NifShape* shape) {
  const uint64_t n = (uint64_t)gw * gh;
  hipError_t e;
  const int blocks = 256;
  if (n > s.grid_cap) {
    if (s.zgrid) (void)hipFree(s.zgrid);
    if (s.err_part) (void)hipFree(s.err_part);
    s.zgrid = nullptr;
    s.err_part = nullptr;
    s.grid_cap = 0;
    if ((e = hipMalloc((void**)&s.zgrid, n * 3 * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.err_part, 2 * blocks * sizeof(float))) != hipSuccess) return e;
    s.grid_cap = n;
  }
  if (layered) {
    LayeredIO io{};
    io.source = kLayeredGrid;
    io.gw = gw;
    io.gh = gh;
    io.n = n;
    io.out = s.zgrid;
    // frags: the operand-precision weights; bias: the FP32 master
    if ((e = nif_layered(*layered, prec, *shape, frags, bias, cm, io, st)) != hipSuccess) return e;
  } else if ((e = launch_nif_grid(arch, prec, frags, bias, cm, gw, gh, s.zgrid, num_cus, st)) != hipSuccess) {
    return e;
  }
  hipLaunchKernelGGL(k_grid_err, dim3(blocks), dim3(256), 0, st, s.zgrid, t.map, (int)t.w, (int)t.h, gw, gh,
                     s.err_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  std::vector<float> p(2 * blocks);
  if ((e = hipMemcpy(p.data(), s.err_part, p.size() * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  double se = 0.0, mx = 0.0;
  for (int b = 0; b < blocks; ++b) {
    se += p[2 * b];
    mx = std::max(mx, (double)p[2 * b + 1]);
  }
  const double mse = se / (3.0 * (double)n);
  out[0] = (float)mse;
  out[1] = (float)(10.0 * std::log10(mx * mx / std::max(mse, 1e-30)));
  return hipSuccess;
}

}  // namespace npt
