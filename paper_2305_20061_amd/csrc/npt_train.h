// npt_train.h -- on-device HDR-NIF training (Sec. 3.2.1): uniform (u,v)
// samples with bilinear targets, log compression, Huber loss, hand-written
// backward pass on MFMA GEMMs, Adam with FP32 master weights; and the
// layer-serial inference used for network shapes other than the
// LDS-resident default.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "npt_shared.h"

namespace npt {

// Shape of the MLP at run time: 4 n_freq Fourier features -> layers x
// [dense hidden + ReLU] -> dense 3.  hidden is a multiple of 32 (the MFMA
// tile).  skip: 0, or the hidden layer (1..layers-1) whose input is the
// previous layer's output followed by the features again (skip-concat,
// Sec. 3.2); that previous layer is narrowed to hidden - 4 n_freq outputs so
// that the concatenation, and so every hidden layer's input after the first,
// is hidden wide.
struct NifShape {
  int hidden;
  int layers;
  int skip;
  int n_freq;
};
__host__ __device__ inline int shape_feat(const NifShape& s) { return 4 * s.n_freq; }
__host__ __device__ inline int shape_in(const NifShape& s, int l) { return l == 0 ? shape_feat(s) : s.hidden; }
__host__ __device__ inline int shape_out(const NifShape& s, int l) {
  return l == s.layers ? 3 : (s.skip != 0 && l + 1 == s.skip ? s.hidden - shape_feat(s) : s.hidden);
}
// column of layer `skip`'s input where the features start
__host__ __device__ inline int shape_skip_col(const NifShape& s) { return s.hidden - shape_feat(s); }
// shapes the training and layer-serial kernels accept
__host__ __device__ inline bool shape_ok(const NifShape& s) {
  return s.hidden >= 32 && s.hidden % 32 == 0 && s.layers >= 1 && s.n_freq >= 1 && s.n_freq <= 16 &&
         (s.skip == 0 || (s.skip >= 1 && s.skip < s.layers && s.hidden > shape_feat(s)));
}
// offsets of W_l and b_l in the flat parameter vector [W_0, b_0, ..., W_L, b_L]
__host__ __device__ inline int64_t shape_w_offset(const NifShape& s, int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += (int64_t)shape_out(s, i) * shape_in(s, i) + shape_out(s, i);
  return o;
}
__host__ __device__ inline int64_t shape_b_offset(const NifShape& s, int l) {
  return shape_w_offset(s, l) + (int64_t)shape_out(s, l) * shape_in(s, l);
}
__host__ __device__ inline int64_t shape_params(const NifShape& s) {
  return shape_w_offset(s, s.layers) + 3 * (int64_t)s.hidden + 3;
}

struct TrainConfig {
  uint32_t batch;
  uint64_t samples;
  float lr, beta1, beta2, eps, delta;
  uint64_t seed;
  int prec;          // GEMM operand precision (NPT_FP32 / FP16 / BF16)
  float loss_scale;  // per-sample output gradient scale before low-precision GEMMs
  ColourMatrix cm;   // fixed output colour matrix (network output -> log RGB)
  int master_prec;   // NPT_FP32, or NPT_FP16: binary16 master weights, stochastically rounded updates
  NifShape shape;
  int path;          // 0: the fused step where available, 1: layer-by-layer GEMMs
};

struct TrainTargets {
  const float4* map;
  uint32_t w, h;
  float* master;  // FP32 parameters [shape_params]
  float* m;       // Adam first moments
  float* v;       // Adam second moments
};

// Two-launch training step (k_train_fused.hip) for the LDS-resident shapes
// with FP16 operands and batches of a multiple of 128: operand copies
// of the weights as MFMA fragments (forward and transposed), per-workgroup
// gradient sums and losses, Adam.
struct FusedScratch {
  void* fpack = nullptr;     // forward weight fragments of layers 0..L-1
  void* tpack = nullptr;     // transposed fragments of layers 1..L-1
  int32_t* fmap = nullptr;   // parameter -> position in fpack (-1: none)
  int32_t* tmap = nullptr;   // parameter -> position in tpack (-1: none)
  float* partial = nullptr;  // [workgroups][params]
  float* loss = nullptr;     // per-step losses
  float* loss_part = nullptr;  // [workgroups]
  int32_t* bmap = nullptr;   // parameter -> position in the head table (-1: none)
  float* head = nullptr;     // head table: hidden biases, output biases and weights (FP32)
  size_t bytes[9] = {};
  int arch = -1;             // shape the maps were built for
  void release();
};
// Device scratch of the training step, sized on first use.
struct TrainScratch {
  void* act = nullptr;      // X0 [B][4 n_freq] then the inputs of layers 1..L, operand precision
  void* dp = nullptr;       // two [B][hidden] back-propagated pre-activation gradients
  void* wp = nullptr;       // parameters in operand precision
  float* target = nullptr;  // [B][3] log1p(bilinear) targets
  float* dy = nullptr;      // [B][3] output-layer gradients (scaled)
  float* partial = nullptr; // [splits][params] per-chunk gradient sums
  float* sub = nullptr;     // [B / 64][3 hidden + 3] per-run column sums (bias and output-layer gradients)
  float* grad = nullptr;    // [params]
  float* loss_part = nullptr;
  float* loss = nullptr;    // per-step losses
  float* zgrid = nullptr;   // grid evaluation outputs
  float* err_part = nullptr;
  size_t bytes[10] = {};    // allocated bytes of act .. loss
  uint64_t grid_cap = 0;
  FusedScratch fused;
  void release();
};

bool fused_train_ok(const TrainConfig& c);
hipError_t fused_train(FusedScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0, uint32_t steps,
                       bool update, float* grad_out, float* loss_out, hipStream_t st);

hipError_t train_run(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0, uint32_t steps,
                     float* first_loss, float* last_loss, hipStream_t st);
hipError_t train_gradient(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step,
                          float* d_grad, float* d_loss, hipStream_t st);

// Layer-serial inference (any NifShape, FP32 / FP16 / BF16 operands): rays in
// chunks; Fourier features, one GEMM (bias + ReLU epilogue) per hidden
// layer, then the output layer, colour matrix and expm1.  The operand copy
// wp of the weights is row-major [out][in] as the master; biases come from
// the FP32 master.  Sources as the LDS-resident kernel: the environment
// queue of one depth (count read back from the device), world directions,
// or the centres of a (u,v) grid (log-space RGB out).
enum : int { kLayeredQueue = 0, kLayeredDirs = 1, kLayeredGrid = 2 };
struct LayeredIO {
  int source;
  EnvQueue env;
  float4* L;
  const uint32_t* cnt;
  uint32_t depth;
  const float* dirs;
  float* out;
  uint64_t n;
  uint32_t gw, gh;
};
struct LayeredScratch {
  void* x[3] = {nullptr, nullptr, nullptr};  // ping-pong activations [chunk][hidden], features [chunk][4 n_freq]
  size_t cap = 0;                   // bytes of each
  void release();
};
hipError_t nif_layered(LayeredScratch& ls, int prec, const NifShape& shape, const void* wp, const float* master,
                       const ColourMatrix& cm, const LayeredIO& io, hipStream_t st);
// operand-precision copy of the master weights (wp, n values)
hipError_t launch_params_convert(int prec, const float* master, void* wp, int64_t n, hipStream_t st);
// the values the layered inference multiplies: weights from wp, biases from the master
hipError_t launch_params_dequant(int prec, const NifShape& shape, const float* master, const void* wp, float* out,
                                 hipStream_t st);

// grid evaluation (log-MSE, log-PSNR) of whichever inference path serves
// the context: layered when `layered` is set, else the LDS-resident kernel
hipError_t grid_eval(TrainScratch& s, int prec, int arch, const void* frags, const float* bias,
                     const ColourMatrix& cm, const TrainTargets& t, uint32_t gw, uint32_t gh, int num_cus,
                     float out[2], hipStream_t st, LayeredScratch* layered = nullptr, const NifShape* shape = nullptr);

// counters of the render loop (k_render.hip)
hipError_t launch_stats_clear(unsigned long long* stats, hipStream_t s);
hipError_t launch_stats_add(const uint32_t* cnt, unsigned long long* stats, hipStream_t s);

}  // namespace npt
