// npt_train.h -- on-device HDR-NIF training (Sec. 3.2.1): uniform (u,v)
// samples with bilinear targets, log compression, Huber loss, hand-written
// backward pass on MFMA GEMMs, Adam with FP32 master weights.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "npt_shared.h"

namespace npt {

struct TrainConfig {
  uint32_t batch;
  uint64_t samples;
  float lr, beta1, beta2, eps, delta;
  uint64_t seed;
  int prec;          // GEMM operand precision (NPT_FP32 / FP16 / BF16)
  float loss_scale;  // per-sample output gradient scale before low-precision GEMMs
  ColourMatrix cm;   // fixed output colour matrix (network output -> log RGB)
  int master_prec;   // NPT_FP32, or NPT_FP16: binary16 master weights, stochastically rounded updates
};

struct TrainTargets {
  const float4* map;
  uint32_t w, h;
  float* master;  // FP32 parameters [kParams]
  float* m;       // Adam first moments
  float* v;       // Adam second moments
};

// Device scratch of the training step, sized on first use.
struct TrainScratch {
  void* act = nullptr;      // X0 [B][64] then H1..H5 [B][96], operand precision
  void* dp = nullptr;       // two [B][96] back-propagated pre-activation gradients
  void* wp = nullptr;       // parameters in operand precision
  float* target = nullptr;  // [B][3] log1p(bilinear) targets
  float* dy = nullptr;      // [B][3] output-layer gradients (scaled)
  float* partial = nullptr; // [splits][kParams] per-chunk gradient sums
  float* sub = nullptr;     // [B / 64][291] per-run column sums (bias and output-layer gradients)
  float* grad = nullptr;    // [kParams]
  float* loss_part = nullptr;
  float* loss = nullptr;    // per-step losses
  float* zgrid = nullptr;   // grid evaluation outputs
  float* err_part = nullptr;
  uint32_t batch_cap = 0, elem_bytes = 0, steps_cap = 0;
  uint64_t grid_cap = 0;
  void release();
};

hipError_t train_run(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step0, uint32_t steps,
                     float* first_loss, float* last_loss, hipStream_t st);
hipError_t train_gradient(TrainScratch& s, const TrainConfig& c, const TrainTargets& t, uint32_t step,
                          float* d_grad, float* d_loss, hipStream_t st);
hipError_t grid_eval(TrainScratch& s, int prec, const void* frags, const float* bias, const ColourMatrix& cm,
                     const TrainTargets& t, uint32_t gw, uint32_t gh, int num_cus, float out[2], hipStream_t st);

// counters of the render loop (k_render.hip)
hipError_t launch_stats_clear(unsigned long long* stats, hipStream_t s);
hipError_t launch_stats_add(const uint32_t* cnt, unsigned long long* stats, hipStream_t s);

}  // namespace npt
