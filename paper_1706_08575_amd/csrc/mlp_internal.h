// Learned-weight MLP: parameter layout and the handle behind ftcg_mlp.
#pragma once

#include "ftcg_internal.h"

namespace ftcg {

// flat parameter vector (float32 master copy and its half copy):
// W1 [32][64] row-major, b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1]
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + 32 * 64;
constexpr int MLP_W2 = MLP_B1 + 64;
constexpr int MLP_B2 = MLP_W2 + 64 * 64;
constexpr int MLP_W3 = MLP_B2 + 64;
constexpr int MLP_B3 = MLP_W3 + 64;
constexpr int MLP_NPARAM = MLP_B3 + 1;       // 6337
constexpr int MLP_NPARAM_PAD = 6400;         // partial-gradient row (params + loss slot)

}  // namespace ftcg

struct ftcg_mlp_s {
  hipStream_t stream = nullptr;
  ftcg::DevBuf params;     // float32 master
  ftcg::DevBuf params16;   // half copy used by inference
  ftcg::DevBuf adam_m, adam_v;
  ftcg::DevBuf grad;
  ftcg::DevBuf partial;
  ftcg::DevBuf loss_dev;   // per-minibatch loss sums of the current pattern
  int loss_slot = 0;
  int64_t step = 0;
  float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  // training workspace
  ftcg::DevBuf feat, base, target;
  ftcg_plan labels = nullptr;   // internal plan computing plain weights of training patterns
  float* host = nullptr;        // pinned scratch
};

namespace ftcg {
void launch_knn_features(ftcg_plan p, const double* k, float* feat, double* base, const double* alpha,
                         float* target);
void launch_learned_weights(ftcg_plan p, const double* k, const ftcg_mlp_s* mlp);
void launch_mlp_forward(const ftcg_mlp_s* mlp, const float* feat, int64_t n, float* y);
void launch_mlp_grad(ftcg_mlp_s* mlp, const float* X, const float* T, int64_t m, int64_t mb, int64_t nmb,
                     int64_t batch, int fp16, int adam, float lr, float* grad_out);
void launch_params_to_half(ftcg_mlp_s* mlp);
void launch_audit(ftcg_plan p, const double* k, double* est_dev);
}  // namespace ftcg
