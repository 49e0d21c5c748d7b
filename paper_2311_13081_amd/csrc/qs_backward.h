// Discrete adjoint of a taped rollout (qs_backward.hip).
#pragma once
#include "qs_device.h"

namespace qs {

// Scratch owned by the handle for the backward pass.
struct BwdBufs {
  int N = 0, K = 0, H = 0;
  float* seg = nullptr;    // per-step recompute records of one segment
  float* lam = nullptr;    // adjoint carried between segments [145][N]
  float* gpart = nullptr;  // per-workgroup actor-gradient partials
  int n_parts = 0;
};

hipError_t bwd_alloc(BwdBufs& bw, int N, int K, int H);
void bwd_free(BwdBufs& bw);
hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        hipStream_t st);

}  // namespace qs
