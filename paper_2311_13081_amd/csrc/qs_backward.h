// Discrete adjoint of a taped rollout (qs_backward.hip).
#pragma once
#include "qs_device.h"

namespace qs {

// Scratch owned by the handle for the backward pass (allocated at create).
struct BwdBufs {
  int N = 0, K = 0, H = 0;
  int n_parts = 0;         // workgroups of the weight-gradient reduction
  float* seg = nullptr;    // [K][REC_F][N] per-step recompute record of a segment
  float* dz = nullptr;     // [K][132][N] layer cotangents of a segment
  float* lam = nullptr;    // [145][N] state and history adjoints between segments
  float* gth = nullptr;    // [8][N] parameter gradients
  float* gpart = nullptr;  // [n_parts][13828] per-workgroup weight-gradient partials
  float* gsum = nullptr;   // [13828] sink when no actor gradient is requested
};

hipError_t bwd_alloc(BwdBufs& bw, int N, int K, int H);
void bwd_free(BwdBufs& bw);
hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        hipStream_t st);

}  // namespace qs
