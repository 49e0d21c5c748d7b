// Discrete adjoint of a taped rollout (qs_backward.hip).
#pragma once
#include "qs_device.h"

namespace qs {

// Scratch owned by the handle for the backward pass (allocated at create).
// Segments are pipelined over three streams (recompute, reverse sweep on the
// caller's stream, weight gradients) with NBUF rotating segment buffers.
constexpr int BWD_NBUF = 4;
struct BwdBufs {
  int N = 0, K = 0, H = 0;
  int n_parts = 0;                    // partial slots of the weight gradients (dw_gx x groups)
  int dw_gx = 1;                      // weight-gradient workgroups along the 64-env chunks
  int dw_groups = 1;                  // step groups per 64-env chunk
  int n_cu = 0;                       // compute units of the device
  float* seg[BWD_NBUF] = {};          // [K] steps of REC_F blocked rows (rb_at) per env: record
  float* dz[BWD_NBUF] = {};           // [K] steps of 132 blocked rows per env: layer cotangents
  hipStream_t s_rec = nullptr, s_dw = nullptr;
  hipEvent_t e_init = nullptr, e_rec[BWD_NBUF] = {}, e_rev[BWD_NBUF] = {},
             e_dw[BWD_NBUF] = {};
  float* lam = nullptr;    // [145][N] state and history adjoints between segments
  float* gth = nullptr;    // [8][N] parameter gradients
  float* gpart = nullptr;  // [n_parts] weight-gradient partial slots (k_bwd_dw's layout)
  float* gsum = nullptr;   // [13828] sink when no actor gradient is requested
};

hipError_t bwd_alloc(BwdBufs& bw, int N, int K, int H);
// Reverse sweep with one env per lane (qs_reverse1.hip) for one segment of n
// steps from step t0: record rec, checkpoint ck (its episode index keys the
// disturbance), adjoint carry lam [145][N], parameter gradients gth [8][N],
// layer cotangents out to dz.  prepare: once per device (LDS size).
hipError_t reverse1_prepare();
hipError_t launch_reverse1(const DevCfg& c, const float* theta, const float* W, const float* ck,
                           const float* rec, int n, int t0, const float* d_rewards,
                           const float* d_states, float* lam, float* gth, float* dz,
                           hipStream_t st);
void bwd_free(BwdBufs& bw);
// held[i]: the segment whose record bw.seg[i] holds already (written by the
// taped rollout or a recompute of an earlier backward on the same tape), or
// -1; those segments are not recomputed.  Updated to what the buffers hold
// afterwards.
hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        int held[BWD_NBUF], hipStream_t st);

// The same backward with every buffer of bw's shape carved out of `scratch`
// (bwd_scratch_floats(bw) floats, device memory the caller owns) instead of
// the handle's allocations: one segment buffer, every kernel in order on st,
// the last segment recomputed.  The handle's tape is read as usual.  Results
// equal run_backward's bit for bit.
size_t bwd_scratch_floats(const BwdBufs& bw);
hipError_t run_backward_in(const DevCfg& c, const SimBufs& b, const BwdBufs& bw, float* scratch,
                           const float* W, const float* tape, int K, int T,
                           const float* d_rewards, const float* d_states, float* grad_actor,
                           float* grad_params, hipStream_t st);

}  // namespace qs
