// Launchers of the forward kernels (qs_forward.hip) and the backward kernels
// (qs_backward.hip), called by the host runtime (qs_api.hip).
#pragma once
#include "qs_device.h"

namespace qs {

// Intermediates of the plain five-kernel step, [K][N] each.
struct PlainBufs {
  float* obs;  // [146][N]
  float* h1;   // [64][N]
  float* h2;   // [64][N]
  float* act;  // [4][N]
};

hipError_t launch_init(const DevCfg& c, const SimBufs& b, int params, hipStream_t st);
// Snapshots; ret [2][N] = {running return, last finished return}, last_len
// [N]; any pointer may be NULL.
hipError_t launch_get_state(const SimBufs& b, int N, float* state, float* hist, int32_t* t_ep,
                            int32_t* ep, float* ret, int32_t* last_len, hipStream_t st);
hipError_t launch_set_state(const SimBufs& b, int N, const float* state, const float* hist,
                            const int32_t* t_ep, const int32_t* ep, const float* ret,
                            const int32_t* last_len, hipStream_t st);
hipError_t launch_plain_step(const DevCfg& c, const SimBufs& b, const PlainBufs& p,
                             const float* W, const float* ext_act, float* reward, uint8_t* done,
                             float* state_out, hipStream_t st);
hipError_t launch_copy_state(const SimBufs& b, int N, float* out, hipStream_t st);
// Resets the envs with mask[e] != 0 to their next episode (accumulators
// closed as by an in-step reset).
hipError_t launch_reset_envs(const DevCfg& c, const SimBufs& b, const uint8_t* mask,
                             hipStream_t st);
// out[i] = reward of post-step state s[:, i] ([17][M]) and action a[:, i]
// ([4][M]) under the reward constants of c.
hipError_t launch_reward_batch(const DevCfg& c, const float* s, const float* a, int M, float* out,
                               hipStream_t st);
// Observations of the current state: actor observation [146][N] (with the
// noise of the coming step when enabled) and critic observation [28][N];
// either may be NULL.
hipError_t launch_observe(const DevCfg& c, const SimBufs& b, float* actor_obs, float* critic_obs,
                          hipStream_t st);
// Dynamics-only rollout with given actions ([4][N] constant if a_tstride == 0,
// [T][4][N] if a_tstride == 4).
hipError_t launch_dyn_rollout(const DevCfg& c, const SimBufs& b, const float* act, int a_tstride,
                              int T, float* rewards, uint8_t* dones, float* states,
                              hipStream_t st);
// Per-step record of the backward recompute, REC_F rows per env: x_t (17),
// a_t (4), layer-1 and layer-2 pre-activations (64 + 64), the 18 state
// features of the observation o_t (as the actor saw them, noise included)
// and 4 rows of ReLU masks, in the layout of the kernel family that writes
// them (the reverse sweep of the same family reads them).  The
// one-env-per-lane kernel uses its matrix-core tile layout: lane l of a
// 64-env block keeps bit 16 n + 4 bb + v of word w = n / 2 (layer 1, words
// 0-1; layer 2, words 2-3) set when neuron 16 n + 4 (l / 16) + v of env 16 bb
// + l % 16 of the block has a positive pre-activation; the word sits in row
// REC_M + w, column l.  The quarter-lane and split-actor kernels write one
// word per env and quarter k, in row REC_M + k of the env's column: bit
// 8 n + r for layer-1 neuron 16 n + 4 k + r, bit 8 n + 4 + r for layer 2
// (quarter_mask).
// The 128 history features of o_t are not stored per step: they are the
// actions of the 32 previous steps.  After the n step records of a segment
// comes its action tape: per 64-env block, (NH + n) slots of NA rows, slot s
// < NH the checkpoint's history slot s (oldest first), slot NH + t the
// action of step t; the history slot sl of step t is tape slot t + sl.  One
// block's tape is one contiguous span (48 KB for n = 16).
constexpr int REC_X = 0, REC_A = REC_X + NS, REC_Z1 = REC_A + NA, REC_Z2 = REC_Z1 + NHID,
              REC_O = REC_Z2 + NHID, REC_M = REC_O + 18, REC_F = REC_M + 4;

// Tape checkpoint of a differentiable rollout, CK_F rows of [N]: state (17),
// history oldest first (128), then the step within the episode and the
// episode index as int32 bit patterns (they key the observation noise and the
// episode disturbance of the recompute).
constexpr int CK_TEP = NS + NH * NA, CK_EP = CK_TEP + 1, CK_F = CK_EP + 1;

// The backward's per-step records (and the layer cotangents) are blocked by
// 64 envs: within one step, row f of env e sits at rb_at(e, F) + 64 f, F the
// rows per env.  The rows of a block are 256 B apart and a block's record of
// a step is one contiguous span, so the readers, which take a few envs of
// many rows at a time, stay within a few DRAM pages.  A step holds rb_pad(N)
// env slots; the slots of envs >= N in the last block are never written.
constexpr int RB = 64;
__host__ __device__ inline size_t rb_pad(int N) { return (size_t)((N + RB - 1) / RB) * RB; }
__host__ __device__ inline size_t rb_at(int e, int F) {
  return (size_t)(e / RB) * F * RB + (size_t)(e % RB);
}
// Step t of a record buffer, and the action tape of a segment of n steps.
__host__ __device__ inline size_t rec_step(int t, int N) { return (size_t)t * REC_F * rb_pad(N); }
__host__ __device__ inline size_t rec_act(int n, int N) { return (size_t)n * REC_F * rb_pad(N); }
// floats of a record buffer for segments of up to K steps
__host__ __device__ inline size_t rec_floats(int K, int N) {
  return ((size_t)K * REC_F + (size_t)(NH + K) * NA) * rb_pad(N);
}

// Where a launch writes the backward's record: the steps [from, from +
// total) cut into segments of len steps (the last one may be shorter), the
// last segment into buf[0], the one before it into buf[1], ... (at most
// REC_SEGS segments, each in its own record buffer).
constexpr int REC_SEGS = 4;
struct RecSpan {
  float* buf[REC_SEGS];
  int from, len, total;
};
// Where global step gt is recorded: the segment's buffer, the step within
// the segment and the segment's length (false: gt is not recorded).
struct RecAt {
  float* base;
  int step, n;
};
__device__ inline bool rec_at(const RecSpan& rs, int gt, RecAt& r) {
  const int rt = gt - rs.from;
  r.base = rs.buf[0];
  r.step = 0;
  r.n = 1;
  if (!rs.buf[0] || rt < 0 || rt >= rs.total) return false;
  const int segs = (rs.total + rs.len - 1) / rs.len, k = rt / rs.len;
  r.step = rt - k * rs.len;
  r.n = k == segs - 1 ? rs.total - k * rs.len : rs.len;
  r.base = rs.buf[segs - 1 - k];
  return true;
}
// the recorded segments of a span (at most REC_SEGS)
inline bool rec_span_ok(const RecSpan& rs) {
  return !rs.buf[0] || (rs.len >= 1 && rs.total >= 1 && (rs.total + rs.len - 1) / rs.len <= REC_SEGS);
}
hipError_t launch_recompute(const DevCfg& c, const SimBufs& b, const float* W, int T,
                            const float* ck_in, float* rec, hipStream_t st);
// Quarter-lane fused kernel (qs_fused4.hip): 16 envs per wave, 4 lanes per
// env; the kernel of taped rollouts (tape: CK_F-row checkpoints every
// ckpt_every steps).  With ck_in != NULL it starts from that checkpoint and
// leaves the env state alone (the backward's recompute).  With rs.buf[0] !=
// NULL it writes the backward's record of the span rs (the recompute: its
// one segment; a taped rollout: its last segments).
hipError_t launch_fused4(const DevCfg& c, const SimBufs& b, const float* W, int T, int t_base,
                         float* rewards, uint8_t* dones, float* states, float* tape,
                         int ckpt_every, const float* ck_in, const RecSpan& rs, hipStream_t st);
// Split-actor fused kernel (qs_split.hip): 16 envs per workgroup of 4 waves,
// wave w evaluating neuron tile w of layers 1 and 2; tape and record modes as
// the quarter-lane kernel, whose results it reproduces bit for bit.
hipError_t launch_split(const DevCfg& c, const SimBufs& b, const float* W, int T, int t_base,
                        float* rewards, uint8_t* dones, float* states, float* tape,
                        int ckpt_every, const float* ck_in, const RecSpan& rs, hipStream_t st);
// The kernel of taped rollouts and of their backward recompute (the two must
// agree bit for bit): with the fp32 actor the split-actor kernel below 16384
// envs (the quarter-lane kernel leaves SIMDs idle there), the one-env-per-lane
// kernel from 65536 envs (one wave per SIMD, no repeated dynamics), the
// quarter-lane kernel between them and for the bf16 actor.
constexpr int TAPE_SPLIT_MAX_ENVS = 16384;
constexpr int TAPE_LANE_MIN_ENVS = 65536;
enum TapedKernel { TAPED_SPLIT, TAPED_QUARTER, TAPED_LANE };
inline TapedKernel taped_kernel(const DevCfg& c) {
  if (c.flags & F_ACTOR_BF16) return TAPED_QUARTER;
  if (c.n_envs < TAPE_SPLIT_MAX_ENVS) return TAPED_SPLIT;
  return c.n_envs >= TAPE_LANE_MIN_ENVS ? TAPED_LANE : TAPED_QUARTER;
}
// One-env-per-lane fused kernel (qs_fused.hip), actor on fp32 MFMA or VALU.
hipError_t launch_fused(bool mfma, const DevCfg& c, const SimBufs& b, const float* W,
                        const float* ext_act, int T, int t_base, float* rewards, uint8_t* dones,
                        float* states, hipStream_t st);
// The same kernel (fp32 matrix-core actor) with the tape mode of
// launch_fused4 and the record mode for one or more segments (rs.buf[0] ==
// NULL: no record).
hipError_t launch_fused_taped(const DevCfg& c, const SimBufs& b, const float* W, int T,
                              int t_base, float* rewards, uint8_t* dones, float* states,
                              float* tape, int ckpt_every, const float* ck_in, const RecSpan& rs,
                              hipStream_t st);

}  // namespace qs
