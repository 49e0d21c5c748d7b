// Forward kernels of the batched quadrotor step: initialisation and reset,
// snapshots, the plain five-kernel step, and the fused multi-step kernel with
// the actor either on the vector ALUs or on fp32 matrix cores (MFMA).
//
// Layout: one env per lane, struct-of-arrays in HBM ([K][N]) so every global
// access of a wave is a contiguous 256-byte segment.  Actor weights are staged
// in LDS once per workgroup.
#include "qs_actor.h"
#include "qs_forward.h"

namespace qs {

// ---------------------------------------------------------------------------
// Init / reset / snapshots
// ---------------------------------------------------------------------------

// Draws per-env parameters (when params != 0) and episode-0 start states.
__global__ void k_init(DevCfg c, SimBufs b, int params) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float th[NP];
  if (params) {
    env_params(c, (uint32_t)e, th);
#pragma unroll
    for (int i = 0; i < NP; ++i) b.theta[i * N + e] = th[i];
  } else {
#pragma unroll
    for (int i = 0; i < NP; ++i) th[i] = b.theta[i * N + e];
  }
  float s[NS];
  const float ah = reset_state(c, (uint32_t)e, 0u, th[0], th[4], th[5], th[6], s);
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[i * N + e] = s[i];
  for (int i = 0; i < NH * NA; ++i) b.ring[i * N + e] = ah;
  b.head[e] = 0;
  b.t_ep[e] = 0;
  b.ep[e] = 0;
}

__global__ void k_get_state(SimBufs b, int N, float* state, float* hist, int32_t* t_ep,
                            int32_t* ep) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state)
    for (int i = 0; i < NS; ++i) state[i * N + e] = b.state[i * N + e];
  if (hist) {
    const int h = b.head[e];
    for (int s = 0; s < NH; ++s) {
      const int slot = (h + s) & (NH - 1);
#pragma unroll
      for (int a = 0; a < NA; ++a) hist[(s * NA + a) * N + e] = b.ring[(slot * NA + a) * N + e];
    }
  }
  if (t_ep) t_ep[e] = b.t_ep[e];
  if (ep) ep[e] = b.ep[e];
}

__global__ void k_set_state(SimBufs b, int N, const float* state, const float* hist,
                            const int32_t* t_ep, const int32_t* ep) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state)
    for (int i = 0; i < NS; ++i) b.state[i * N + e] = state[i * N + e];
  if (hist) {
    for (int i = 0; i < NH * NA; ++i) b.ring[i * N + e] = hist[i * N + e];
    b.head[e] = 0;
  }
  if (t_ep) b.t_ep[e] = t_ep[e];
  if (ep) b.ep[e] = ep[e];
}

// ---------------------------------------------------------------------------
// Plain path: five kernels per step, every intermediate through HBM.
// ---------------------------------------------------------------------------

// obs[146][N] = {p, R(q), v, w, H oldest..newest}
__global__ void __launch_bounds__(256) k_plain_obs(SimBufs b, int N, float* __restrict__ obs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float q[4], Rm[9];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = b.state[(3 + i) * N + e];
  rotmat(q, Rm);
#pragma unroll
  for (int i = 0; i < 3; ++i) obs[i * N + e] = b.state[i * N + e];
#pragma unroll
  for (int i = 0; i < 9; ++i) obs[(3 + i) * N + e] = Rm[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) obs[(12 + i) * N + e] = b.state[(7 + i) * N + e];
#pragma unroll
  for (int i = 0; i < 3; ++i) obs[(15 + i) * N + e] = b.state[(10 + i) * N + e];
  const int h = b.head[e];
  for (int s = 0; s < NH; ++s) {
    const int slot = (h + s) & (NH - 1);
#pragma unroll
    for (int a = 0; a < NA; ++a)
      obs[(18 + s * NA + a) * N + e] = b.ring[(slot * NA + a) * N + e];
  }
}

// out[NOUT][N] = act(Wl in[NIN][N] + bl), act = ReLU or tanh.  Weights are
// staged transposed in LDS so every lane reads the same address (broadcast).
template <int NIN, int NOUT, bool TANH>
__global__ void __launch_bounds__(256) k_plain_dense(int N, const float* __restrict__ Wl,
                                                     const float* __restrict__ bl,
                                                     const float* __restrict__ in,
                                                     float* __restrict__ out) {
  __shared__ float sW[NIN * NOUT];
  __shared__ float sb[NOUT];
  for (int i = threadIdx.x; i < NIN * NOUT; i += blockDim.x) {
    const int k = i / NOUT, n = i % NOUT;
    sW[i] = Wl[n * NIN + k];
  }
  for (int i = threadIdx.x; i < NOUT; i += blockDim.x) sb[i] = bl[i];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float acc[NOUT];
#pragma unroll
  for (int n = 0; n < NOUT; ++n) acc[n] = sb[n];
  for (int k = 0; k < NIN; ++k) {
    const float x = in[k * N + e];
#pragma unroll
    for (int n = 0; n < NOUT; ++n) acc[n] = fmaf(sW[k * NOUT + n], x, acc[n]);
  }
#pragma unroll
  for (int n = 0; n < NOUT; ++n) out[n * N + e] = TANH ? tanhf(acc[n]) : fmaxf(acc[n], 0.0f);
}

// Dynamics, reward, history push, episode bookkeeping and reset.
__global__ void __launch_bounds__(256) k_plain_dyn(DevCfg c, SimBufs b,
                                                   const float* __restrict__ act,
                                                   float* __restrict__ reward_out,
                                                   uint8_t* __restrict__ done_out,
                                                   float* __restrict__ state_out) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float th[NP], x[NS], a[NA], u[NA];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[i * N + e];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = b.state[i * N + e];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    a[i] = act[i * N + e];
    u[i] = action_to_rpm(c, a[i]);
  }
  const Body<float> B = make_body<float>(th);
  rk4_step<float>(B, c.arm, c.km, c.g, c.dt, (c.flags & F_RENORM_Q) != 0, x, u);
  const float r = reward(c, x, a);
  int h = b.head[e];
#pragma unroll
  for (int i = 0; i < NA; ++i) b.ring[(h * NA + i) * N + e] = a[i];
  h = (h + 1) & (NH - 1);
  int t_ep = b.t_ep[e] + 1;
  const uint32_t d = episode_end(c, x, t_ep);
  if (d && (c.flags & F_AUTORESET)) {
    const int ep = b.ep[e] + 1;
    b.ep[e] = ep;
    t_ep = 0;
    const float ah = reset_state(c, (uint32_t)e, (uint32_t)ep, th[0], th[4], th[5], th[6], x);
    for (int i = 0; i < NH * NA; ++i) b.ring[i * N + e] = ah;
    h = 0;
  }
  b.head[e] = h;
  b.t_ep[e] = t_ep;
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[i * N + e] = x[i];
  if (reward_out) reward_out[e] = r;
  if (done_out) done_out[e] = (uint8_t)d;
  if (state_out)
#pragma unroll
    for (int i = 0; i < NS; ++i) state_out[i * N + e] = x[i];
}

// Copies the state to a [17][N] slice (start state of a recorded rollout).
__global__ void k_copy_state(SimBufs b, int N, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i * N + e] = b.state[i * N + e];
}

// ---------------------------------------------------------------------------
// Fused multi-step kernel
// ---------------------------------------------------------------------------

// T steps of the whole step (observation, actor, action map, RK4, reward,
// history push, termination, truncation, reset) with state and history kept
// in registers.  Outputs indexed by t_base + t.  ext_act ([T][4][N]) replaces
// the actor when non-NULL.  Inactive lanes of the last wave shadow the wave's
// first env (read only) so every MFMA operand is finite.
// Recompute mode of the backward pass (rec != NULL): the start state and
// history come from checkpoint ck_in ([145][N], history oldest first); each
// step records x_t, a_t, z1, z2 and o_t into rec ([T][REC_F][N]); nothing
// else is written.  Record mode is a run-time switch rather than a template
// parameter so that the taped forward and the recompute execute the same
// machine code and produce bit-identical trajectories.
template <bool MFMA>
__global__ void __launch_bounds__(256)
k_fused(DevCfg c, SimBufs b, const float* __restrict__ W, const float* __restrict__ ext_act,
        int T, int t_base, float* __restrict__ rewards, uint8_t* __restrict__ dones,
        float* __restrict__ states, float* __restrict__ tape, int ckpt_every,
        const float* __restrict__ ck_in, float* __restrict__ rec) {
  __shared__ __attribute__((aligned(16))) float lds[LDS_FLOATS];
  const int N = c.n_envs;
  if (ext_act == nullptr) stage_actor<MFMA>(W, lds);
  __syncthreads();
  const int env = blockIdx.x * blockDim.x + threadIdx.x;
  const int first = env - (threadIdx.x & 63);
  if (first >= N) return;  // whole wave past the end
  const bool active = env < N;
  const int e = active ? env : first;
  const bool REC = MFMA && rec != nullptr;

  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[i * N + e];
  const Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;

  float x[NS];
  float H[NH * NA];
  int head0 = 0, t_ep = 0, ep = 0;
  if (REC) {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = ck_in[(size_t)i * N + e];
#pragma unroll
    for (int i = 0; i < NH * NA; ++i) H[i] = ck_in[(size_t)(NS + i) * N + e];
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = b.state[i * N + e];
    head0 = b.head[e];
#pragma unroll
    for (int sl = 0; sl < NH; ++sl) {
      const int slot = (head0 + sl) & (NH - 1);
#pragma unroll
      for (int a = 0; a < NA; ++a) H[sl * NA + a] = b.ring[(slot * NA + a) * N + e];
    }
    t_ep = b.t_ep[e];
    ep = b.ep[e];
  }
  bool was_reset = false;

  if (states && t_base == 0 && active)
#pragma unroll
    for (int i = 0; i < NS; ++i) states[i * N + e] = x[i];

  for (int t = 0; t < T; ++t) {
    // Keeps the weight reads inside the step: hoisting them out of the time
    // loop would pin thousands of loop-invariant values in registers.
    __asm__ volatile("" ::: "memory");
    const uint32_t eo = opaque((uint32_t)e);
    // Re-read each step through an opaque copy so the optimiser cannot split
    // the loop into separate record and no-record versions.
    const bool rec_on = opaque(REC ? 1u : 0u) != 0u;
    const int gt = t_base + t;
    if (tape && (gt % ckpt_every) == 0 && active) {
      float* ck = tape + (size_t)(gt / ckpt_every) * (NS + NH * NA) * N;
#pragma unroll
      for (int i = 0; i < NS; ++i) ck[(size_t)i * N + eo] = x[i];
#pragma unroll
      for (int i = 0; i < NH * NA; ++i) ck[(size_t)(NS + i) * N + eo] = H[i];
    }
    float a[NA];
    float* rt = rec_on ? rec + (size_t)t * REC_F * N : nullptr;
    if (ext_act) {
#pragma unroll
      for (int i = 0; i < NA; ++i) a[i] = ext_act[((size_t)t * NA + i) * N + eo];
    } else {
      float Rm[9];
      rotmat(x + 3, Rm);
      const float* s = x;
      float z3[NA];
      if (MFMA)
        actor_mfma(lds, s, Rm, H, z3, rec_on ? rt + (size_t)REC_Z1 * N : nullptr,
                   rec_on ? rt + (size_t)REC_Z2 * N : nullptr, N, first);
      else
        actor_valu(lds, s, Rm, H, z3);
#pragma unroll
      for (int i = 0; i < NA; ++i) a[i] = tanhf(z3[i]);
      if (rec_on && active) {
#pragma unroll
        for (int i = 0; i < 3; ++i) rt[(size_t)(REC_O + i) * N + eo] = s[i];
#pragma unroll
        for (int i = 0; i < 9; ++i) rt[(size_t)(REC_O + 3 + i) * N + eo] = Rm[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) rt[(size_t)(REC_O + 12 + i) * N + eo] = s[7 + i];
#pragma unroll
        for (int i = 0; i < NH * NA; ++i) rt[(size_t)(REC_O + 18 + i) * N + eo] = H[i];
      }
    }
    if (rec_on && active) {
#pragma unroll
      for (int i = 0; i < NS; ++i) rt[(size_t)(REC_X + i) * N + eo] = x[i];
#pragma unroll
      for (int i = 0; i < NA; ++i) rt[(size_t)(REC_A + i) * N + eo] = a[i];
    }
    float u[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) u[i] = action_to_rpm(c, a[i]);
    rk4_step<float>(B, c.arm, c.km, c.g, c.dt, renorm, x, u);
    const float r = reward(c, x, a);
#pragma unroll
    for (int i = 0; i < (NH - 1) * NA; ++i) H[i] = H[i + NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) H[(NH - 1) * NA + i] = a[i];
    ++t_ep;
    const uint32_t d = episode_end(c, x, t_ep);
    if (d && (c.flags & F_AUTORESET)) {
      ++ep;
      t_ep = 0;
      was_reset = true;
      const float ah = reset_state(c, (uint32_t)e, (uint32_t)ep, th[0], th[4], th[5], th[6], x);
#pragma unroll
      for (int i = 0; i < NH * NA; ++i) H[i] = ah;
    }
    if (active) {
      if (rewards) rewards[(size_t)gt * N + eo] = r;
      if (dones) dones[(size_t)gt * N + eo] = (uint8_t)d;
      if (states)
#pragma unroll
        for (int i = 0; i < NS; ++i) states[((size_t)(gt + 1) * NS + i) * N + eo] = x[i];
    }
  }
  if (!active || REC) return;
  const uint32_t ef = opaque((uint32_t)e);
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + ef] = x[i];
  // The ring keeps slots older than this launch in place; only the T newest
  // logical slots (all 32 after a reset) are written.
  const int head1 = (head0 + T) & (NH - 1);
#pragma unroll
  for (int sl = 0; sl < NH; ++sl) {
    if (was_reset || sl >= NH - T) {
      const int slot = (head1 + sl) & (NH - 1);
#pragma unroll
      for (int a = 0; a < NA; ++a) b.ring[(size_t)(slot * NA + a) * N + ef] = H[sl * NA + a];
    }
  }
  b.head[ef] = head1;
  b.t_ep[ef] = t_ep;
  b.ep[ef] = ep;
}

// ---------------------------------------------------------------------------
// Dynamics-only rollout: the policy is replaced by given actions, either held
// constant ([4][N], a_tstride = 0) or one set per step ([T][4][N],
// a_tstride = 4).  One env per thread, no LDS, so many waves fit per SIMD.
// The action history is brought up to date once at the end (the last 32
// applied actions, or the reset fill after a reset), so a later policy step
// observes exactly what it would have after stepping one by one.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_dyn_rollout(DevCfg c, SimBufs b, const float* __restrict__ act, int a_tstride, int T,
              float* __restrict__ rewards, uint8_t* __restrict__ dones,
              float* __restrict__ states) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  const Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;
  float x[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = b.state[(size_t)i * N + e];
  int t_ep = b.t_ep[e], ep = b.ep[e];
  int last_reset = -1;  // step after which the history was refilled
  float ah = 0.0f;
  if (states)
#pragma unroll
    for (int i = 0; i < NS; ++i) states[(size_t)i * N + e] = x[i];
  for (int t = 0; t < T; ++t) {
    float a[NA], u[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      a[i] = act[((size_t)t * a_tstride + i) * N + e];
      u[i] = action_to_rpm(c, a[i]);
    }
    rk4_step<float>(B, c.arm, c.km, c.g, c.dt, renorm, x, u);
    const float r = reward(c, x, a);
    ++t_ep;
    const uint32_t d = episode_end(c, x, t_ep);
    if (d && (c.flags & F_AUTORESET)) {
      ++ep;
      t_ep = 0;
      last_reset = t;
      ah = reset_state(c, (uint32_t)e, (uint32_t)ep, th[0], th[4], th[5], th[6], x);
    }
    if (rewards) rewards[(size_t)t * N + e] = r;
    if (dones) dones[(size_t)t * N + e] = (uint8_t)d;
    if (states)
#pragma unroll
      for (int i = 0; i < NS; ++i) states[((size_t)(t + 1) * NS + i) * N + e] = x[i];
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = x[i];
  // history: slot 31 newest.  Actions applied after the last reset, older
  // slots from the previous history (or the reset fill).
  const int head0 = b.head[e];
  const int n_new = T - 1 - last_reset;  // actions pushed since the last reset (or all T)
  float hist[NH * NA];
  for (int s = 0; s < NH; ++s) {
    const int age = NH - 1 - s;  // 0 = newest
    for (int i = 0; i < NA; ++i) {
      float v;
      if (age < n_new) {
        v = act[((size_t)(T - 1 - age) * a_tstride + i) * N + e];
      } else if (last_reset >= 0) {
        v = ah;
      } else {
        const int sl = s + n_new;  // logical slot in the old history
        v = b.ring[(size_t)((((head0 + sl) & (NH - 1)) * NA) + i) * N + e];
      }
      hist[s * NA + i] = v;
    }
  }
  for (int i = 0; i < NH * NA; ++i) b.ring[(size_t)i * N + e] = hist[i];
  b.head[e] = 0;
  b.t_ep[e] = t_ep;
  b.ep[e] = ep;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(int n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_init(const DevCfg& c, const SimBufs& b, int params, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(nblk(c.n_envs, 256)), dim3(256), 0, st, c, b, params);
  return hipGetLastError();
}

hipError_t launch_get_state(const SimBufs& b, int N, float* state, float* hist, int32_t* t_ep,
                            int32_t* ep, hipStream_t st) {
  hipLaunchKernelGGL(k_get_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, state, hist, t_ep,
                     ep);
  return hipGetLastError();
}

hipError_t launch_set_state(const SimBufs& b, int N, const float* state, const float* hist,
                            const int32_t* t_ep, const int32_t* ep, hipStream_t st) {
  hipLaunchKernelGGL(k_set_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, state, hist, t_ep,
                     ep);
  return hipGetLastError();
}

hipError_t launch_plain_step(const DevCfg& c, const SimBufs& b, const PlainBufs& p,
                             const float* W, const float* ext_act, float* reward, uint8_t* done,
                             float* state_out, hipStream_t st) {
  const int N = c.n_envs;
  const dim3 g(nblk(N, 256)), blk(256);
  const float* act = ext_act;
  if (!ext_act) {
    hipLaunchKernelGGL(k_plain_obs, g, blk, 0, st, b, N, p.obs);
    hipLaunchKernelGGL((k_plain_dense<NO, NHID, false>), g, blk, 0, st, N, W + OFF_W1, W + OFF_B1,
                       p.obs, p.h1);
    hipLaunchKernelGGL((k_plain_dense<NHID, NHID, false>), g, blk, 0, st, N, W + OFF_W2,
                       W + OFF_B2, p.h1, p.h2);
    hipLaunchKernelGGL((k_plain_dense<NHID, NA, true>), g, blk, 0, st, N, W + OFF_W3, W + OFF_B3,
                       p.h2, p.act);
    act = p.act;
  }
  hipLaunchKernelGGL(k_plain_dyn, g, blk, 0, st, c, b, act, reward, done, state_out);
  return hipGetLastError();
}

hipError_t launch_dyn_rollout(const DevCfg& c, const SimBufs& b, const float* act, int a_tstride,
                              int T, float* rewards, uint8_t* dones, float* states,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_dyn_rollout, dim3(nblk(c.n_envs, 256)), dim3(256), 0, st, c, b, act,
                     a_tstride, T, rewards, dones, states);
  return hipGetLastError();
}

hipError_t launch_copy_state(const SimBufs& b, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, out);
  return hipGetLastError();
}

hipError_t launch_fused(bool mfma, const DevCfg& c, const SimBufs& b, const float* W,
                        const float* ext_act, int T, int t_base, float* rewards, uint8_t* dones,
                        float* states, float* tape, int ckpt_every, hipStream_t st) {
  const dim3 g(nblk(c.n_envs, 256)), blk(256);
  if (mfma)
    hipLaunchKernelGGL(k_fused<true>, g, blk, 0, st, c, b, W, ext_act, T, t_base, rewards, dones,
                       states, tape, ckpt_every, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_fused<false>, g, blk, 0, st, c, b, W, ext_act, T, t_base, rewards, dones,
                       states, tape, ckpt_every, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_recompute(const DevCfg& c, const SimBufs& b, const float* W, int T,
                            const float* ck_in, float* rec, hipStream_t st) {
  // the kernel of taped rollouts, in record mode
  return launch_fused4(c, b, W, T, 0, nullptr, nullptr, nullptr, nullptr, 1, ck_in, rec, st);
}

}  // namespace qs
