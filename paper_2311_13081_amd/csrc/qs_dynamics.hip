// Dynamics-only rollouts of the batched quadrotor step (the policy replaced by
// given actions), one env per thread with the state in registers.
#include "qs_device.h"
#include "qs_forward.h"

namespace qs {
// ---------------------------------------------------------------------------
// Dynamics-only rollout: the policy is replaced by given actions, either held
// constant ([4][N], a_tstride = 0) or one set per step ([T][4][N],
// a_tstride = 4).  One env per thread, no LDS, so many waves fit per SIMD.
// The action history is brought up to date once at the end (the last 32
// applied actions, or the reset fill after a reset), so a later policy step
// observes exactly what it would have after stepping one by one.
// ---------------------------------------------------------------------------
template <bool DIST, bool HELD>
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
  Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;
  float x[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = b.state[(size_t)i * N + e];
  int t_ep = b.t_ep[e], ep = b.ep[e];
  EpAcc acc;
  acc.load(b, N, e);
  if (DIST) {
    float d[6];
    disturbance(c, (uint32_t)e, (uint32_t)ep, d);
    set_disturbance(B, d);
  }
  const float wh = hover_rpm(c, th[0], th[4], th[5], th[6]);
  const float ah0 = rpm_to_action(c, wh);
  // next episode's start state drawn ahead (long launches only)
  const bool ahead = T >= 2 * RESERVE_PERIOD;
  float nx[NRES];
  bool have = ahead;
  if (ahead) draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);
  int last_reset = -1;  // step after which the history was refilled
  float ah = 0.0f;
  if (states)
#pragma unroll
    for (int i = 0; i < NS; ++i) states[(size_t)i * N + e] = x[i];
  // the action of the step is loaded one step ahead (held actions: once)
  if (HELD) a_tstride = 0;
  float an[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) an[i] = act[(size_t)i * N + e];
  for (int t = 0; t < T; ++t) {
    // per-step opaque env index: keeps the 64-bit output addresses from being
    // hoisted out of the loop and held in registers
    const uint32_t eo = opaque((uint32_t)e);
    float a[NA], u[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      a[i] = an[i];
      u[i] = action_to_rpm(c, a[i]);
    }
    if (!HELD && t + 1 < T) {
#pragma unroll
      for (int i = 0; i < NA; ++i) an[i] = act[((size_t)(t + 1) * a_tstride + i) * N + eo];
    }
    rk4_step<float, DIST>(B, c.arm, c.km, c.g, c.dt, renorm, x, u);
    const float r = reward(c, x, a);
    ++t_ep;
    const uint32_t d = episode_end(c, x, t_ep);
    acc.add(r, d && (c.flags & F_AUTORESET), t_ep);
    if (d && (c.flags & F_AUTORESET)) {
      ++ep;
      t_ep = 0;
      last_reset = t;
      ah = ah0;
      reset_from_reserve(c, (uint32_t)e, (uint32_t)ep, wh, nx, have, x);
      if (DIST) {
        float d[6];
        disturbance(c, (uint32_t)e, (uint32_t)ep, d);
        set_disturbance(B, d);
      }
    }
    if (ahead && (t & (RESERVE_PERIOD - 1)) == RESERVE_PERIOD - 1 && !have) {
      draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);
      have = true;
    }
    if (rewards) rewards[(size_t)t * N + eo] = r;
    if (dones) dones[(size_t)t * N + eo] = (uint8_t)d;
    if (states)
#pragma unroll
      for (int i = 0; i < NS; ++i) states[((size_t)(t + 1) * NS + i) * N + eo] = x[i];
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = x[i];
  // History, logical slot 31 newest.  Pushing T actions advances the ring
  // head by T, so a slot older than this launch keeps its place; only the
  // actions applied since the last reset (and the reset fill before them)
  // are written.
  const int head1 = (b.head[e] + T) & (NH - 1);
  const int n_new = T - 1 - last_reset;  // actions pushed since the last reset (or all T)
#pragma unroll 1
  for (int s = 0; s < NH; ++s) {
    const int age = NH - 1 - s;  // 0 = newest
    if (age >= n_new && last_reset < 0) continue;
    const size_t slot = (size_t)((head1 + s) & (NH - 1)) * NA;
    for (int i = 0; i < NA; ++i)
      b.ring[(slot + i) * N + e] =
          age < n_new ? act[((size_t)(T - 1 - age) * a_tstride + i) * N + e] : ah;
  }
  b.head[e] = head1;
  b.t_ep[e] = t_ep;
  b.ep[e] = ep;
  acc.store(b, N, (uint32_t)e);
}

static inline unsigned nblk(int n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_dyn_rollout(const DevCfg& c, const SimBufs& b, const float* act, int a_tstride,
                              int T, float* rewards, uint8_t* dones, float* states,
                              hipStream_t st) {
  auto k = (c.flags & F_DISTURB) ? (a_tstride ? k_dyn_rollout<true, false>
                                               : k_dyn_rollout<true, true>)
                                  : (a_tstride ? k_dyn_rollout<false, false>
                                               : k_dyn_rollout<false, true>);
  hipLaunchKernelGGL(k, dim3(nblk(c.n_envs, 256)), dim3(256), 0, st, c, b, act, a_tstride, T,
                     rewards, dones, states);
  return hipGetLastError();
}

}  // namespace qs
