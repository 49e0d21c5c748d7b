// Fused multi-step kernel of the batched quadrotor step with one env per
// lane: observation, actor (vector ALUs or fp32 matrix cores), action map,
// RK4, reward, history push, termination and reset for T steps in one launch.
//
// Layout: struct-of-arrays in HBM ([K][N]) so every global access of a wave is
// a contiguous 256-byte segment; actor weights are staged in LDS once per
// workgroup.
#include "qs_actor.h"
#include "qs_forward.h"

namespace qs {
// ---------------------------------------------------------------------------
// Fused multi-step kernel
// ---------------------------------------------------------------------------

// T steps of the whole step (observation, actor, action map, RK4, reward,
// history push, termination, truncation, reset, episode accumulators) with
// state and history kept in registers.  Outputs indexed by t_base + t.  ext_act ([T][4][N]) replaces
// the actor when non-NULL.  Inactive lanes of the last wave shadow the wave's
// first env (read only) so every MFMA operand is finite.  EXTRAS (the
// training extras or a set point are on): the episode disturbance enters the
// dynamics and the actor sees its observation with noise and the set-point
// shift; without them the kernel carries none of that code.
//
// TAPE (fp32 matrix-core actor only): the differentiable modes of the
// quarter-lane kernel.  With tape != NULL a CK_F-row checkpoint every
// ckpt_every steps; with ck_in != NULL the launch starts from that
// checkpoint and leaves the env state alone (the backward's recompute); with
// rs.buf[0] != NULL the backward's record (blocked by 64 envs) of the steps
// [rs.from, rs.from + rs.total), segment by segment (RecSpan): the taped
// forward records up to the last REC_SEGS segments, a recompute its one
// segment.  The taped forward and the recompute run this same code, so they
// agree bit for bit.
//
// EXT: the actions come from ext_act and the kernel holds no actor; without
// it the loop issues no vector-memory load at all.  (Vector loads and stores
// share one completion counter: a wait for a load issued in the loop would
// also wait for every record and output store issued before it -- with the
// external-action loads only on a runtime branch, the waits at the branch's
// join would drain the step's stores on every step.)
template <bool MFMA, bool EXTRAS, bool BF16, bool TAPE, bool EXT = false>
__global__ void __launch_bounds__(256)
k_fused(DevCfg c, SimBufs b, const float* __restrict__ W, const float* __restrict__ ext_act,
        int T, int t_base, float* __restrict__ rewards, uint8_t* __restrict__ dones,
        float* __restrict__ states, float* __restrict__ tape, int ckpt_every,
        const float* __restrict__ ck_in, RecSpan rs) {
  __shared__ __attribute__((aligned(16))) float lds[LDS_FLOATS];
  const int N = c.n_envs;
  if constexpr (!EXT) {
    if constexpr (BF16)
      stage_actor_bf16(W, lds);
    else
      stage_actor<MFMA>(W, lds);
  }
  __syncthreads();
  const int env = blockIdx.x * blockDim.x + threadIdx.x;
  const int first = env - (threadIdx.x & 63);
  if (first >= N) return;  // whole wave past the end
  const bool active = env < N;
  const int e = active ? env : first;

  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[i * N + e];
  Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;

  // from a checkpoint (the backward's recompute): no write-back of the env
  // state or of the episode accumulators
  const bool REC = TAPE && ck_in != nullptr;
  float x[NS];
  float H[NH * NA];
  int head0 = 0, t_ep = 0, ep = 0;
  EpAcc acc;
  if (REC) {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = ck_in[(size_t)i * N + e];
#pragma unroll
    for (int i = 0; i < NH * NA; ++i) H[i] = ck_in[(size_t)(NS + i) * N + e];
    t_ep = __float_as_int(ck_in[(size_t)CK_TEP * N + e]);
    ep = __float_as_int(ck_in[(size_t)CK_EP * N + e]);
    acc.cur = acc.last = 0.0f, acc.len = 0;
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
    acc.load(b, N, e);
  }
  // record (TAPE): byte offsets of the wave's 64-env block within a step's
  // record (wave uniform), of the lane's own column, and of its place in a
  // matrix-core tile row.  Lanes of envs past the batch write their slots
  // too (copies of the first env's values): the backward's cotangents there
  // are zero.
  const int lane = threadIdx.x & 63;
  const uint32_t blk = __builtin_amdgcn_readfirstlane((uint32_t)(first / RB));
  const uint32_t rstride = 4u * REC_F * (uint32_t)rb_pad(N);  // bytes per recorded step
  const uint32_t s_rblk = 4u * blk * (REC_F * RB);
  const uint32_t v_own = 4u * (uint32_t)lane, v_tile = 4u * (uint32_t)(4 * (lane >> 4) * RB + (lane & 15));
  const int rec_segs = TAPE && rs.buf[0] ? (rs.total + rs.len - 1) / rs.len : 0;
  SetPoint sp;
  if (EXTRAS) sp.load(c, N, e);
  if (EXTRAS) {
    float d[6];
    disturbance(c, (uint32_t)e, (uint32_t)ep, d);
    set_disturbance(B, d);
  }
  bool was_reset = false;
  const float wh = hover_rpm(c, th[0], th[4], th[5], th[6]);
  const float ah = rpm_to_action(c, wh);
  // next episode's start state drawn ahead (long launches only)
  const bool ahead = T >= 2 * RESERVE_PERIOD;
  float nx[NRES];
  bool have = ahead;
  if (ahead) draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);

  if (states && t_base == 0 && active)
#pragma unroll
    for (int i = 0; i < NS; ++i) states[i * N + e] = x[i];

  for (int t = 0; t < T; ++t) {
    // Keeps the weight reads inside the step: hoisting them out of the time
    // loop would pin thousands of loop-invariant values in registers.
    __asm__ volatile("" ::: "memory");
    const uint32_t eo = opaque((uint32_t)e);
    const int gt = t_base + t;
    if (TAPE && tape && (gt % ckpt_every) == 0 && active) {
      float* ck = tape + (size_t)(gt / ckpt_every) * CK_F * N;
#pragma unroll
      for (int i = 0; i < NS; ++i) ck[(size_t)i * N + eo] = x[i];
#pragma unroll
      for (int i = 0; i < NH * NA; ++i) ck[(size_t)(NS + i) * N + eo] = H[i];
      ck[(size_t)CK_TEP * N + eo] = __int_as_float(t_ep);
      ck[(size_t)CK_EP * N + eo] = __int_as_float(ep);
    }
    // wave uniform: the record branches below are scalar branches around one
    // copy of the actor.  Recorded step gt: segment k of the span, its step
    // rt_step, its buffer (the span's last segment in buf[0]) and length;
    // the segment's action tape follows its n_k step records.
    const int rt = gt - rs.from;
    const bool rec_on = TAPE && rec_segs > 0 && rt >= 0 && rt < rs.total;
    const int rk = rec_on ? rt / rs.len : 0;
    const int rt_step = rt - rk * rs.len;
    const int n_k = rk == rec_segs - 1 ? rs.total - rk * rs.len : rs.len;
    const __amdgpu_buffer_rsrc_t rrec =
        span_rsrc(rs.buf[rec_on ? rec_segs - 1 - rk : 0],
                  rec_on ? 4u * (uint32_t)rec_floats(n_k, N) : 0u);
    const uint32_t s_act = __builtin_amdgcn_readfirstlane(
        (uint32_t)n_k * rstride + 4u * blk * (uint32_t)((NH + n_k) * NA * RB));
    float a[NA];
    if constexpr (EXT) {
#pragma unroll
      for (int i = 0; i < NA; ++i) a[i] = ext_act[((size_t)t * NA + i) * N + eo];
    } else {
      float Rm[9];
      rotmat(x + 3, Rm);
      float z3[NA];
      // the observed state features (the set-point shift and the noise
      // under EXTRAS)
      float so[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) so[i] = x[i];
      if constexpr (EXTRAS) {
        if ((c.flags & F_OBS_NOISE) || c.target) {
          float f[18] = {x[0],  x[1],  x[2],  Rm[0], Rm[1], Rm[2], Rm[3], Rm[4],  Rm[5],
                         Rm[6], Rm[7], Rm[8], x[7],  x[8],  x[9],  x[10], x[11], x[12]};
          sp.apply(c, f);
          add_obs_noise(c, (uint32_t)e, (uint32_t)ep, t_ep, f);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            so[i] = f[i];
            so[7 + i] = f[12 + i];
            so[10 + i] = f[15 + i];
          }
#pragma unroll
          for (int i = 0; i < 9; ++i) Rm[i] = f[3 + i];
        }
      }
      // the step's block in the record
      const uint32_t s_rt =
          __builtin_amdgcn_readfirstlane((uint32_t)(rt_step > 0 ? rt_step : 0) * rstride + s_rblk);
      if constexpr (BF16) {
        actor_mfma_bf16(lds, so, Rm, H, z3);
      } else if constexpr (MFMA) {
        if constexpr (TAPE) {
          const ZRec zr{rrec, s_rt + 4u * REC_Z1 * RB, s_rt + 4u * REC_Z2 * RB, v_tile,
                        s_rt + 4u * REC_M * RB, v_own};
          actor_mfma<true>(lds, so, Rm, H, z3, &zr, rec_on);
        } else {
          actor_mfma(lds, so, Rm, H, z3);
        }
      } else {
        actor_valu(lds, so, Rm, H, z3);
      }
#pragma unroll
      for (int i = 0; i < NA; ++i) a[i] = tanh_act(z3[i]);
      if (TAPE && rec_on) {
        // own-env rows: x_t, a_t, the observed state features; the step's
        // action (and, first, the checkpoint's history) on the action tape
        const float of[18] = {so[0], so[1], so[2],  Rm[0],  Rm[1],  Rm[2],  Rm[3],  Rm[4],  Rm[5],
                              Rm[6], Rm[7], Rm[8], so[7], so[8], so[9], so[10], so[11], so[12]};
#pragma unroll
        for (int i = 0; i < NS; ++i) bst1(x[i], rrec, v_own, s_rt + 4u * (REC_X + i) * RB);
#pragma unroll
        for (int i = 0; i < NA; ++i) bst1(a[i], rrec, v_own, s_rt + 4u * (REC_A + i) * RB);
#pragma unroll
        for (int i = 0; i < 18; ++i) bst1(of[i], rrec, v_own, s_rt + 4u * (REC_O + i) * RB);
        if (rt_step == 0) {
#pragma unroll
          for (int i = 0; i < NH * NA; ++i) bst1(H[i], rrec, v_own, s_act + 4u * i * RB);
        }
        const uint32_t s_a =
            __builtin_amdgcn_readfirstlane(s_act + 4u * (uint32_t)(NH + rt_step) * (NA * RB));
#pragma unroll
        for (int i = 0; i < NA; ++i) bst1(a[i], rrec, v_own, s_a + 4u * i * RB);
      }
    }
    float u[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) u[i] = action_to_rpm(c, a[i]);
    rk4_step<float, EXTRAS>(B, c.arm, c.km, c.g, c.dt, renorm, x, u);
    const float r = reward(c, x, a);
    ++t_ep;
    const uint32_t d = episode_end(c, x, t_ep);
    const bool rst = d && (c.flags & F_AUTORESET);
    acc.add(r, rst, t_ep);
    // history push and the reset fill in one pass: one select per slot
#pragma unroll
    for (int i = 0; i < (NH - 1) * NA; ++i) H[i] = rst ? ah : H[i + NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) H[(NH - 1) * NA + i] = rst ? ah : a[i];
    if (rst) {
      ++ep;
      t_ep = 0;
      was_reset = true;
      reset_from_reserve(c, (uint32_t)e, (uint32_t)ep, wh, nx, have, x);
      if (EXTRAS) {
        float dd[6];
        disturbance(c, (uint32_t)e, (uint32_t)ep, dd);
        set_disturbance(B, dd);
      }
    }
    if (ahead && (t & (RESERVE_PERIOD - 1)) == RESERVE_PERIOD - 1 && !have) {
      draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);
      have = true;
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
  acc.store(b, N, ef);
}

static inline unsigned nblk(int n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_fused(bool mfma, const DevCfg& c, const SimBufs& b, const float* W,
                        const float* ext_act, int T, int t_base, float* rewards, uint8_t* dones,
                        float* states, hipStream_t st) {
  const dim3 g(nblk(c.n_envs, 256)), blk(256);
  const bool ex = (c.flags & (F_DISTURB | F_OBS_NOISE)) != 0 || c.target != nullptr;
  // the bf16 actor option runs on the matrix-core kernel
  const bool bf = mfma && (c.flags & F_ACTOR_BF16) != 0;
  auto k = ext_act ? (ex ? k_fused<false, true, false, false, true>
                         : k_fused<false, false, false, false, true>)
           : bf ? (ex ? k_fused<true, true, true, false> : k_fused<true, false, true, false>)
           : mfma ? (ex ? k_fused<true, true, false, false> : k_fused<true, false, false, false>)
                  : (ex ? k_fused<false, true, false, false> : k_fused<false, false, false, false>);
  hipLaunchKernelGGL(k, g, blk, 0, st, c, b, W, ext_act, T, t_base, rewards, dones, states,
                     nullptr, 1, nullptr, RecSpan{});
  return hipGetLastError();
}

hipError_t launch_fused_taped(const DevCfg& c, const SimBufs& b, const float* W, int T,
                              int t_base, float* rewards, uint8_t* dones, float* states,
                              float* tape, int ckpt_every, const float* ck_in, const RecSpan& rs,
                              hipStream_t st) {
  const dim3 g(nblk(c.n_envs, 256)), blk(256);
  const bool ex = (c.flags & (F_DISTURB | F_OBS_NOISE)) != 0 || c.target != nullptr;
  if (!rec_span_ok(rs)) return hipErrorInvalidValue;
  auto k = ex ? k_fused<true, true, false, true> : k_fused<true, false, false, true>;
  hipLaunchKernelGGL(k, g, blk, 0, st, c, b, W, nullptr, T, t_base, rewards, dones, states, tape,
                     ckpt_every, ck_in, rs);
  return hipGetLastError();
}

}  // namespace qs
