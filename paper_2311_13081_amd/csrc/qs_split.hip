// Fused multi-step kernel with the actor split over the four waves of a
// workgroup, for batches too small to give every SIMD a quarter-lane wave
// (4096 envs make 256 quarter-lane waves for 1024 SIMDs).
//
// A workgroup advances 16 envs.  Each of its 4 waves holds them in the
// quarter-lane layout (lane L = j + 16 k: env j, quarter k; register c of
// quarter k is observation feature q_phi(c, k)), so every env sits on 16
// lanes.  Wave w evaluates neuron tile w (16 neurons) of layers 1 and 2 on
// fp32 MFMA, a quarter of the matrix work of a quarter-lane wave; the four
// tiles are exchanged through LDS with one barrier per layer.  Every wave
// then evaluates layer 3 and the dynamics of the 16 envs: the same
// arithmetic on identical inputs, so the copies agree bit for bit, and the
// MFMA chains are those of the quarter-lane kernel, so its results are the
// same too.  Wave 0 writes the outputs.
#include "qs_forward.h"
#include "qs_quarter.h"

namespace qs {

// Layers 1 and 2 for tile w of the workgroup's 16 envs, exchange through
// xz1/xz2 ([tile][lane]), layer 3 in every wave.  When rz1/rz2 are given,
// writes this wave's tile of the layer pre-activations to the record (rows
// 16 w + 4 lg + r; rec_lane_off addresses row 4 lg of this lane's env) and
// returns the lane's ReLU mask word (quarter_mask, from the exchanged tiles,
// the same in every wave) in zmask.
__device__ inline void actor_split(const float* lds, const float F[Q_C], f4q* xz1, f4q* xz2,
                                   float z3[NA], float* __restrict__ rz1,
                                   float* __restrict__ rz2, bool rec_lane,
                                   uint32_t rec_lane_off, uint32_t& zmask) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int w = threadIdx.x >> 6;
  f4q acc1;
#pragma unroll
  for (int cc = 0; cc < Q_CP / 4; ++cc) {
    const f4q wt = *reinterpret_cast<const f4q*>(
        &lds[Q_W1 + (lg * NHID + 16 * w + li) * Q_W1_P + 4 * cc]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * cc + q;
      if (c < Q_C)
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(
            wt[q], F[c], c == 0 ? *reinterpret_cast<const f4q*>(&lds[Q_B1 + 16 * w + 4 * lg]) : acc1,
            0, 0, 0);
    }
  }
  if (rz1 && rec_lane)
#pragma unroll
    for (int r = 0; r < 4; ++r) rz1[(size_t)(16 * w + r) * RB + rec_lane_off] = acc1[r];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc1[r] = relu_bits(acc1[r]);
  xz1[w * 64 + lane] = acc1;
  __syncthreads();
  f4q z1[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) z1[n] = xz1[n * 64 + lane];
  f4q acc2;
  const f4q b2 = *reinterpret_cast<const f4q*>(&lds[Q_B2 + 16 * w + 4 * lg]);
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const f4q wt = *reinterpret_cast<const f4q*>(&lds[Q_W2 + (16 * w + li) * 68 + 16 * n + 4 * lg]);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(wt[v], z1[n][v], (n == 0 && v == 0) ? b2 : acc2,
                                                  0, 0, 0);
  }
  if (rz2 && rec_lane)
#pragma unroll
    for (int r = 0; r < 4; ++r) rz2[(size_t)(16 * w + r) * RB + rec_lane_off] = acc2[r];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc2[r] = relu_bits(acc2[r]);
  xz2[w * 64 + lane] = acc2;
  __syncthreads();
  f4q z2[4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) z2[n2] = xz2[n2 * 64 + lane];
  zmask = rz1 ? quarter_mask(z1, z2) : 0u;
  layer3_q(lds, z2, z3);
}

// T steps of the whole env step for 16 envs per workgroup (blockDim 256).
// A barrier separates each layer's writes of the exchange buffers from the
// reads, and the next step's writes of a buffer come after the barrier that
// follows every wave's reads of it, so two barriers per step suffice.
// As the quarter-lane kernel: with tape != NULL, checkpoints every
// ckpt_every steps; with rec != NULL, record mode from checkpoint ck_in (no
// write-back of the env state).  Wave 0 writes everything except the layer
// pre-activations, which each wave writes for its own tile.
template <bool EXTRAS>
__global__ void __launch_bounds__(256)
k_split(DevCfg c, SimBufs b, const float* __restrict__ W, int T, int t_base,
        float* __restrict__ rewards, uint8_t* __restrict__ dones, float* __restrict__ states,
        float* __restrict__ tape, int ckpt_every, const float* __restrict__ ck_in,
        RecSpan rs) {
  __shared__ __attribute__((aligned(16))) float lds[Q_TOTAL];
  __shared__ f4q xz1[4 * 64], xz2[4 * 64];
  const int N = c.n_envs;
  const int env0 = blockIdx.x * 16;
  if (env0 >= N) return;  // the whole workgroup (no barrier is reached)
  stage_q(W, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63, j = lane & 15, k = lane >> 4;
  const bool writer = threadIdx.x < 64;  // wave 0
  const int env = env0 + j;
  const bool active = env < N;
  const int e = active ? env : env0;
  // from a checkpoint (the backward's recompute): no write-back of the env
  // state; the steps of the span rs are recorded (rec_at)
  const bool REC = ck_in != nullptr;

  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;

  float x[NS];
  float F[Q_C];  // F[0..4] observation state part (refreshed each step), F[5..36] history
  int head0 = 0, t_ep = 0, ep = 0;
  if (REC) {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = ck_in[(size_t)i * N + e];
#pragma unroll
    for (int s = 0; s < NH; ++s) F[5 + s] = ck_in[(size_t)(NS + s * NA + k) * N + e];
    t_ep = __float_as_int(ck_in[(size_t)CK_TEP * N + e]);
    ep = __float_as_int(ck_in[(size_t)CK_EP * N + e]);
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = b.state[(size_t)i * N + e];
    head0 = b.head[e];
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int slot = (head0 + s) & (NH - 1);
      F[5 + s] = b.ring[(size_t)(slot * NA + k) * N + e];
    }
    t_ep = b.t_ep[e];
    ep = b.ep[e];
  }
  // episode accumulators: the recompute from a checkpoint leaves them alone
  EpAcc acc;
  if (REC)
    acc.cur = acc.last = 0.0f, acc.len = 0;
  else
    acc.load(b, N, e);
  SetPoint sp;
  if (EXTRAS) sp.load(c, N, e);
  bool was_reset = false;
  const float wh = hover_rpm(c, th[0], th[4], th[5], th[6]);
  const float ah = rpm_to_action(c, wh);
  if (EXTRAS) {
    float d[6];
    disturbance(c, (uint32_t)e, (uint32_t)ep, d);
    set_disturbance(B, d);
  }
  // next episode's start state drawn ahead (long launches only)
  const bool ahead = T >= 2 * RESERVE_PERIOD;
  float nx[NRES];
  bool have = ahead;
  if (ahead) draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);

  if (states && t_base == 0 && active && writer)
#pragma unroll
    for (int i = 0; i < NS; ++i)
      if ((i & 3) == k) states[(size_t)i * N + e] = x[i];

  for (int t = 0; t < T; ++t) {
    __asm__ volatile("" ::: "memory");
    const uint32_t eo = opaque((uint32_t)e);
    const int gt = t_base + t;
    RecAt ra;
    const bool rec_on = rec_at(rs, gt, ra);  // wave uniform
    const int rt_step = ra.step;
    if (tape && (gt % ckpt_every) == 0 && active && writer) {
      float* ck = tape + (size_t)(gt / ckpt_every) * CK_F * N;
#pragma unroll
      for (int i = 0; i < NS; ++i)
        if ((i & 3) == k) ck[(size_t)i * N + eo] = x[i];
      const uint32_t kc = opaque((uint32_t)(k * N + e));
#pragma unroll
      for (int s = 0; s < NH; ++s) ck[(size_t)(NS + s * NA) * N + kc] = F[5 + s];
      if (k == 0) {
        ck[(size_t)CK_TEP * N + eo] = __int_as_float(t_ep);
        ck[(size_t)CK_EP * N + eo] = __int_as_float(ep);
      }
    }
    quarter_state_features<EXTRAS>(c, (uint32_t)e, (uint32_t)ep, t_ep, k, x, F, sp);
    float* rt = rec_on ? ra.base + rec_step(rt_step, N) : nullptr;
    const uint32_t zoff = opaque((uint32_t)(rb_at(env0 + j, REC_F) + 4 * k * RB));
    float z3[NA];
    uint32_t zmask;
    actor_split(lds, F, xz1, xz2, z3, rec_on ? rt + (size_t)REC_Z1 * RB : nullptr,
                rec_on ? rt + (size_t)REC_Z2 * RB : nullptr, active, zoff, zmask);
    float a[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = tanh_act(z3[i]);
    if (rec_on && active && writer) {
      const uint32_t koff = opaque((uint32_t)(rb_at(e, REC_F) + k * RB));
      const uint32_t roff = opaque((uint32_t)rb_at(e, REC_F));
#pragma unroll
      for (int cc = 0; cc < 5; ++cc)
        if (q_phi(cc, k) >= 0) rt[(size_t)(REC_O + 4 * cc) * RB + koff] = F[cc];
      float* act = ra.base + rec_act(ra.n, N);
      const uint32_t aoff = opaque((uint32_t)(rb_at(e, (NH + ra.n) * NA) + k * RB));
      if (rt_step == 0) {
#pragma unroll
        for (int s = 0; s < NH; ++s) act[(size_t)(s * NA) * RB + aoff] = F[5 + s];
      }
      act[(size_t)((NH + rt_step) * NA) * RB + aoff] = k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
#pragma unroll
      for (int i = 0; i < NS; ++i)
        if ((i & 3) == k) rt[(size_t)(REC_X + i) * RB + roff] = x[i];
      rt[(size_t)REC_A * RB + koff] = k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
      rt[(size_t)REC_M * RB + koff] = __uint_as_float(zmask);
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
    for (int s = 5; s < Q_C - 1; ++s) F[s] = rst ? ah : F[s + 1];
    F[Q_C - 1] = rst ? ah : k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
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
    if (active && writer) {
      if (k == 0 && rewards) rewards[(size_t)gt * N + eo] = r;
      if (k == 1 && dones) dones[(size_t)gt * N + eo] = (uint8_t)d;
      if (states)
#pragma unroll
        for (int i = 0; i < NS; ++i)
          if ((i & 3) == k) states[((size_t)(gt + 1) * NS + i) * N + eo] = x[i];
    }
  }
  if (!active || !writer || REC) return;
  const uint32_t ef = opaque((uint32_t)e);
#pragma unroll
  for (int i = 0; i < NS; ++i)
    if ((i & 3) == k) b.state[(size_t)i * N + ef] = x[i];
  const int head1 = (head0 + T) & (NH - 1);
#pragma unroll
  for (int s = 0; s < NH; ++s) {
    if (was_reset || s >= NH - T) {
      const int slot = (head1 + s) & (NH - 1);
      b.ring[(size_t)(slot * NA + k) * N + ef] = F[5 + s];
    }
  }
  if (k == 0) {
    b.head[ef] = head1;
    b.t_ep[ef] = t_ep;
    b.ep[ef] = ep;
    acc.store(b, N, ef);
  }
}

hipError_t launch_split(const DevCfg& c, const SimBufs& b, const float* W, int T, int t_base,
                        float* rewards, uint8_t* dones, float* states, float* tape,
                        int ckpt_every, const float* ck_in, const RecSpan& rs, hipStream_t st) {
  if (!rec_span_ok(rs)) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((c.n_envs + 15) / 16);
  const bool ex = (c.flags & (F_DISTURB | F_OBS_NOISE)) != 0 || c.target != nullptr;
  auto k = ex ? k_split<true> : k_split<false>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, c, b, W, T, t_base, rewards, dones, states,
                     tape, ckpt_every, ck_in, rs);
  return hipGetLastError();
}

}  // namespace qs
