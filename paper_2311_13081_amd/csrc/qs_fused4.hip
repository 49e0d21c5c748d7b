// Fused multi-step kernel, quarter-lane layout: each wave advances 16 envs
// and each env occupies 4 lanes (lane L = j + 16 k: env j of the wave,
// quarter k).  Compared with the one-env-per-lane kernel this quadruples the
// number of waves for a given batch (so small batches fill the chip and large
// ones keep two waves per SIMD, whose vector instructions interleave) and
// cuts the per-lane history from 128 to 32 registers.
//
// Observation layout across the 4 lanes of an env: register c of quarter k
// holds feature PHI(c, k):
//   c = 0..4:  state feature 4c + k (p, R row-major, v, w: 18 values; the two
//              slots 4*4+2, 4*4+3 are padding);
//   c = 5..36: action history slot c-5 (oldest first), component k.
// This is exactly the B operand of v_mfma_f32_16x16x4f32 for 16 envs with
// K-chunk c, so layer 1 is 37 x 4 MFMAs against W1 columns read in PHI order
// (zeros for padding).  Layer 2 chains through the result registers as in
// the one-env-per-lane kernel; layer 3 is one 16-block 4x4x1 MFMA per layer-2
// result register, and two swap-and-add rounds across 32 and 16 lanes add
// the lane groups' partial sums and leave the 4 actions of env j in all 4 of
// its lanes.  The dynamics run replicated on the 4 lanes
// (identical inputs, identical arithmetic, identical results); memory writes
// are split among the lanes.
//
// Optional bf16 actor (config flag 16): weights are staged in LDS as bf16 and
// the layer inputs are rounded to bf16 (round to nearest even) before
// v_mfma_f32_16x16x32_bf16; accumulation, biases, activations and the whole
// dynamics stay fp32.  The same quarter layout serves: one bf16 instruction
// takes 8 consecutive chunks of the lane's quarter as its 8 K-elements.
#include "qs_forward.h"
#include "qs_quarter.h"

namespace qs {

typedef __bf16 bf8q __attribute__((ext_vector_type(8)));

// Actor for the wave's 16 envs.  F: this lane's 37 layer-1 operands.  Returns
// z3 (pre-tanh) of this lane's env in every lane.  When rz1/rz2 are given,
// writes the layer pre-activations (64 rows of the blocked record; the lane
// offset rec_lane_off addresses row 4 lg of this lane's env) and returns the
// lane's ReLU mask word (quarter_mask) in zmask.
__device__ inline void actor_q(const float* lds, const float F[Q_C], float z3[NA],
                               float* __restrict__ rz1, float* __restrict__ rz2, int N,
                               int env0, uint32_t rec_lane_off, uint32_t& zmask) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  // bias tiles enter as the accumulator input of each chain's first product
  f4q acc1[4];
#pragma unroll
  for (int cc = 0; cc < Q_CP / 4; ++cc) {
    f4q w[4];
#pragma unroll
    for (int n = 0; n < 4; ++n)
      w[n] = *reinterpret_cast<const f4q*>(
          &lds[Q_W1 + (lg * NHID + 16 * n + li) * Q_W1_P + 4 * cc]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * cc + q;
      if (c < Q_C) {
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc1[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              w[n][q], F[c],
              c == 0 ? *reinterpret_cast<const f4q*>(&lds[Q_B1 + 16 * n + 4 * lg]) : acc1[n], 0,
              0, 0);
      }
    }
  }
  const int env = env0 + li;
  if (rz1 && env < N) {
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) rz1[(size_t)(16 * n + r) * RB + rec_lane_off] = acc1[n][r];
  }
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc1[n][r] = relu_bits(acc1[n][r]);
  f4q acc2[4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const f4q w = *reinterpret_cast<const f4q*>(&lds[Q_W2 + (16 * n2 + li) * 68 + 16 * n + 4 * lg]);
      const f4q b2 = *reinterpret_cast<const f4q*>(&lds[Q_B2 + 16 * n2 + 4 * lg]);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc2[n2] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[v], acc1[n][v],
                                                        (n == 0 && v == 0) ? b2 : acc2[n2], 0, 0, 0);
    }
  if (rz2 && env < N) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r) rz2[(size_t)(16 * n2 + r) * RB + rec_lane_off] = acc2[n2][r];
  }
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc2[n2][r] = relu_bits(acc2[n2][r]);
  zmask = rz1 ? quarter_mask(acc1, acc2) : 0u;
  layer3_q(lds, acc2, z3);
}

// ---------------------------------------------------------------------------
// bf16 actor.  LDS layout in bf16 elements:
//   QB_W1: row lg * 64 + neuron, 40 chunks (PHI order of quarter lg, zero
//          padded): one lane reads the 8 chunks of one instruction as 16 B;
//          the pitch of 20 dwords puts 8 consecutive lanes on distinct banks.
//   QB_W2: row = output neuron, pitch 72; within a row, instruction m (layer-1
//          tiles 2m, 2m+1) and lane group lg hold the 8 inputs
//          32m + 16 (e >> 2) + 4 lg + (e & 3), e = 0..7, which is the order in
//          which the previous layer's result registers arrive.
//   QB_W3: as QB_W2 for the 4 outputs (rows 4..15 zero).
// Biases stay fp32 after the bf16 part.
// ---------------------------------------------------------------------------
constexpr int QB_P1 = 40, QB_P2 = 72;
constexpr int QB_W1 = 0, QB_W2 = QB_W1 + 4 * NHID * QB_P1, QB_W3 = QB_W2 + NHID * QB_P2,
              QB_BF16_END = QB_W3 + 16 * QB_P2;
constexpr int QB_FBASE = QB_BF16_END / 2;  // first fp32 slot after the bf16 part
constexpr int QB_B1 = QB_FBASE, QB_B2 = QB_B1 + NHID, QB_B3 = QB_B2 + NHID,
              QB_TOTAL = QB_B3 + 4;          // in floats
static_assert(QB_BF16_END % 8 == 0, "fp32 part must stay 16-byte aligned");

// Input index (within 0..63) of element e of instruction m, lane group lg.
__host__ __device__ constexpr int qb_in(int m, int lg, int e) {
  return 32 * m + 16 * (e >> 2) + 4 * lg + (e & 3);
}

__device__ inline void stage_qb(const float* __restrict__ W, float* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __bf16* h = reinterpret_cast<__bf16*>(lds);
  for (int idx = tid; idx < 4 * NHID * QB_P1; idx += nt) {
    const int c = idx % QB_P1, row = idx / QB_P1, nrn = row & (NHID - 1), k = row / NHID;
    const int f = c < Q_C ? q_phi(c, k) : -1;
    h[QB_W1 + idx] = (__bf16)(f >= 0 ? W[OFF_W1 + nrn * NO + f] : 0.0f);
  }
  for (int idx = tid; idx < NHID * QB_P2; idx += nt) {
    const int r = idx / QB_P2, col = idx % QB_P2;
    float v = 0.0f;
    if (col < NHID) v = W[OFF_W2 + r * NHID + qb_in(col >> 5, (col >> 3) & 3, col & 7)];
    h[QB_W2 + idx] = (__bf16)v;
  }
  for (int idx = tid; idx < 16 * QB_P2; idx += nt) {
    const int r = idx / QB_P2, col = idx % QB_P2;
    float v = 0.0f;
    if (r < NA && col < NHID) v = W[OFF_W3 + r * NHID + qb_in(col >> 5, (col >> 3) & 3, col & 7)];
    h[QB_W3 + idx] = (__bf16)v;
  }
  for (int i = tid; i < NHID; i += nt) {
    lds[QB_B1 + i] = W[OFF_B1 + i];
    lds[QB_B2 + i] = W[OFF_B2 + i];
  }
  for (int i = tid; i < NA; i += nt) lds[QB_B3 + i] = W[OFF_B3 + i];
}

// bf16 operand of one instruction from two result tiles (ReLU applied).
__device__ inline bf8q relu_pack(const f4q& lo, const f4q& hi) {
  bf8q v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = (__bf16)fmaxf(lo[e], 0.0f);
    v[4 + e] = (__bf16)fmaxf(hi[e], 0.0f);
  }
  return v;
}

// Same contract as actor_q, bf16 operands (the mask from the fp32
// accumulators).
__device__ inline void actor_qb(const float* lds, const float F[Q_C], float z3[NA],
                                float* __restrict__ rz1, float* __restrict__ rz2, int N,
                                int env0, uint32_t rec_lane_off, uint32_t& zmask) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const __bf16* h = reinterpret_cast<const __bf16*>(lds);
  f4q acc1[4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc1[n][r] = lds[QB_B1 + 16 * n + 4 * lg + r];
#pragma unroll
  for (int g = 0; g < QB_P1 / 8; ++g) {
    bf8q x;
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (__bf16)(8 * g + e < Q_C ? F[8 * g + e] : 0.0f);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const bf8q w = *reinterpret_cast<const bf8q*>(
          &h[QB_W1 + (lg * NHID + 16 * n + li) * QB_P1 + 8 * g]);
      acc1[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, acc1[n], 0, 0, 0);
    }
  }
  const int env = env0 + li;
  if (rz1 && env < N) {
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) rz1[(size_t)(16 * n + r) * RB + rec_lane_off] = acc1[n][r];
  }
  f4q acc2[4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc2[n2][r] = lds[QB_B2 + 16 * n2 + 4 * lg + r];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const bf8q x = relu_pack(acc1[2 * m], acc1[2 * m + 1]);
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const bf8q w =
          *reinterpret_cast<const bf8q*>(&h[QB_W2 + (16 * n2 + li) * QB_P2 + 32 * m + 8 * lg]);
      acc2[n2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, acc2[n2], 0, 0, 0);
    }
  }
  if (rz2 && env < N) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r) rz2[(size_t)(16 * n2 + r) * RB + rec_lane_off] = acc2[n2][r];
  }
  zmask = rz1 ? quarter_mask(acc1, acc2) : 0u;
  f4q acc3;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc3[r] = lg == 0 ? lds[QB_B3 + r] : 0.0f;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const bf8q x = relu_pack(acc2[2 * m], acc2[2 * m + 1]);
    const bf8q w = *reinterpret_cast<const bf8q*>(&h[QB_W3 + li * QB_P2 + 32 * m + 8 * lg]);
    acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, acc3, 0, 0, 0);
  }
  const int src = li << 2;
#pragma unroll
  for (int o = 0; o < NA; ++o)
    z3[o] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(acc3[o])));
}

// Two waves per SIMD (256 registers each): one wave alone issues vector
// instructions at about half the rate the SIMD can execute them, two
// interleave theirs (matrix-core and vector instructions do not overlap,
// within a wave or across the two).
template <bool BF16, bool EXTRAS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_fused4(DevCfg c, SimBufs b, const float* __restrict__ W, int T, int t_base,
         float* __restrict__ rewards, uint8_t* __restrict__ dones, float* __restrict__ states,
         float* __restrict__ tape, int ckpt_every, const float* __restrict__ ck_in,
         RecSpan rs) {
  __shared__ __attribute__((aligned(16))) float lds[BF16 ? QB_TOTAL : Q_TOTAL];
  const int N = c.n_envs;
  if (BF16)
    stage_qb(W, lds);
  else
    stage_q(W, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63, j = lane & 15, k = lane >> 4;
  const int env0 = (blockIdx.x * blockDim.x + threadIdx.x - lane) / 4;  // first env of the wave
  if (env0 >= N) return;
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

  if (states && t_base == 0 && active)
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
    if (tape && (gt % ckpt_every) == 0 && active) {
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
    // observation state part: 18 features, this quarter keeps 4c + k
    quarter_state_features<EXTRAS>(c, (uint32_t)e, (uint32_t)ep, t_ep, k, x, F, sp);
    float* rt = rec_on ? ra.base + rec_step(rt_step, N) : nullptr;
    float z3[NA];
    uint32_t zmask;
    // per-lane part of record addresses, recomputed every step (see opaque())
    const uint32_t zoff = opaque((uint32_t)(rb_at(env0 + j, REC_F) + 4 * k * RB));
    const uint32_t koff = opaque((uint32_t)(rb_at(e, REC_F) + k * RB));
    const uint32_t roff = opaque((uint32_t)rb_at(e, REC_F));
    if (BF16)
      actor_qb(lds, F, z3, rec_on ? rt + (size_t)REC_Z1 * RB : nullptr,
               rec_on ? rt + (size_t)REC_Z2 * RB : nullptr, N, env0, zoff, zmask);
    else
      actor_q(lds, F, z3, rec_on ? rt + (size_t)REC_Z1 * RB : nullptr,
              rec_on ? rt + (size_t)REC_Z2 * RB : nullptr, N, env0, zoff, zmask);
    float a[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = tanh_act(z3[i]);
    if (rec_on && active) {
      // the state features (feature 4 cc + k); the history ones are earlier
      // actions, kept on the segment's action tape
#pragma unroll
      for (int cc = 0; cc < 5; ++cc)
        if (q_phi(cc, k) >= 0) rt[(size_t)(REC_O + 4 * cc) * RB + koff] = F[cc];
      // action tape of the segment: the checkpoint history once, then a_t
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
        float d[6];
        disturbance(c, (uint32_t)e, (uint32_t)ep, d);
        set_disturbance(B, d);
      }
    }
    if (ahead && (t & (RESERVE_PERIOD - 1)) == RESERVE_PERIOD - 1 && !have) {
      draw_ahead(c, (uint32_t)e, (uint32_t)(ep + 1), wh, nx);
      have = true;
    }
    if (active) {
      if (k == 0 && rewards) rewards[(size_t)gt * N + eo] = r;
      if (k == 1 && dones) dones[(size_t)gt * N + eo] = (uint8_t)d;
      if (states)
#pragma unroll
        for (int i = 0; i < NS; ++i)
          if ((i & 3) == k) states[((size_t)(gt + 1) * NS + i) * N + eo] = x[i];
    }
  }
  if (!active || REC) return;
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

hipError_t launch_fused4(const DevCfg& c, const SimBufs& b, const float* W, int T, int t_base,
                         float* rewards, uint8_t* dones, float* states, float* tape,
                         int ckpt_every, const float* ck_in, const RecSpan& rs, hipStream_t st) {
  if (!rec_span_ok(rs)) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((c.n_envs + 63) / 64);
  const bool bf = (c.flags & F_ACTOR_BF16) != 0;
  const bool ex = (c.flags & (F_DISTURB | F_OBS_NOISE)) != 0 || c.target != nullptr;
  auto k = bf ? (ex ? k_fused4<true, true> : k_fused4<true, false>)
              : (ex ? k_fused4<false, true> : k_fused4<false, false>);
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, c, b, W, T, t_base, rewards, dones, states,
                     tape, ckpt_every, ck_in, rs);
  return hipGetLastError();
}

}  // namespace qs
