// Forward kernels of the batched quadrotor step: initialisation and reset,
// snapshots, and the plain five-kernel step (the fused kernels live in
// qs_fused.hip and qs_fused4.hip, dynamics-only rollouts in qs_dynamics.hip).
//
// Layout: one env per lane, struct-of-arrays in HBM ([K][N]) so every global
// access of a wave is a contiguous 256-byte segment.
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
  b.ret[e] = 0.0f;
  b.ret[(size_t)N + e] = 0.0f;
  b.last_len[e] = 0;
}

// Snapshot copies.  Each thread loads a batch of rows before storing any of
// them: the source and destination may not be assumed disjoint, so a
// load-store-load sequence would wait out one memory round trip per row.
__global__ void k_get_state(SimBufs b, int N, float* state, float* hist, int32_t* t_ep,
                            int32_t* ep, float* ret, int32_t* last_len) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state) {
    float v[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = b.state[i * N + e];
#pragma unroll
    for (int i = 0; i < NS; ++i) state[i * N + e] = v[i];
  }
  if (hist) {
    const int h = b.head[e];
#pragma unroll
    for (int s0 = 0; s0 < NH; s0 += 8) {
      float v[8 * NA];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int slot = (h + s0 + s) & (NH - 1);
#pragma unroll
        for (int a = 0; a < NA; ++a) v[s * NA + a] = b.ring[(slot * NA + a) * N + e];
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int a = 0; a < NA; ++a) hist[((s0 + s) * NA + a) * N + e] = v[s * NA + a];
    }
  }
  if (t_ep) t_ep[e] = b.t_ep[e];
  if (ep) ep[e] = b.ep[e];
  if (ret) {
    const float r0 = b.ret[e], r1 = b.ret[(size_t)N + e];
    ret[e] = r0;
    ret[(size_t)N + e] = r1;
  }
  if (last_len) last_len[e] = b.last_len[e];
}

__global__ void k_set_state(SimBufs b, int N, const float* state, const float* hist,
                            const int32_t* t_ep, const int32_t* ep, const float* ret,
                            const int32_t* last_len) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state) {
    float v[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = state[i * N + e];
#pragma unroll
    for (int i = 0; i < NS; ++i) b.state[i * N + e] = v[i];
  }
  if (hist) {
#pragma unroll
    for (int i0 = 0; i0 < NH * NA; i0 += 32) {
      float v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = hist[(i0 + i) * N + e];
#pragma unroll
      for (int i = 0; i < 32; ++i) b.ring[(i0 + i) * N + e] = v[i];
    }
    b.head[e] = 0;
  }
  if (t_ep) b.t_ep[e] = t_ep[e];
  if (ep) b.ep[e] = ep[e];
  if (ret) {
    const float r0 = ret[e], r1 = ret[(size_t)N + e];
    b.ret[e] = r0;
    b.ret[(size_t)N + e] = r1;
  }
  if (last_len) b.last_len[e] = last_len[e];
}

// ---------------------------------------------------------------------------
// Plain path: five kernels per step, every intermediate through HBM.
// ---------------------------------------------------------------------------

// obs[146][N] = {p, R(q), v, w, H oldest..newest}
__global__ void __launch_bounds__(256) k_plain_obs(DevCfg c, SimBufs b, float* __restrict__ obs) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float q[4], f[18];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = b.state[(3 + i) * N + e];
  rotmat(q, f + 3);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    f[i] = b.state[i * N + e];
    f[12 + i] = b.state[(7 + i) * N + e];
    f[15 + i] = b.state[(10 + i) * N + e];
  }
  SetPoint sp;
  sp.load(c, N, e);
  sp.apply(c, f);
  add_obs_noise(c, (uint32_t)e, (uint32_t)b.ep[e], b.t_ep[e], f);
#pragma unroll
  for (int i = 0; i < 18; ++i) obs[i * N + e] = f[i];
  const int h = b.head[e];
  for (int s = 0; s < NH; ++s) {
    const int slot = (h + s) & (NH - 1);
#pragma unroll
    for (int a = 0; a < NA; ++a)
      obs[(size_t)(18 + s * NA + a) * N + e] = b.ring[(slot * NA + a) * N + e];
  }
}

// The three actor layers of the plain path on fp32 matrix cores, in the
// product order and lane layout of the fused kernel's actor; only the layer
// outputs go through HBM ([64][N], [64][N], [4][N]).  The hidden layers give
// each 64-env block two waves, one per half of the neuron tiles (a
// workgroup of four waves takes 128 envs), so two waves share a SIMD and one
// wave's loads and stores overlap the other's products.  Lanes of envs past
// the batch load the last env and store nothing.
//
// Layer 1, h1[64][N] = ReLU(W1 obs + b1): 147 rank-1 updates per 16-neuron
// tile with the 4-block 16x16x1 product, the bias first (a constant input 1);
// B = input k of the lane's env, A = the weights of 16 neurons for all four
// 16-env blocks.  Result register 4 bb + v of tile n holds neuron 16 n + 4 g
// + v of env 16 bb + i (lane 16 g + i).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_plain_l1_mfma(int N, const float* __restrict__ W, const float* __restrict__ in,
                float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float sW[NHID * M_W1_LD];
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wv = threadIdx.x >> 6, th = wv & 1;  // tiles 2 th, 2 th + 1
  const int first = blockIdx.x * 128 + 64 * (wv >> 1);
  // every input load in flight before the weights are staged
  const int e = min(first + lane, N - 1);
  float xin[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) xin[k] = in[(size_t)k * N + e];
  __builtin_amdgcn_sched_barrier(0);
  stage_lds(sW, NHID * M_W1_LD, W, [](int i) {
    const int r = i / M_W1_LD, k = i % M_W1_LD;
    return k == 0 ? OFF_B1 + r : k <= NO ? OFF_W1 + r * NO + k - 1 : -1;
  });
  __syncthreads();
  if (first >= N) return;
  const f16 zero16 = {};
  f16 acc[2];
#pragma unroll
  for (int kc = 0; kc < M_W1_LD / 4; ++kc) {
    f4 w[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
      w[j] = *reinterpret_cast<const f4*>(&sW[(16 * (2 * th + j) + li) * M_W1_LD + 4 * kc]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int col = 4 * kc + kk;  // 0: bias, k + 1: input k
      if (col == 0) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x1f32(w[j][0], 1.0f, zero16, 0, 0, 0);
      } else if (col <= NO) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x1f32(w[j][kk], xin[col - 1], acc[j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int oe = first + 16 * bb + li;
    if (oe < N)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(16 * (2 * th + j) + 4 * lg + v) * N + oe] = relu_bits(acc[j][4 * bb + v]);
  }
}

// Layer 2, h2[64][N] = ReLU(W2 h1 + b2): 16x16x4 products, chain (n2, bb)
// for neurons 16 n2.. and envs 16 bb..; the K-chunk of product (n, v) is
// the inputs {16 n + 4 g + v} (lane 16 g + i holds input 16 n + 4 g + v of
// env 16 bb + i), the bias tile the accumulator input of the first product.
// Result register v of chain (n2, bb): neuron 16 n2 + 4 g + v of env 16 bb + i.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_plain_l2_mfma(int N, const float* __restrict__ W, const float* __restrict__ in,
                float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float sW[NHID * M_W2_LD];
  __shared__ __attribute__((aligned(16))) float sb[NHID];
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wv = threadIdx.x >> 6, th = wv & 1;  // tiles n2 = 2 th, 2 th + 1
  const int first = blockIdx.x * 128 + 64 * (wv >> 1);
  // every input load in flight before the weights are staged: x[n][v][bb]
  float x[4][4][4];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int e = min(first + 16 * bb + li, N - 1);
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v) x[n][v][bb] = in[(size_t)(16 * n + 4 * lg + v) * N + e];
  }
  __builtin_amdgcn_sched_barrier(0);
  stage_lds(sW, NHID * M_W2_LD, W, [](int i) {
    const int r = i / M_W2_LD, k = i % M_W2_LD;
    return k < NHID ? OFF_W2 + r * NHID + k : -1;
  });
  stage_lds(sb, NHID, W, [](int i) { return OFF_B2 + i; });
  __syncthreads();
  if (first >= N) return;
  f4 acc[2][4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n2 = 2 * th + j;
      const f4 w = *reinterpret_cast<const f4*>(&sW[(16 * n2 + li) * M_W2_LD + 16 * n + 4 * lg]);
      const f4 b2 = *reinterpret_cast<const f4*>(&sb[16 * n2 + 4 * lg]);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          acc[j][bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              w[v], x[n][v][bb], (n == 0 && v == 0) ? b2 : acc[j][bb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int oe = first + 16 * bb + li;
    if (oe < N)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(16 * (2 * th + j) + 4 * lg + v) * N + oe] = relu_bits(acc[j][bb][v]);
  }
}

// Layer 3, act[4][N] = tanh(W3 h2 + b3): the input registers of the fused
// kernel's layer 3 (register v of (n2, bb) in lane 16 g + i: input 16 n2 + 4 g
// + v of env 16 bb + i) loaded from h2, then the same 4x4x1 products and
// cross-lane sums (layer3_one_lane).
__global__ void __launch_bounds__(256) k_plain_l3_mfma(int N, const float* __restrict__ W,
                                                       const float* __restrict__ in,
                                                       float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float sW[NA * M_W2_LD + NA];  // W3 rows, then b3
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int first = blockIdx.x * blockDim.x + threadIdx.x - lane;
  f4 h[4][4];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int e = min(first + 16 * bb + li, N - 1);
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int v = 0; v < 4; ++v) h[n2][bb][v] = in[(size_t)(16 * n2 + 4 * lg + v) * N + e];
  }
  __builtin_amdgcn_sched_barrier(0);
  stage_lds(sW, NA * M_W2_LD, W, [](int i) {
    const int r = i / M_W2_LD, k = i % M_W2_LD;
    return k < NHID ? OFF_W3 + r * NHID + k : -1;
  });
  stage_lds(sW + NA * M_W2_LD, NA, W, [](int i) { return OFF_B3 + i; });
  __syncthreads();
  if (first >= N) return;
  float z3[NA];
  layer3_one_lane(sW, 0, NA * M_W2_LD, h, z3);
  if (first + lane < N)
#pragma unroll
    for (int o = 0; o < NA; ++o) out[(size_t)o * N + first + lane] = tanh_act(z3[o]);
}

// Dynamics, reward, history push, episode bookkeeping and reset.  DIST: the
// dynamics carry the episode disturbance terms (instantiated as the fused
// kernel instantiates its dynamics: with the training extras or a set point).
template <bool DIST>
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
  Body<float> B = make_body<float>(th);
  if (DIST) {
    float dist[6];
    disturbance(c, (uint32_t)e, (uint32_t)b.ep[e], dist);
    set_disturbance(B, dist);
  }
  rk4_step<float, DIST>(B, c.arm, c.km, c.g, c.dt, (c.flags & F_RENORM_Q) != 0, x, u);
  const float r = reward(c, x, a);
  int h = b.head[e];
#pragma unroll
  for (int i = 0; i < NA; ++i) b.ring[(h * NA + i) * N + e] = a[i];
  h = (h + 1) & (NH - 1);
  int t_ep = b.t_ep[e] + 1;
  const uint32_t d = episode_end(c, x, t_ep);
  EpAcc acc;
  acc.load(b, N, e);
  acc.add(r, d && (c.flags & F_AUTORESET), t_ep);
  acc.store(b, N, (uint32_t)e);
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

// Observations of the current state (for a caller that runs its own policy
// or critic): the actor observation with the noise of the coming step, and
// the critic's privileged observation {p, R, v, w, w_m, f_r, tau_r} (Sec. IV).
__global__ void __launch_bounds__(256) k_observe(DevCfg c, SimBufs b, float* __restrict__ aobs,
                                                 float* __restrict__ cobs) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  float x[NS], f[18];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = b.state[i * N + e];
  rotmat(x + 3, f + 3);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    f[i] = x[i];
    f[12 + i] = x[7 + i];
    f[15 + i] = x[10 + i];
  }
  const uint32_t ep = (uint32_t)b.ep[e];
  if (cobs) {
    float d[6];
    disturbance(c, (uint32_t)e, ep, d);
#pragma unroll
    for (int i = 0; i < 18; ++i) cobs[i * N + e] = f[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) cobs[(18 + i) * N + e] = x[13 + i];
#pragma unroll
    for (int i = 0; i < 6; ++i) cobs[(22 + i) * N + e] = d[i];
  }
  if (aobs) {
    SetPoint sp;
    sp.load(c, N, e);
    sp.apply(c, f);
    add_obs_noise(c, (uint32_t)e, ep, b.t_ep[e], f);
#pragma unroll
    for (int i = 0; i < 18; ++i) aobs[i * N + e] = f[i];
    const int h = b.head[e];
    for (int s = 0; s < NH; ++s) {
      const int slot = (h + s) & (NH - 1);
#pragma unroll
      for (int a = 0; a < NA; ++a)
        aobs[(size_t)(18 + s * NA + a) * N + e] = b.ring[(slot * NA + a) * N + e];
    }
  }
}

// Ends the episodes of the envs with mask[e] != 0 and starts their next ones,
// as an in-step reset does: episode + 1, step 0, the start state of (env,
// episode + 1), the history filled with the env's hover action, and the
// episode accumulators closed (the running return and the step count become
// the last finished episode's).
__global__ void k_reset_envs(DevCfg c, SimBufs b, const uint8_t* __restrict__ mask) {
  const int N = c.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N || !mask[e]) return;
  float th[NP], s[NS];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  const int ep = b.ep[e] + 1;
  const float ah = reset_state(c, (uint32_t)e, (uint32_t)ep, th[0], th[4], th[5], th[6], s);
#pragma unroll
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = s[i];
  for (int i = 0; i < NH * NA; ++i) b.ring[(size_t)i * N + e] = ah;
  b.ret[(size_t)N + e] = b.ret[e];
  b.ret[e] = 0.0f;
  b.last_len[e] = b.t_ep[e];
  b.head[e] = 0;
  b.t_ep[e] = 0;
  b.ep[e] = ep;
}

// Rewards of given transitions under the configured reward constants: r(s',
// a) of the reward equation (Sec. IV) for M post-step states s [17][M] and
// actions a [4][M] (e.g. a replay buffer re-scored after the constants
// changed).
__global__ void __launch_bounds__(256) k_reward_batch(DevCfg c, const float* __restrict__ s,
                                                      const float* __restrict__ a, int M,
                                                      float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  float x[NS], u[NA];
#pragma unroll
  for (int k = 0; k < NS; ++k) x[k] = s[(size_t)k * M + i];
#pragma unroll
  for (int k = 0; k < NA; ++k) u[k] = a[(size_t)k * M + i];
  out[i] = reward(c, x, u);
}

// Copies the state to a [17][N] slice (start state of a recorded rollout).
__global__ void k_copy_state(SimBufs b, int N, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i * N + e] = b.state[i * N + e];
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
                            int32_t* ep, float* ret, int32_t* last_len, hipStream_t st) {
  hipLaunchKernelGGL(k_get_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, state, hist, t_ep,
                     ep, ret, last_len);
  return hipGetLastError();
}

hipError_t launch_set_state(const SimBufs& b, int N, const float* state, const float* hist,
                            const int32_t* t_ep, const int32_t* ep, const float* ret,
                            const int32_t* last_len, hipStream_t st) {
  hipLaunchKernelGGL(k_set_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, state, hist, t_ep,
                     ep, ret, last_len);
  return hipGetLastError();
}

hipError_t launch_plain_step(const DevCfg& c, const SimBufs& b, const PlainBufs& p,
                             const float* W, const float* ext_act, float* reward, uint8_t* done,
                             float* state_out, hipStream_t st) {
  const int N = c.n_envs;
  const dim3 g(nblk(N, 256)), blk(256);
  const float* act = ext_act;
  if (!ext_act) {
    hipLaunchKernelGGL(k_plain_obs, g, blk, 0, st, c, b, p.obs);
    const dim3 g2(nblk(N, 128));  // 128 envs per workgroup (two waves per 64-env block)
    hipLaunchKernelGGL(k_plain_l1_mfma, g2, blk, 0, st, N, W, p.obs, p.h1);
    hipLaunchKernelGGL(k_plain_l2_mfma, g2, blk, 0, st, N, W, p.h1, p.h2);
    hipLaunchKernelGGL(k_plain_l3_mfma, g, blk, 0, st, N, W, p.h2, p.act);
    act = p.act;
  }
  const bool ex = (c.flags & (F_DISTURB | F_OBS_NOISE)) != 0 || c.target != nullptr;
  hipLaunchKernelGGL(ex ? k_plain_dyn<true> : k_plain_dyn<false>, g, blk, 0, st, c, b, act,
                     reward, done, state_out);
  return hipGetLastError();
}


hipError_t launch_observe(const DevCfg& c, const SimBufs& b, float* actor_obs, float* critic_obs,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_observe, dim3(nblk(c.n_envs, 256)), dim3(256), 0, st, c, b, actor_obs,
                     critic_obs);
  return hipGetLastError();
}

hipError_t launch_reset_envs(const DevCfg& c, const SimBufs& b, const uint8_t* mask,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_reset_envs, dim3(nblk(c.n_envs, 256)), dim3(256), 0, st, c, b, mask);
  return hipGetLastError();
}

hipError_t launch_reward_batch(const DevCfg& c, const float* s, const float* a, int M, float* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_reward_batch, dim3(nblk(M, 256)), dim3(256), 0, st, c, s, a, M, out);
  return hipGetLastError();
}

hipError_t launch_copy_state(const SimBufs& b, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_state, dim3(nblk(N, 256)), dim3(256), 0, st, b, N, out);
  return hipGetLastError();
}


hipError_t launch_recompute(const DevCfg& c, const SimBufs& b, const float* W, int T,
                            const float* ck_in, float* rec, hipStream_t st) {
  // the kernel of taped rollouts, in record mode: one segment of T steps
  const RecSpan one{{rec, nullptr, nullptr, nullptr}, 0, T, T};
  switch (taped_kernel(c)) {
    case TAPED_SPLIT:
      return launch_split(c, b, W, T, 0, nullptr, nullptr, nullptr, nullptr, 1, ck_in, one, st);
    case TAPED_LANE:
      return launch_fused_taped(c, b, W, T, 0, nullptr, nullptr, nullptr, nullptr, 1, ck_in, one,
                                st);
    default:
      return launch_fused4(c, b, W, T, 0, nullptr, nullptr, nullptr, nullptr, 1, ck_in, one, st);
  }
}

}  // namespace qs
