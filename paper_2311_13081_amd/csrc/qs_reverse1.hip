// Reverse sweep of a segment with one env per lane (64 envs per wave, one
// 64-env block of the record), for large batches.
//
// The quarter-lane sweep (qs_backward.hip) repeats the dynamics adjoint on
// the four lanes of an env and needs about 440 registers, so it runs as
// rounds of one wave per SIMD with three quarters of its vector work
// duplicated.  Here every lane owns one env: the dynamics adjoint, the state
// adjoint (17), the history adjoint (32 x 4) and the parameter gradients are
// per lane, and only the actor's input VJP is spread over the lanes of the
// wave as matrix-core tiles:
//   dz3 = ga (1 - a^2)                       own lane;
//   dz2 = (W3^T dz3) [z2 > 0]                4-block v_mfma_f32_16x16x1f32, one
//        rank-1 update per action with B = the lane's own dz3 value (the
//        pattern of the forward's layer 1): register 4 bb + v of tile n
//        holds neuron 16 n + 4 lg + v of env 16 bb + li (lane li + 16 lg);
//   dz1 = (W2^T dz2) [z1 > 0]                v_mfma_f32_16x16x4f32 chained over
//        the dz2 registers as B operands (K-chunk = neurons 16 n + 4 k + v),
//        the same tile layout out;
//   do  = W1^T dz1                            the same over the dz1 registers,
//        ten 16-feature tiles; register r of block bb holds feature
//        16 p + 4 lg + r of env 16 bb + li;
// the ReLU masks come as bits in that tile layout from the one-lane
// forward's record (4 words per lane and step), so the sweep loads no
// pre-activations;
// and a 4 x 4 transpose across the lane groups (two permlane32 and two
// permlane16 swaps per register) brings every feature of a tile to the lane
// of its env, where the observation's share joins the state and history
// adjoints.  The per-step inputs and outputs use the blocked layouts of the
// record and the cotangent buffer (row f of env e at (e / 64) F 64 + 64 f +
// e % 64), so a lane's own-env rows are whole 256-byte rows of the wave.
#include "qs_actor.h"
#include "qs_backward.h"
#include "qs_forward.h"
#include "qs_reverse.h"

namespace qs {

// LDS (floats):
//   L_W3T[n][i]             = W3[i][n] (one 16-byte read: the 4 output weights of neuron n);
//   L_W2Q[mt][n][g][i][v]   = W2[16 n + 4 g + v][16 mt + i];
//   L_W1Q[p][mt][g][i][v]   = W1[16 mt + 4 g + v][16 p + i] (0 past feature 145).
constexpr int L_W3T = 0, L_W2Q = L_W3T + NHID * NA, L_W1Q = L_W2Q + NHID * NHID,
              L_TOTAL = L_W1Q + 10 * 4 * 4 * 16 * 4;
// History adjoint: the older HR slots of each env in a per-wave ring in LDS
// ([HR][4][64 lanes] after the weights: moving the slots one step older is a
// turn of the ring), the newest NH - HR in registers.  Each step adds the
// observation's share into every slot: in the ring that is a read, an add
// and a write of LDS per value, in registers an accumulator-register move or
// two.  Of HR = 4, 8, 16 and 24 (the largest the LDS holds for four waves),
// 8 measured fastest (377 us per 16-step segment at 65536 envs against 395
// for 24); with fewer the registers no longer fit beside the rest.
constexpr int HR = 8;
constexpr int L_RING = HR * NA * 64;
constexpr int L_BYTES = (L_TOTAL + 4 * L_RING) * 4;
static_assert(L_BYTES <= 160 * 1024, "weights and four history rings must fit in LDS");

__device__ inline void stage_reverse1(const float* __restrict__ W, float* lds, bool bf16) {
  stage_lds(lds + L_W3T, NHID * NA, W,
            [](int i) { return OFF_W3 + (i & 3) * NHID + (i >> 2); }, bf16);
  stage_lds(lds + L_W2Q, NHID * NHID, W, [](int i) {
    const int v = i & 3, li = (i >> 2) & 15, g = (i >> 6) & 3, n = (i >> 8) & 3, mt = i >> 10;
    return OFF_W2 + (16 * n + 4 * g + v) * NHID + 16 * mt + li;
  }, bf16);
  stage_lds(lds + L_W1Q, 10 * 4 * 4 * 16 * 4, W, [](int i) {
    const int v = i & 3, li = (i >> 2) & 15, g = (i >> 6) & 3, mt = (i >> 8) & 3, p = i >> 10;
    const int f = 16 * p + li, neuron = 16 * mt + 4 * g + v;
    return f < NO ? OFF_W1 + neuron * NO + f : -1;
  }, bf16);
}

// v where bit b of the mask word m is set, +0 elsewhere (the sign-extended
// one-bit field is all ones or zero)
__device__ inline float keep_if(float v, uint32_t m, int b) {
  return __uint_as_float(__float_as_uint(v) & (uint32_t)__builtin_amdgcn_sbfe((int)m, b, 1));
}

// Inputs of one reverse step: the own env's recorded state and action and
// cotangents, and the lane's ReLU mask words (column lane of the block).
struct StepIn1 {
  float x[NS], a[NA], dS[NS], dR;
  uint32_t m[4];
};

// sr: byte offset of the step's block in the record; vown / vlane: the
// lane's byte offsets of its env's column and of its own column.
__device__ inline void load_step1(StepIn1& in, __amdgpu_buffer_rsrc_t rrec, uint32_t sr,
                                  uint32_t vown, uint32_t vlane,
                                  const float* __restrict__ d_rewards,
                                  const float* __restrict__ d_states, int t, int N, int e) {
  const uint32_t eo = opaque((uint32_t)e);
#pragma unroll
  for (int w = 0; w < 4; ++w)
    in.m[w] = __float_as_uint(bld1(rrec, vlane, sr + 4u * (REC_M + w) * RB));
#pragma unroll
  for (int i = 0; i < NS; ++i) in.x[i] = bld1(rrec, vown, sr + 4u * (REC_X + i) * RB);
#pragma unroll
  for (int i = 0; i < NA; ++i) in.a[i] = bld1(rrec, vown, sr + 4u * (REC_A + i) * RB);
  in.dR = d_rewards ? d_rewards[(size_t)t * N + eo] : 1.0f;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    in.dS[i] = d_states ? d_states[((size_t)t * NS + i) * N + eo] : 0.0f;
}

// One segment of n steps (steps t0 .. t0 + n - 1 of the rollout), last to
// first.  lam ([145][N]) carries the state and history adjoints between
// segments, gth_io ([8][N]) the parameter gradients; dz receives the layer
// cotangents of every (step, env) of the segment.  Lanes of envs >= N
// shadow the block's first env (loads only), so every operand is finite.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_bwd_reverse1(DevCfg c, const float* __restrict__ theta, const float* __restrict__ W,
               const float* __restrict__ ck, const float* __restrict__ rec, int n, int t0,
               const float* __restrict__ d_rewards, const float* __restrict__ d_states,
               float* __restrict__ lam, float* __restrict__ gth_io, float* __restrict__ dz) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  stage_reverse1(W, lds, (c.flags & F_ACTOR_BF16) != 0);
  __syncthreads();
  const int N = c.n_envs;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int env0 = blockIdx.x * blockDim.x + threadIdx.x - lane;  // a 64-env block
  if (env0 >= N) return;
  const int env = env0 + lane;
  const bool active = env < N;
  const int e = active ? env : env0;
  // byte offsets: the block's record and cotangent spans within a step (wave
  // uniform), the lane's env column, its own column, and its place in a
  // matrix-core tile row (row 4 lg, column li)
  const uint32_t rbp = (uint32_t)rb_pad(N);
  const uint32_t blk = __builtin_amdgcn_readfirstlane(env0 / RB);
  const uint32_t s_rblk = 4u * blk * (REC_F * RB), s_zblk = 4u * blk * (DZ_F * RB);
  const uint32_t vown = 4u * (uint32_t)(e - env0), vlane = 4u * (uint32_t)lane;
  const uint32_t vtile = 4u * (uint32_t)(4 * lg * RB + li);
  const __amdgpu_buffer_rsrc_t rrec = span_rsrc(rec, 4u * (uint32_t)rec_floats(n, N));
  const __amdgpu_buffer_rsrc_t rdz = span_rsrc(dz, 4u * (uint32_t)n * DZ_F * rbp);

  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = theta[(size_t)i * N + e];
  Body<float> B = make_body<float>(th);
  {
    // the episode disturbance of the segment (no resets in a taped rollout)
    float d[6];
    disturbance(c, (uint32_t)e, (uint32_t)__float_as_int(ck[(size_t)CK_EP * N + e]), d);
    set_disturbance(B, d);
  }
  const bool renorm = (c.flags & F_RENORM_Q) != 0;

  // history adjoint: slot s < HR at ring row (s + base) mod HR, slot s >= HR
  // in lR[s - HR]
  float* ring = lds + L_TOTAL + (threadIdx.x >> 6) * L_RING + lane;
  int base = 0;
  float ls[NS], lR[NH - HR][NA], gth[NP];
#pragma unroll
  for (int i = 0; i < NS; ++i) ls[i] = lam[(size_t)i * N + e];
#pragma unroll
  for (int s = 0; s < NH; ++s)
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const float v = lam[(size_t)(NS + s * NA + a) * N + e];
      if (s < HR)
        ring[(s * NA + a) * 64] = v;
      else
        lR[s - HR][a] = v;
    }
#pragma unroll
  for (int i = 0; i < NP; ++i) gth[i] = gth_io[(size_t)i * N + e];

  StepIn1 cur, nxt;
  load_step1(cur, rrec, 4u * (uint32_t)(n - 1) * (REC_F * rbp) + s_rblk, vown, vlane, d_rewards,
             d_states, t0 + n - 1, N, e);
  for (int tl = n - 1; tl >= 0; --tl) {
    __asm__ volatile("" ::: "memory");
    const uint32_t sz = 4u * (uint32_t)tl * (DZ_F * rbp) + s_zblk;  // the step's cotangents
    const int tp = tl > 0 ? tl - 1 : 0;

    float gx[NS], ga[NA];
    reverse_dynamics(c, B, th, renorm, cur.x, cur.a, cur.dR, ls, lR[NH - HR - 1], gx, ga, gth);
    // the next step's inputs, in flight during the input VJP below
    load_step1(nxt, rrec, 4u * (uint32_t)tp * (REC_F * rbp) + s_rblk, vown, vlane, d_rewards,
               d_states, t0 + tp, N, e);
    // Lanes of envs >= N take dz3 = 0: the layer products keep envs apart
    // (one env per column), so their columns of dz2 and dz1 are zero too and
    // every lane stores unconditionally -- zeros into the slots of envs >= N,
    // which the weight-gradient pass expects there.
    float d3[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      d3[i] = active ? ga[i] * (1.0f - cur.a[i] * cur.a[i]) : 0.0f;
      bst1(d3[i], rdz, vlane, sz + 4u * (2 * NHID + i) * RB);
    }
    // dz2 = (W3^T dz3) [z2 > 0]: one rank-1 update per action
    f16 d2[4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const f4 w3 = *reinterpret_cast<const f4*>(&lds[L_W3T + 4 * (16 * n2 + li)]);
      d2[n2] = f16{};
#pragma unroll
      for (int i = 0; i < NA; ++i)
        d2[n2] = __builtin_amdgcn_mfma_f32_16x16x1f32(w3[i], d3[i], d2[n2], 0, 0, 0);
    }
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * bb + v;
          d2[n2][r] = keep_if(d2[n2][r], cur.m[2 + (n2 >> 1)], 16 * (n2 & 1) + r);
          bst1(d2[n2][r], rdz, vtile, sz + 4u * ((NHID + 16 * n2 + v) * RB + 16 * bb));
        }
    // dz1 = (W2^T dz2) [z1 > 0]: chains over the dz2 registers, 16 per
    // (tile, block)
    f4 d1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) d1[mt][bb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int n2 = 0; n2 < 4; ++n2) {
        const f4 wv =
            *reinterpret_cast<const f4*>(&lds[L_W2Q + (((mt * 4 + n2) * 4 + lg) * 16 + li) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            d1[mt][bb] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], d2[n2][4 * bb + v], d1[mt][bb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d1[mt][bb][r] = keep_if(d1[mt][bb][r], cur.m[mt >> 1], 16 * (mt & 1) + 4 * bb + r);
          bst1(d1[mt][bb][r], rdz, vtile, sz + 4u * ((16 * mt + r) * RB + 16 * bb));
        }

    // the history adjoint moves one slot older: H_t[s] feeds H_{t+1}[s - 1]
    // (registers shift, the ring turns; the ring's newest slot moves to the
    // registers and its freed row becomes the zero oldest slot)
    {
      const int top = (HR - 1 + base) % HR;
#pragma unroll
      for (int s = NH - HR - 1; s >= 1; --s)
#pragma unroll
        for (int a = 0; a < NA; ++a) lR[s][a] = lR[s - 1][a];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        lR[0][a] = ring[(top * NA + a) * 64];
        ring[(top * NA + a) * 64] = 0.0f;
      }
      base = __builtin_amdgcn_readfirstlane(top);  // wave-uniform
    }

    // do = W1^T dz1 tile by tile, each tile transposed into the env lanes
    float gf[18];
#pragma unroll
    for (int p = 0; p < 10; ++p) {
      f4 o[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) o[bb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const f4 wv =
            *reinterpret_cast<const f4*>(&lds[L_W1Q + (((p * 4 + mt) * 4 + lg) * 16 + li) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            o[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], d1[mt][bb][v], o[bb], 0, 0, 0);
      }
      // o[bb][r] in lane li + 16 lg: feature 16 p + 4 lg + r of env 16 bb + li.
      // Swapping the upper half of o[0] with the lower half of o[2] (and o[1]
      // with o[3]), then the odd 16-lane rows of the first results with the
      // even rows of the second, leaves in lane li + 16 bb the value of
      // lane group x of block bb in result x: feature 16 p + 4 x + r of the
      // lane's own env.
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const auto h02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(o[0][r]),
                                                          __float_as_uint(o[2][r]), false, false);
        const auto h13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(o[1][r]),
                                                          __float_as_uint(o[3][r]), false, false);
        const auto q01 = __builtin_amdgcn_permlane16_swap(h02[0], h13[0], false, false);
        const auto q23 = __builtin_amdgcn_permlane16_swap(h02[1], h13[1], false, false);
        const float val[4] = {__uint_as_float(q01[0]), __uint_as_float(q01[1]),
                              __uint_as_float(q23[0]), __uint_as_float(q23[1])};
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int f = 16 * p + 4 * x + r;
          const int sl = (f - 18) / NA, a = (f - 18) % NA;
          if (f < 18) {
            gf[f] = val[x];
          } else if (f < 18 + HR * NA) {
            const int row = (sl + base) % HR;
            ring[(row * NA + a) * 64] += val[x];
          } else if (f < NO) {
            lR[sl - HR][a] += val[x];
          }
        }
      }
    }
    // the state features' share: p, v, w directly, R(q) through its VJP
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      gx[i] += gf[i];
      gx[7 + i] += gf[12 + i];
      gx[10 + i] += gf[15 + i];
    }
    {
      float gq[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      const float q[4] = {cur.x[3], cur.x[4], cur.x[5], cur.x[6]};
      rotmat_vjp(q, gf + 3, gq);
#pragma unroll
      for (int i = 0; i < 4; ++i) gx[3 + i] += gq[i];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) ls[i] = gx[i] + cur.dS[i];
    cur = nxt;
  }
  if (!active) return;
  const uint32_t ef = opaque((uint32_t)e);
#pragma unroll
  for (int i = 0; i < NS; ++i) lam[(size_t)i * N + ef] = ls[i];
#pragma unroll
  for (int s = 0; s < NH; ++s)
#pragma unroll
    for (int a = 0; a < NA; ++a)
      lam[(size_t)(NS + s * NA + a) * N + ef] =
          s < HR ? ring[(((s + base) % HR) * NA + a) * 64] : lR[s - HR][a];
#pragma unroll
  for (int i = 0; i < NP; ++i) gth_io[(size_t)i * N + ef] = gth[i];
}

static inline unsigned nblk(int n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t reverse1_prepare() {
  return hipFuncSetAttribute((const void*)k_bwd_reverse1,
                             hipFuncAttributeMaxDynamicSharedMemorySize, L_BYTES);
}

hipError_t launch_reverse1(const DevCfg& c, const float* theta, const float* W, const float* ck,
                           const float* rec, int n, int t0, const float* d_rewards,
                           const float* d_states, float* lam, float* gth, float* dz,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_bwd_reverse1, dim3(nblk(c.n_envs, 256)), dim3(256), L_BYTES, st, c,
                     theta, W, ck, rec, n, t0, d_rewards, d_states, lam, gth, dz);
  return hipGetLastError();
}

}  // namespace qs
