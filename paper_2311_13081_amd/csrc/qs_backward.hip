// Discrete adjoint of a taped rollout.
//
// The taped forward stored checkpoints (state, history) every K steps.  The
// backward walks the segments last to first; per segment:
//   1. recompute: the fused MFMA kernel restarts from the checkpoint and
//      records x_t, a_t, the layer pre-activations z1, z2 and the state
//      features of o_t per step (the history features are earlier actions);
//   2. reverse sweep (k_bwd_reverse): four lanes per env, the adjoints of
//      the state and of the action history in registers, stepping back
//      through reward, quaternion renormalisation, the four RK4 stages, the
//      action map, the actor (on MFMA) and the history shift; per-env
//      parameter gradients accumulate in registers; the layer cotangents
//      dz1, dz2, dz3 of every (step, env) go to scratch;
//   3. weight gradients (k_bwd_dw): sum over (step, env) rows of dz (x) input
//      on fp32 MFMA, one workgroup per (64-env chunk, step group)
//      accumulating into its own partial; biases come from a constant-one
//      input column.
// Finally k_bwd_reduce adds the workgroup partials in a fixed order, so the
// result does not depend on scheduling.
#include "qs_actor.h"
#include "qs_backward.h"
#include "qs_forward.h"
#include "qs_reverse.h"

namespace qs {

static inline unsigned nb(int n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// lam = (dS_T, 0), gth = 0.
__global__ void k_bwd_init(int N, const float* __restrict__ dS_T, float* __restrict__ lam,
                           float* __restrict__ gth) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  for (int i = 0; i < NS; ++i) lam[(size_t)i * N + e] = dS_T ? dS_T[(size_t)i * N + e] : 0.0f;
  for (int i = NS; i < LAM_F; ++i) lam[(size_t)i * N + e] = 0.0f;
  for (int i = 0; i < NP; ++i) gth[(size_t)i * N + e] = 0.0f;
}

// Reverse sweep in the quarter-lane layout (16 envs per wave, lane L = j +
// 16 k: env j, quarter k), the adjoint of the forward step (the quarter-lane
// or the split-actor kernel, which compute the same values).  Per lane:
// the state adjoint (17) and the dynamics VJP, replicated over the 4 quarters
// of an env; the history adjoint of action component k (32 slots).  The actor
// VJP runs on 16x16x4 fp32 MFMAs:
//   dh2 = W3^T dz3: one K=4 MFMA per 16-neuron tile (quarter k supplies
//         dz3[k]);
//   dh1 = W2^T dz2, do = W1^T dz1: chained through the result registers.
// The rows of W1^T are taken in the forward's observation order, so tile p
// of do leaves in quarter k exactly the features PHI(4p + r, k): history
// slot 4p + r - 5, component k (the lane's own history adjoint) or, for
// chunks 0..4, state features 4c + k, gathered across quarters with 20
// lane shuffles.
//
// LDS (floats):
//   R_W3 [4][64] = W3;
//   R_W2P[((n*4 + g)*4 + m)*16 + i][v] = W2[16n + 4g + v][16m + i];
//   R_W1P[((m*4 + g)*10 + p)*16 + i][v] = W1[16m + 4g + v][PHI(4p + i%4, i/4)] (0 if pad).
constexpr int R_W3 = 0, R_W2P = R_W3 + NA * NHID, R_W1P = R_W2P + NHID * NHID,
              R_TOTAL = R_W1P + 10 * 16 * NHID;

__host__ __device__ constexpr int r_phi(int c, int k) {
  return c < 5 ? (4 * c + k < 18 ? 4 * c + k : -1) : c < 37 ? 18 + 4 * (c - 5) + k : -1;
}

__device__ inline void stage_reverse(const float* __restrict__ W, float* lds, bool bf16) {
  stage_lds(lds + R_W3, NA * NHID, W, [](int i) { return OFF_W3 + i; }, bf16);
  stage_lds(lds + R_W2P, NHID * NHID, W, [](int idx) {
    const int v = idx & 3, i = (idx >> 2) & 15, m = (idx >> 6) & 3, g = (idx >> 8) & 3,
              n = idx >> 10;
    return OFF_W2 + (16 * n + 4 * g + v) * NHID + 16 * m + i;
  }, bf16);
  stage_lds(lds + R_W1P, 10 * 16 * NHID, W, [](int idx) {
    const int v = idx & 3, i = (idx >> 2) & 15, rest = idx >> 6;  // rest = (m*4 + g)*10 + p
    const int p = rest % 10, g = (rest / 10) & 3, m = rest / 40;
    const int feat = r_phi(4 * p + (i & 3), i >> 2);
    return feat >= 0 ? OFF_W1 + (16 * m + 4 * g + v) * NO + feat : -1;
  }, bf16);
}

// Inputs of one reverse step: the recorded state and action, this lane's
// ReLU mask word (quarter_mask: the signs of its 16 layer-1 and 16 layer-2
// pre-activations, neurons 16 q + 4 k + r), the reward and state cotangents.
struct StepIn {
  float x[NS], a[NA], dS[NS], dR;
  uint32_t zm;
};

__device__ inline void load_step(StepIn& in, const float* __restrict__ rec,
                                 const float* __restrict__ d_rewards,
                                 const float* __restrict__ d_states, int tl, int t0, int N, int e,
                                 int k) {
  const uint32_t eo = opaque((uint32_t)e);
  const uint32_t roff = opaque((uint32_t)rb_at(e, REC_F));
  const uint32_t koff = opaque((uint32_t)(rb_at(e, REC_F) + k * RB));
  const int t = t0 + tl;
  const float* rt = rec + rec_step(tl, N);
#pragma unroll
  for (int i = 0; i < NS; ++i) in.x[i] = rt[(size_t)(REC_X + i) * RB + roff];
#pragma unroll
  for (int i = 0; i < NA; ++i) in.a[i] = rt[(size_t)(REC_A + i) * RB + roff];
  in.zm = __float_as_uint(rt[(size_t)REC_M * RB + koff]);
  in.dR = d_rewards ? d_rewards[(size_t)t * N + eo] : 1.0f;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    in.dS[i] = d_states ? d_states[((size_t)t * NS + i) * N + eo] : 0.0f;
}


// The observation's share of the adjoints, from do (dob: tile p, register r
// of quarter k = the cotangent of feature PHI(4p + r, k)): shifts the
// history adjoint (H_t[s] feeds H_{t+1}[s-1]), gathers the 18 state features
// from the quarters, adds them (through R(q)) to gx and forms the state
// adjoint before the step, ls = gx + dS.
__device__ __forceinline__ void reverse_observation(const float dob[40], const float x[NS],
                                                    const float dS[NS], int j, float gx[NS],
                                                    float lH[NH], float ls[NS]) {
  // descending s reads the older adjoint before it is overwritten
#pragma unroll
  for (int s = NH - 1; s >= 0; --s) lH[s] = (s >= 1 ? lH[s - 1] : 0.0f) + dob[5 + s];
  // state features 4cc + q live in quarter q: gather them into every lane
  float gf[20];
#pragma unroll
  for (int cc = 0; cc < 5; ++cc)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      gf[4 * cc + q] = __int_as_float(
          __builtin_amdgcn_ds_bpermute((j + 16 * q) << 2, __float_as_int(dob[cc])));
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gx[i] += gf[i];
    gx[7 + i] += gf[12 + i];
    gx[10 + i] += gf[15 + i];
  }
  {
    float gq[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const float q[4] = {x[3], x[4], x[5], x[6]};
    rotmat_vjp(q, gf + 3, gq);
#pragma unroll
    for (int i = 0; i < 4; ++i) gx[3 + i] += gq[i];
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) ls[i] = gx[i] + dS[i];
}

// Exchange space of the split sweep, after the staged weights: dz2 and dz1
// tiles [4][64] and do tiles [10][64] (f4 each).
constexpr int R_XCH = (4 + 4 + 10) * 64 * 4;
// Batches up to this size run the split sweep (four times the waves; the
// quarter-lane sweep leaves most SIMDs idle there).
constexpr int REVERSE_SPLIT_MAX_ENVS = 4096;
// Segments recorded by the one-env-per-lane forward (taped_kernel) run the
// one-env-per-lane sweep (qs_reverse1.hip), which reads that kernel's ReLU
// mask rows: one wave of 64 envs per SIMD and no repeated dynamics adjoint.

// Reverse sweep of one segment.  SPLIT = false: 16 envs per wave in the
// quarter-lane layout.  SPLIT = true: 16 envs per workgroup of 4 waves, each
// in that layout; wave w evaluates neuron tile w of dz2 and dz1 and the do
// tiles w, w + 4, w + 8 on MFMA, the tiles go through LDS (three barriers a
// step, each exchange buffer rewritten only after the barrier that follows
// every wave's reads of it), and every wave runs the dynamics and the
// observation adjoints.  The MFMA chains of each tile are the same in both,
// so they agree bit for bit.
template <bool SPLIT>
__global__ void __launch_bounds__(256)
k_bwd_reverse(DevCfg c, const float* __restrict__ theta, const float* __restrict__ W,
              const float* __restrict__ ck, const float* __restrict__ rec, int n, int t0,
              const float* __restrict__ d_rewards,
              const float* __restrict__ d_states, float* __restrict__ lam,
              float* __restrict__ gth_io, float* __restrict__ dz) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  stage_reverse(W, lds, (c.flags & F_ACTOR_BF16) != 0);
  __syncthreads();
  const int N = c.n_envs;
  const int lane = threadIdx.x & 63, j = lane & 15, k = lane >> 4;
  const int w = SPLIT ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const int env0 = SPLIT ? blockIdx.x * 16 : (blockIdx.x * blockDim.x + threadIdx.x - lane) / 4;
  if (env0 >= N) return;  // SPLIT: the whole workgroup
  const int env = env0 + j;
  const bool active = env < N;
  const int e = active ? env : env0;
  f4* xd2 = reinterpret_cast<f4*>(lds + R_TOTAL);
  f4* xd1 = xd2 + 4 * 64;
  f4* xdo = xd1 + 4 * 64;

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

  float ls[NS], lH[NH], gth[NP];
#pragma unroll
  for (int i = 0; i < NS; ++i) ls[i] = lam[(size_t)i * N + e];
#pragma unroll
  for (int s = 0; s < NH; ++s) lH[s] = lam[(size_t)(NS + s * NA + k) * N + e];
#pragma unroll
  for (int i = 0; i < NP; ++i) gth[i] = gth_io[(size_t)i * N + e];

  // The per-step inputs (record rows and cotangents) of step tl - 1 are
  // loaded while step tl is processed, so their latency hides behind it.
  StepIn cur, nxt;
  load_step(cur, rec, d_rewards, d_states, n - 1, t0, N, e, k);
  for (int tl = n - 1; tl >= 0; --tl) {
    __asm__ volatile("" ::: "memory");
    load_step(nxt, rec, d_rewards, d_states, tl > 0 ? tl - 1 : 0, t0, N, e, k);
    // blocked cotangent rows of this env: row k and row 4k
    const uint32_t koff = opaque((uint32_t)(rb_at(e, DZ_F) + k * RB));
    const uint32_t zoff = opaque((uint32_t)(rb_at(e, DZ_F) + 4 * k * RB));
    float* dzt = dz + (size_t)tl * DZ_F * rb_pad(N);

    float gx[NS], ga[NA];
    // newest history slot: component i lives in quarter i of the same env
    float hn[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i)
      hn[i] = __int_as_float(
          __builtin_amdgcn_ds_bpermute((j + 16 * i) << 2, __float_as_int(lH[NH - 1])));
    reverse_dynamics(c, B, th, renorm, cur.x, cur.a, cur.dR, ls, hn, gx, ga, gth);

    // --- actor VJP on matrix cores --------------------------------------------
    float d3[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) d3[i] = ga[i] * (1.0f - cur.a[i] * cur.a[i]);
    const float d3k = k == 0 ? d3[0] : k == 1 ? d3[1] : k == 2 ? d3[2] : d3[3];
    if (active && w == 0) dzt[(size_t)(2 * NHID) * RB + koff] = d3k;
    // do = W1^T dz1 in observation order: tile p, register r of quarter k is
    // the cotangent of feature PHI(4p + r, k)
    float dob[40];
    if (!SPLIT) {
      // dz2 = (W3^T dz3) * [z2 > 0]: tile q rows 16q + 4k + r, env j
      f4 dz2[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        dz2[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(lds[R_W3 + k * NHID + 16 * q + j], d3k,
                                                      f4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dz2[q][r] = (cur.zm >> (8 * q + 4 + r)) & 1u ? dz2[q][r] : 0.0f;
          if (active) dzt[(size_t)(NHID + 16 * q + r) * RB + zoff] = dz2[q][r];
        }
      }
      // dz1 = (W2^T dz2) * [z1 > 0]
      f4 dz1[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f4 accm = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f4 wv = *reinterpret_cast<const f4*>(
              &lds[R_W2P + (((q * 4 + k) * 4 + mt) * 16 + j) * 4]);
#pragma unroll
          for (int v = 0; v < 4; ++v)
            accm = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], dz2[q][v], accm, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dz1[mt][r] = (cur.zm >> (8 * mt + r)) & 1u ? accm[r] : 0.0f;
          if (active) dzt[(size_t)(16 * mt + r) * RB + zoff] = dz1[mt][r];
        }
      }
#pragma unroll
      for (int p = 0; p < 10; ++p) {
        f4 accp = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const f4 wv = *reinterpret_cast<const f4*>(
              &lds[R_W1P + (((mt * 4 + k) * 10 + p) * 16 + j) * 4]);
#pragma unroll
          for (int v = 0; v < 4; ++v)
            accp = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], dz1[mt][v], accp, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) dob[4 * p + r] = accp[r];
      }
    } else {
      // dz2 tile w
      f4 d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(lds[R_W3 + k * NHID + 16 * w + j], d3k,
                                                   f4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        d2[r] = (cur.zm >> (8 * w + 4 + r)) & 1u ? d2[r] : 0.0f;
        if (active) dzt[(size_t)(NHID + 16 * w + r) * RB + zoff] = d2[r];
      }
      xd2[w * 64 + lane] = d2;
      __syncthreads();
      f4 dz2[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) dz2[q] = xd2[q * 64 + lane];
      // dz1 tile w
      f4 accm = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4 wv =
            *reinterpret_cast<const f4*>(&lds[R_W2P + (((q * 4 + k) * 4 + w) * 16 + j) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          accm = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], dz2[q][v], accm, 0, 0, 0);
      }
      f4 d1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        d1[r] = (cur.zm >> (8 * w + r)) & 1u ? accm[r] : 0.0f;
        if (active) dzt[(size_t)(16 * w + r) * RB + zoff] = d1[r];
      }
      xd1[w * 64 + lane] = d1;
      __syncthreads();
      f4 dz1[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) dz1[mt] = xd1[mt * 64 + lane];
      // do tiles w, w + 4, w + 8
#pragma unroll
      for (int pi = 0; pi < 3; ++pi) {
        const int p = w + 4 * pi;
        if (p < 10) {
          f4 accp = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            const f4 wv = *reinterpret_cast<const f4*>(
                &lds[R_W1P + (((mt * 4 + k) * 10 + p) * 16 + j) * 4]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
              accp = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[v], dz1[mt][v], accp, 0, 0, 0);
          }
          xdo[p * 64 + lane] = accp;
        }
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 10; ++p) {
        const f4 v = xdo[p * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) dob[4 * p + r] = v[r];
      }
    }
    reverse_observation(dob, cur.x, cur.dS, j, gx, lH, ls);
    cur = nxt;
  }
  if (!active || w != 0) return;
  const uint32_t ef = opaque((uint32_t)e);
  const uint32_t kf = opaque((uint32_t)(k * N + e));
#pragma unroll
  for (int i = 0; i < NS; ++i)
    if ((i & 3) == k) lam[(size_t)i * N + ef] = ls[i];
#pragma unroll
  for (int s = 0; s < NH; ++s) lam[(size_t)(NS + s * NA) * N + kf] = lH[s];
  if (k == 0)
#pragma unroll
    for (int i = 0; i < NP; ++i) gth_io[(size_t)i * N + ef] = gth[i];
}

// Weight gradients of one segment: for every (step, env) row,
//   dW1 += dz1 o^T, dW2 += dz2 relu(z1)^T, dW3 += dz3 relu(z2)^T, db += dz,
// the rows being the contraction dimension.  Most of the work runs on fp32
// MFMA (v_mfma_f32_16x16x4f32): A[i][k] (lane i + 16 k) = dz of neuron
// 16 n + i at env e0 + k, B[k][j] = input column 16 t + j at the same env;
// result register r of a tile holds neuron 16 n + 4 lg + r, column 16 t + li.
//
// One workgroup of 8 waves per (64-env block, step group).  The input
// columns fall in column tiles of 16: layer 1's 146 columns make the full
// tiles 0..8 and the 2 columns 144, 145; layer 2's 64 columns the tiles
// 10..13.  Waves g and g + 4 run column group g on alternate steps (two
// waves per SIMD, so one's loads overlap the other's matrix work) and add
// their sums through LDS at the end, half 0 first.  A group owns three full
// tiles with their 4 neuron tiles -- {g, g + 4} of layer 1 and 10 + g of
// layer 2 -- and neuron tile g of the shared tile 8, so each group issues the
// same 52 products per 16-env slab and no product multiplies padding.  The
// rest is small: group 0 takes layer 1's last two columns and its bias
// (16-block v_mfma_f32_4x4x1f32, block b = neurons 4 b .. 4 b + 3, one
// product per env: D[i][j] in lane 4 b + j, register i, is neuron 4 b + i,
// column 144 + j, with column 146 the constant one), group 2 layer 3 (the
// same shape with block b = columns 4 b .. 4 b + 3: lane l, register o holds
// output o, column l) and layer 3's bias, every group layer 2's bias of its
// neuron tile (vector adds of the A operands it already holds).  The dz rows
// (A operands, the same for the four groups of a half) are loaded once per
// step by the half's four waves together, whole 256-byte rows per lane
// group, and staged in LDS; each wave loads its own input columns (B
// operands) from the record or the LDS copy of the action tape, one 16-env
// slab ahead.  The history features of o_t are the actions of the 32
// previous steps, read from the segment's action tape (one contiguous span
// per 64-env block).
constexpr int DW_SPLIT = 8;  // the column tile shared by the four groups
constexpr int DW_NB = 4;     // B operands of a slab: three full tiles, the shared one
// accumulators (f4) of a wave: full tile i, neuron tile n at 4 i + n, then
// the shared tile, layer 2's bias, the small products and layer 3's bias
constexpr int DW_A_SHARED = 12, DW_A_B2 = 13, DW_A_SMALL = 14, DW_A_B3 = 15, DW_NACC = 16;
constexpr int DW_COL_SMALL = 16 * (DW_SPLIT + 1);  // first layer-1 column of the small products

// column tile of B slot i of group G
__host__ __device__ constexpr int dw_tile(int G, int i) {
  return i < 2 ? G + 4 * i : i == 2 ? 10 + G : DW_SPLIT;
}
static_assert(dw_tile(3, 1) == 7 && dw_tile(0, 2) == 10 && dw_tile(3, 2) == 13 &&
                  DW_COL_SMALL + 2 == NO,
              "column groups");

// B operands of a slab; group 2's small products take z2 row l of the
// lane for the slab's env quads 0..3 from the record
struct DwOps {
  f4 b[DW_NB];
  f4 z[4];
};
// A operands of a slab and the small products' A (env quads 0..3 of the
// slab), with group 0's small B (its tape columns), all read from LDS
struct DwA {
  f4 a1[4], a2[4];
  f4 sa[4], sb[4];
};

// LDS staging of one step's dz rows for a half: DZ_F rows of 64 envs, pitch
// DW_AP floats (the 4 extra floats put the 16 rows one ds_read_b128 touches
// on distinct banks).  Wave g of the half loads rows DW_AW g .. DW_AW g +
// DW_AW - 1, four rows per instruction.
constexpr int DW_AP = RB + 4, DW_AW = (DZ_F + 3) / 4, DW_AL = (DW_AW + 3) / 4;
constexpr int DW_ABUF = DZ_F * DW_AP;  // floats per half

__device__ inline f4 const4(float v) { return f4{v, v, v, v}; }

// Raw buffer view of a device array (bounds-checked by the hardware against
// `bytes`: out-of-range loads read zero).  Loads take a 32-bit per-lane byte
// offset, a uniform byte offset and a constant, so the per-tile and per-step
// parts of an address stay scalar.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
__device__ inline f4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// Tiles 1..8 hold history columns: tile 1 mixes the last two state features
// with history and is read from the record with a per-lane offset (the
// source step depends on the column); tiles 2..8 hold action-tape values
// only and read an LDS copy of the block's tape window: the DW_CH steps [w0,
// w0 + DW_CH) observe slots w0 .. w0 + DW_CH + NH - 2, which the workgroup
// copies in (rows (slot - w0) * NA + a, pitch DW_AP) and refills every
// DW_CH steps, so each tape value is read from memory once per window
// instead of once for each of the 32 steps that observe it.
constexpr int DW_CH = 16, DW_TW = (DW_CH + NH) * NA, DW_TBUF = DW_TW * DW_AP;
static_assert(DW_CH % 2 == 0, "a window holds whole iterations (one step per half)");
__host__ __device__ constexpr bool dw_tape(int t) { return t >= 2 && t <= DW_SPLIT; }

// Addressing of one step, in bytes from the dz and record buffers: uniform
// offsets of this step's block, the per-lane offset of tile 1 (group 1), and
// in floats from the LDS tape window (w0 its first slot) those of the tape
// tiles and of group 0's small B operands (tape rows of columns 144, 145).
// Group 2's small B operands (relu(z2) row l of the lane) need no per-step
// lane offset.
struct DwAddr {
  uint32_t dzs, rs;
  uint32_t h[DW_NB];
  uint32_t hs;
};

template <int G>
__device__ inline void dw_addr(DwAddr& d, int tl, int n, int chunk, int N, int lane, int w0) {
  const int li = lane & 15, lg = lane >> 4;
  const uint32_t rbp = (uint32_t)rb_pad(N), rstep = (uint32_t)REC_F * rbp;
  d.dzs = 4u * ((uint32_t)tl * (DZ_F * rbp) + (uint32_t)chunk * (DZ_F * RB));
  d.rs = 4u * ((uint32_t)tl * rstep + (uint32_t)chunk * (REC_F * RB));
  const uint32_t c4 = 4 * lg;
  const uint32_t rbo = (uint32_t)tl * rstep + (uint32_t)chunk * (REC_F * RB) + c4;
  // this block's action tape; history slot sl of step tl is tape slot tl + sl
  const uint32_t tape = (uint32_t)n * rstep + (uint32_t)chunk * ((NH + n) * NA * RB) + c4;
#pragma unroll
  for (int i = 0; i < DW_NB; ++i) {
    const int t = dw_tile(G, i), col = 16 * t + li;
    if (dw_tape(t)) {
      // window row of history column hc: (tl + hc / NA - w0) NA + hc % NA
      d.h[i] = (uint32_t)(((tl - w0) * NA + col - 18) * DW_AP + 4 * lg);
    } else if (t == 1) {
      const int hc = col < 18 ? 0 : col - 18;
      const uint32_t o_hist = tape + (uint32_t)((tl + (hc >> 2)) * NA + (hc & 3)) * RB;
      d.h[i] = 4u * (col < 18 ? rbo + (REC_O + col) * RB : o_hist);
    } else {
      d.h[i] = 0;
    }
  }
  // group 0: lane 4 b + j takes column 144 + j (j = 2, 3: constants, any
  // valid row)
  const int j = lane & 3;
  d.hs = G == 0 ? (uint32_t)(((tl - w0) * NA + DW_COL_SMALL - 18 + (j < 2 ? j : 0)) * DW_AP) : 0u;
}

// Issues the record B loads of slab q of a step; dw_prepare finishes the
// operands when they are used, so the loads stay in flight during the
// previous slab's matrix work.  loff: the lane's byte offset 4 (li * RB +
// 4 lg).
template <int G>
__device__ inline void dw_load_slab(DwOps& o, __amdgpu_buffer_rsrc_t rrec, const DwAddr& d,
                                    uint32_t loff, int q) {
  if (G == 2) {
    // z2 row l, envs 16 q + 4 k .. + 3 (64 rows of 16 bytes per load)
    const uint32_t lo = 4u * (uint32_t)((threadIdx.x & 63) * RB);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.z[k] = bld4(rrec, lo + 64 * q + 16 * k, d.rs + 4 * (REC_Z2 * RB));
  }
#pragma unroll
  for (int i = 0; i < DW_NB; ++i) {
    const int t = dw_tile(G, i);
    if (dw_tape(t)) continue;
    if (t == 1) {
      o.b[i] = bld4(rrec, d.h[i] + 64 * q, 0);
    } else {
      const int row = t == 0 ? REC_O : REC_Z1 + 16 * (t - 10);
      o.b[i] = bld4(rrec, loff + 64 * q, d.rs + 4 * (row * RB));
    }
  }
}

// The tape B operands of slab q from the LDS window.
template <int G>
__device__ inline void dw_load_tape(DwOps& o, const float* tw, const DwAddr& d, int q) {
#pragma unroll
  for (int i = 0; i < DW_NB; ++i)
    if (dw_tape(dw_tile(G, i))) o.b[i] = *reinterpret_cast<const f4*>(&tw[d.h[i] + 16 * q]);
}

// Copies tape slots [w0, w0 + DW_CH + NH) of 64-env block `chunk` (those
// below NH + n) into the window tw, every thread of the 512 issuing its six
// 16-byte loads before its first store.
constexpr int DW_TLD = DW_TW * (RB / 4) / 512;
static_assert(DW_TW * (RB / 4) % 512 == 0, "the window splits evenly over the workgroup");
__device__ inline void dw_stage_tape(float* tw, __amdgpu_buffer_rsrc_t rrec, int chunk, int n,
                                     int N, int w0) {
  const uint32_t rbp = (uint32_t)rb_pad(N);
  // the block's tape, in bytes from the record's start
  const uint32_t base =
      4u * ((uint32_t)n * REC_F * rbp + (uint32_t)chunk * (uint32_t)((NH + n) * NA * RB));
  const int rows = min(DW_TW, (NH + n - w0) * NA);
  f4 v[DW_TLD];
#pragma unroll
  for (int j = 0; j < DW_TLD; ++j) {
    const int k = (int)threadIdx.x + 512 * j, r = k >> 4, c = 4 * (k & 15);
    const int rr = r < rows ? r : rows - 1;
    v[j] = bld4(rrec, 4u * (uint32_t)((w0 * NA + rr) * RB + c), base);
  }
#pragma unroll
  for (int j = 0; j < DW_TLD; ++j) {
    const int k = (int)threadIdx.x + 512 * j, r = k >> 4, c = 4 * (k & 15);
    if (r < rows) *reinterpret_cast<f4*>(&tw[r * DW_AP + c]) = v[j];
  }
}

// This wave's share of step tl's dz rows (whole rows: lane l takes envs
// 4 (l & 15) .. + 3 of row DW_AW g + 4 j + (l >> 4)); rows past the share
// load a valid row and are not stored.
__device__ inline void dw_a_load(f4 an[DW_AL], __amdgpu_buffer_rsrc_t rdz, int tl, int chunk,
                                 int N, int g, int lane) {
  const uint32_t rbp = (uint32_t)rb_pad(N);
  const uint32_t so = 4u * ((uint32_t)tl * (DZ_F * rbp) + (uint32_t)chunk * (DZ_F * RB));
#pragma unroll
  for (int j = 0; j < DW_AL; ++j) {
    int r = DW_AW * g + 4 * j + (lane >> 4);
    r = r < DZ_F ? r : DZ_F - 1;
    an[j] = bld4(rdz, 4u * (uint32_t)(r * RB + 4 * (lane & 15)), so);
  }
}
__device__ inline void dw_a_store(const f4 an[DW_AL], float* sA, int g, int lane) {
#pragma unroll
  for (int j = 0; j < DW_AL; ++j) {
    const int jr = 4 * j + (lane >> 4), r = DW_AW * g + jr;
    if (jr < DW_AW && r < DZ_F) *reinterpret_cast<f4*>(&sA[r * DW_AP + 4 * (lane & 15)]) = an[j];
  }
}
// A operands of slab q from the staged rows, and the small products'
// operands of envs 16 q + 4 k .. + 3 held in LDS: group 0 A = dz1 row l, B =
// the tape rows of columns 144 + (l & 3) at window offset hs (lanes with
// l & 3 >= 2 take constants, set by dw_prepare); group 2 A = dz3 row l & 3.
template <int G>
__device__ inline void dw_read_a(DwA& a, const float* sA, const float* tw, uint32_t hs, int q,
                                 int lane) {
  const int li = lane & 15, c = 16 * q + 4 * (lane >> 4);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    a.a1[nt] = *reinterpret_cast<const f4*>(&sA[(16 * nt + li) * DW_AP + c]);
    a.a2[nt] = *reinterpret_cast<const f4*>(&sA[(NHID + 16 * nt + li) * DW_AP + c]);
  }
  if (G == 0 || G == 2) {
    const int row = G == 0 ? lane : 2 * NHID + (lane & 3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a.sa[k] = *reinterpret_cast<const f4*>(&sA[row * DW_AP + 16 * q + 4 * k]);
      if (G == 0) a.sb[k] = *reinterpret_cast<const f4*>(&tw[hs + 16 * q + 4 * k]);
    }
  }
}

// ReLU of the pre-activation columns, the constant columns of group 0's
// small products (one at the bias column 146, zero at 147) and the
// forward's bf16 rounding of its inputs.  Envs >= N of the last block need
// nothing: their dz slots are zero (cleared at allocation; the
// one-env-per-lane sweep writes zeros there) and their record slots are
// zero or finite copies of a batch env's values (the one-env-per-lane
// forward writes those), so they add nothing.
template <int G, bool BF16>
__device__ inline void dw_prepare(DwOps& o, DwA& a, int lane) {
#pragma unroll
  for (int i = 0; i < DW_NB; ++i) {
    const int t = dw_tile(G, i);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float v = t < 10 ? o.b[i][m] : relu_bits(o.b[i][m]);
      if (BF16) v = (float)(__bf16)v;
      o.b[i][m] = v;
    }
  }
  if (G == 0 || G == 2) {
    const int j = lane & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        float v = G == 2 ? relu_bits(o.z[k][m]) : a.sb[k][m];
        if (BF16) v = (float)(__bf16)v;
        if (G == 2)
          o.z[k][m] = v;
        else
          a.sb[k][m] = j < 2 ? v : j == 2 ? 1.0f : 0.0f;
      }
  }
}

// The products of one slab: m walks the four envs a lane group holds
// (16x16x4: K = the four lane groups), k and m the 16 envs one at a time
// (4x4x1: K = one env).
template <int G>
__device__ inline void dw_mfma(f4* acc, float* bs, const DwOps& o, const DwA& A) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int t = dw_tile(G, i);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[4 * i + nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
            t < 10 ? A.a1[nt][m] : A.a2[nt][m], o.b[i][m], acc[4 * i + nt], 0, 0, 0);
    }
    acc[DW_A_SHARED] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a1[G][m], o.b[3][m],
                                                            acc[DW_A_SHARED], 0, 0, 0);
  }
  if (G == 0 || G == 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m)
        acc[DW_A_SMALL] = __builtin_amdgcn_mfma_f32_4x4x1f32(
            A.sa[k][m], G == 2 ? o.z[k][m] : A.sb[k][m], acc[DW_A_SMALL], 0, 0, 0);
  }
  // biases: layer 2's of neuron tile G (bs[0]), layer 3's (group 2, bs[1])
  bs[0] += (A.a2[G][0] + A.a2[G][1]) + (A.a2[G][2] + A.a2[G][3]);
  if (G == 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) bs[1] += (A.sa[k][0] + A.sa[k][1]) + (A.sa[k][2] + A.sa[k][3]);
  }
}

// This half's steps t_lo + half, t_lo + half + 2, ... of the group, the four
// 16-env slabs of a step in turn, each slab's B loads issued one slab ahead
// into the other of two operand buffers (a copy between them would wait for
// the loads in flight), the next step's dz share loaded during this step and
// staged after it.  Both halves run the same number of iterations (every
// wave meets every barrier); a half without a step left reads a valid step
// and skips the products.  sA: this half's staging buffer.
// Barrier discipline: the four column groups run separate instantiations of
// this loop, so their waves reach the workgroup barriers at different
// program locations; the hardware barrier counts arriving waves, and every
// wave executes the same sequence of barriers (one before the loop, two per
// iteration but the last, iters uniform over the workgroup), so they pair up.
// A loop in the kernel body with the group switched per step would keep the
// barriers in uniform code, but it keeps every group's operand slots live
// across the switch and spills.
template <int G, bool BF16>
__device__ inline void dw_accumulate(f4* acc, float* bs, const float* __restrict__ rec,
                                     const float* __restrict__ dz, int N, int chunk, int t_lo,
                                     int t_hi, int n, int half, float* sA, float* tw) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int iters = (t_hi - t_lo + 1) / 2;  // half 0's steps, the same in every wave
  if (iters <= 0) return;
  const uint32_t rbp = (uint32_t)rb_pad(N);
  const __amdgpu_buffer_rsrc_t rrec =
      buf_rsrc(rec, 4u * ((uint32_t)n * REC_F * rbp + (uint32_t)(NH + n) * NA * rbp));
  const __amdgpu_buffer_rsrc_t rdz = buf_rsrc(dz, 4u * ((uint32_t)n * DZ_F * rbp));
  const uint32_t loff = 4u * (uint32_t)(li * RB + 4 * lg);
  auto step = [&](int i) {
    const int t = t_lo + half + 2 * i;
    return t < t_hi ? t : t_hi - 1;
  };
  int w0 = t_lo;  // first slot of the tape window
  dw_stage_tape(tw, rrec, chunk, n, N, w0);
  f4 an[DW_AL];
  dw_a_load(an, rdz, step(0), chunk, N, G, lane);
  dw_a_store(an, sA, G, lane);
  __syncthreads();
  DwOps ob0, ob1;
  DwA A;
  DwAddr d;
  dw_addr<G>(d, step(0), n, chunk, N, lane, w0);
  dw_load_slab<G>(ob0, rrec, d, loff, 0);
  dw_load_tape<G>(ob0, tw, d, 0);
  // scheduling barriers keep each slab's loads ahead of the previous slab's
  // matrix work (left alone, the scheduler interleaves a slab's products
  // with its own loads and the waits then cover the loads just issued)
  for (int i = 0; i < iters; ++i) {
    const bool live = t_lo + half + 2 * i < t_hi;
    const bool more = i + 1 < iters;
    // unconditional (the last iteration reloads its own step): a load under
    // a branch would leave the waits below counting it conservatively
    dw_a_load(an, rdz, step(more ? i + 1 : i), chunk, N, G, lane);
    dw_load_slab<G>(ob1, rrec, d, loff, 1);
    dw_load_tape<G>(ob1, tw, d, 1);
    __builtin_amdgcn_sched_barrier(0);
    dw_read_a<G>(A, sA, tw, d.hs, 0, lane);
    dw_prepare<G, BF16>(ob0, A, lane);
    if (live) dw_mfma<G>(acc, bs, ob0, A);
    __builtin_amdgcn_sched_barrier(0);
    dw_load_slab<G>(ob0, rrec, d, loff, 2);
    dw_load_tape<G>(ob0, tw, d, 2);
    __builtin_amdgcn_sched_barrier(0);
    dw_read_a<G>(A, sA, tw, d.hs, 1, lane);
    dw_prepare<G, BF16>(ob1, A, lane);
    if (live) dw_mfma<G>(acc, bs, ob1, A);
    __builtin_amdgcn_sched_barrier(0);
    dw_load_slab<G>(ob1, rrec, d, loff, 3);
    dw_load_tape<G>(ob1, tw, d, 3);
    __builtin_amdgcn_sched_barrier(0);
    dw_read_a<G>(A, sA, tw, d.hs, 2, lane);
    dw_prepare<G, BF16>(ob0, A, lane);
    if (live) dw_mfma<G>(acc, bs, ob0, A);
    __builtin_amdgcn_sched_barrier(0);
    // slab 3's small-product tape rows are this step's (d moves on below)
    const uint32_t hs = d.hs;
    // the next step's window (refilled below when the next step opens one)
    const bool refill = more && (i + 1) % (DW_CH / 2) == 0;
    const int w0n = refill ? w0 + DW_CH : w0;
    dw_addr<G>(d, step(more ? i + 1 : i), n, chunk, N, lane, w0n);
    dw_load_slab<G>(ob0, rrec, d, loff, 0);
    __builtin_amdgcn_sched_barrier(0);
    dw_read_a<G>(A, sA, tw, hs, 3, lane);
    dw_prepare<G, BF16>(ob1, A, lane);
    if (live) dw_mfma<G>(acc, bs, ob1, A);
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      __syncthreads();  // every wave is done with this step's staged rows
      dw_a_store(an, sA, G, lane);
      if (refill) {
        w0 = w0n;
        dw_stage_tape(tw, rrec, chunk, n, N, w0);
      }
      __syncthreads();
    }
    // after the barrier: the window holds the next step's slots
    dw_load_tape<G>(ob0, tw, d, 0);
  }
}

// The workgroup's 64-env chunks x, x + gx, ... in turn; the barrier before
// each chunk but the first lets every wave finish reading the previous
// chunk's last staged step (its iteration ends without one).
template <int G, bool BF16>
__device__ inline void dw_chunks(f4* acc, float* bs, const float* __restrict__ rec,
                                 const float* __restrict__ dz, int N, int t_lo, int t_hi, int n,
                                 int half, float* sA, float* tw) {
  const int n_chunks = (N + RB - 1) / RB;
  for (int chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    if (chunk != (int)blockIdx.x) __syncthreads();
    dw_accumulate<G, BF16>(acc, bs, rec, dz, N, chunk, t_lo, t_hi, n, half, sA, tw);
  }
}

// A partial slot holds the sums in the accumulators' own register layout:
// [group 4][accumulator DW_NACC][lane 64][register 4] floats, so a wave adds
// its sums with whole-wave vector loads and stores; dw_slot maps a flat
// gradient index to its place in a slot (k_bwd_reduce gathers with it).
// The bias sums are reduced within the wave first: layer 2's bias of neuron
// 16 g + i sits in lane i, register 0 of accumulator DW_A_B2 of group g,
// layer 3's bias of output o in lane o, register 0 of DW_A_B3 of group 2.
constexpr int DW_SLOT = 4 * DW_NACC * 64 * 4;

__host__ __device__ constexpr int dw_pos(int g, int a, int lane, int r) {
  return ((g * DW_NACC + a) * 64 + lane) * 4 + r;
}
// a 16x16 product tile: row rr (neuron within the tile), column c
__host__ __device__ constexpr int dw_tile_pos(int g, int a, int rr, int c) {
  return dw_pos(g, a, c + 16 * (rr / 4), rr % 4);
}

// flat gradient index (torch Linear layout) -> place in a slot
__device__ inline int dw_slot(int idx) {
  if (idx < OFF_B1) {
    const int nrn = idx / NO, col = idx % NO;
    if (col >= DW_COL_SMALL) return dw_pos(0, DW_A_SMALL, 4 * (nrn / 4) + col - DW_COL_SMALL, nrn % 4);
    const int t = col / 16, c = col % 16;
    if (t == DW_SPLIT) return dw_tile_pos(nrn / 16, DW_A_SHARED, nrn % 16, c);
    return dw_tile_pos(t % 4, 4 * (t / 4) + nrn / 16, nrn % 16, c);
  }
  if (idx < OFF_W2) {
    const int nrn = idx - OFF_B1;  // the constant column 146
    return dw_pos(0, DW_A_SMALL, 4 * (nrn / 4) + NO - DW_COL_SMALL, nrn % 4);
  }
  if (idx < OFF_B2) {
    const int nrn = (idx - OFF_W2) / NHID, col = (idx - OFF_W2) % NHID;
    return dw_tile_pos(col / 16, 8 + nrn / 16, nrn % 16, col % 16);
  }
  if (idx < OFF_W3) {
    const int nrn = idx - OFF_B2;
    return dw_pos(nrn / 16, DW_A_B2, nrn % 16, 0);
  }
  if (idx < OFF_B3) {
    const int o = (idx - OFF_W3) / NHID, col = (idx - OFF_W3) % NHID;
    return dw_pos(2, DW_A_SMALL, col, o);
  }
  return dw_pos(2, DW_A_B3, idx - OFF_B3, 0);
}

// grid (gx, S step groups), 512 threads; workgroup x takes the 64-env
// chunks x, x + gx, ... in turn, step group sg the steps [sg * per, min(n,
// (sg + 1) * per)), per = ceil(n / S); it accumulates into its own partial
// slot (x * S + sg) across segments.
template <bool BF16>
__global__ void __launch_bounds__(512)
k_bwd_dw(int N, const float* __restrict__ rec, const float* __restrict__ dz, int n, int S,
         float* __restrict__ gpart) {
  // dz staging of the two halves during the loop, then the exchange of sums
  __shared__ __attribute__((aligned(16))) float smem[2 * DW_ABUF + DW_TBUF];
  float* tw = smem + 2 * DW_ABUF;  // the action-tape window
  static_assert(2 * DW_ABUF * 4 >= 4 * DW_NACC * 64 * 16, "exchange fits the staging space");
  f4(*xacc)[DW_NACC][64] = reinterpret_cast<f4(*)[DW_NACC][64]>(smem);
  const int sg = blockIdx.y;
  // the wave index is uniform across the wave: keep it (and every offset
  // derived from it) in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wv & 3, half = wv >> 2;
  const int per = (n + S - 1) / S;
  const int t_lo = sg * per, t_hi = (t_lo + per) < n ? (t_lo + per) : n;
  // the bias sums accumulate in bs (layer 2's, layer 3's) and enter their
  // slots DW_A_B2 and DW_A_B3 after the loop
  f4 acc[DW_NACC];
  float bs[2] = {0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < DW_NACC; ++i) acc[i] = const4(0.0f);
  float* sA = smem + half * DW_ABUF;
  // one loop over the workgroup's chunks inside each group's instantiation
  // (a loop around the switch would keep every group's operand slots live
  // and spill)
  switch (g) {
    case 0: dw_chunks<0, BF16>(acc, bs, rec, dz, N, t_lo, t_hi, n, half, sA, tw); break;
    case 1: dw_chunks<1, BF16>(acc, bs, rec, dz, N, t_lo, t_hi, n, half, sA, tw); break;
    case 2: dw_chunks<2, BF16>(acc, bs, rec, dz, N, t_lo, t_hi, n, half, sA, tw); break;
    default: dw_chunks<3, BF16>(acc, bs, rec, dz, N, t_lo, t_hi, n, half, sA, tw); break;
  }
  acc[DW_A_B2] = f4{bs[0], 0.0f, 0.0f, 0.0f};
  acc[DW_A_B3] = f4{bs[1], 0.0f, 0.0f, 0.0f};
  __syncthreads();  // the staging space becomes the exchange buffer
  // half 1 hands its sums to half 0 (fixed order: half 0 + half 1)
  if (half == 1)
#pragma unroll
    for (int i = 0; i < DW_NACC; ++i) xacc[g][i][lane] = acc[i];
  __syncthreads();
  if (half == 1) return;
#pragma unroll
  for (int i = 0; i < DW_NACC; ++i) {
    const f4 o = xacc[g][i][lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[i][r] += o[r];
  }
  // layer 2's bias sums over the four lane groups (lanes i, i ^ 32, then
  // i ^ 16); every lane of layer 3's output o already holds the whole sum
  {
    float s = acc[DW_A_B2][0];
    s += __shfl_xor(s, 32);
    s += __shfl_xor(s, 16);
    acc[DW_A_B2][0] = s;
  }
  // add into this group's part of the slot: all loads, then all stores
  f4* gp = reinterpret_cast<f4*>(gpart + ((size_t)blockIdx.x * S + sg) * DW_SLOT) + g * DW_NACC * 64;
  f4 old[DW_NACC];
#pragma unroll
  for (int i = 0; i < DW_NACC; ++i) old[i] = gp[i * 64 + lane];
#pragma unroll
  for (int i = 0; i < DW_NACC; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) old[i][r] += acc[i][r];
    gp[i * 64 + lane] = old[i];
  }
}

// grad[i] = sum over the G partial slots of slot g's entry for i, in a fixed
// order:
// DR_SPLIT threads per output each add a contiguous range of slots in
// ascending order, then the range sums are added in ascending range order.
constexpr int DR_OUT = 32, DR_SPLIT = 8;
__global__ void __launch_bounds__(DR_OUT * DR_SPLIT)
k_bwd_reduce(const float* __restrict__ gpart, int G, float* __restrict__ out) {
  __shared__ float part[DR_SPLIT][DR_OUT];
  const int tx = threadIdx.x % DR_OUT, ty = threadIdx.x / DR_OUT;
  const int i = blockIdx.x * DR_OUT + tx;
  const int per = (G + DR_SPLIT - 1) / DR_SPLIT;
  const int g0 = ty * per, g1 = (g0 + per) < G ? (g0 + per) : G;
  float s = 0.0f;
  if (i < NW) {
    const int pl = dw_slot(i);
#pragma unroll 8
    for (int gg = g0; gg < g1; ++gg) s += gpart[(size_t)gg * DW_SLOT + pl];
  }
  part[ty][tx] = s;
  __syncthreads();
  if (ty != 0 || i >= NW) return;
  float t = part[0][tx];
#pragma unroll
  for (int r = 1; r < DR_SPLIT; ++r) t += part[r][tx];
  out[i] = t;
}

__global__ void k_copy(const float* __restrict__ src, float* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------

hipError_t bwd_alloc(BwdBufs& bw, int N, int K, int H) {
  bw.N = N;
  bw.K = K;
  bw.H = H;
  // Weight-gradient pass: one workgroup per CU (the double-buffered staging
  // takes most of the LDS), so about n_cu workgroups: up to n_cu 64-env
  // chunks, each split into step groups to fill the CUs; beyond n_cu chunks,
  // n_cu workgroups that each take every n_cu-th chunk in turn (one partial
  // slot per workgroup, whose sums stay in registers across its chunks).
  const int chunks = (int)nb(N, 64);
  int n_cu = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  int S = n_cu / chunks;
  if (S > K / 2) S = K / 2;  // at least two steps per group: one per half
  if (S < 1) S = 1;
  bw.dw_gx = chunks < n_cu ? chunks : n_cu;
  bw.dw_groups = S;
  bw.n_parts = bw.dw_gx * S;
  hipError_t e;
  // a horizon of J segments uses min(J, BWD_NBUF) of the rotating buffers
  const int nseg = (H + K - 1) / K < BWD_NBUF ? (H + K - 1) / K : BWD_NBUF;
  for (int i = 0; i < BWD_NBUF; ++i) {
    if ((e = hipEventCreateWithFlags(&bw.e_rec[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&bw.e_rev[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&bw.e_dw[i], hipEventDisableTiming)) != hipSuccess) return e;
    if (i >= nseg) continue;
    // zeroed once: the quarter-lane and split kernels never write the slots
    // of envs >= N in the last 64-env block, which must then read as finite
    // (record) and zero (cotangents) in the weight-gradient pass
    if ((e = hipMalloc(&bw.seg[i], rec_floats(K, N) * 4)) != hipSuccess) return e;
    if ((e = hipMemset(bw.seg[i], 0, rec_floats(K, N) * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&bw.dz[i], (size_t)K * DZ_F * rb_pad(N) * 4)) != hipSuccess) return e;
    if ((e = hipMemset(bw.dz[i], 0, (size_t)K * DZ_F * rb_pad(N) * 4)) != hipSuccess) return e;
  }
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&bw.n_cu, hipDeviceAttributeMultiprocessorCount, dev)) !=
      hipSuccess)
    return e;
  if ((e = hipEventCreateWithFlags(&bw.e_init, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipStreamCreateWithFlags(&bw.s_rec, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipStreamCreateWithFlags(&bw.s_dw, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.lam, (size_t)LAM_F * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gth, (size_t)NP * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gpart, (size_t)bw.n_parts * DW_SLOT * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gsum, (size_t)NW * 4)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_bwd_reverse<false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, R_TOTAL * 4)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_bwd_reverse<true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (R_TOTAL + R_XCH) * 4)) !=
      hipSuccess)
    return e;
  return reverse1_prepare();
}

void bwd_free(BwdBufs& bw) {
  for (int i = 0; i < BWD_NBUF; ++i) {
    if (bw.seg[i]) (void)hipFree(bw.seg[i]);
    if (bw.dz[i]) (void)hipFree(bw.dz[i]);
    if (bw.e_rec[i]) (void)hipEventDestroy(bw.e_rec[i]);
    if (bw.e_rev[i]) (void)hipEventDestroy(bw.e_rev[i]);
    if (bw.e_dw[i]) (void)hipEventDestroy(bw.e_dw[i]);
  }
  if (bw.e_init) (void)hipEventDestroy(bw.e_init);
  if (bw.s_rec) (void)hipStreamDestroy(bw.s_rec);
  if (bw.s_dw) (void)hipStreamDestroy(bw.s_dw);
  void* ptrs[] = {bw.lam, bw.gth, bw.gpart, bw.gsum};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  bw = BwdBufs{};
}

#define BWD_TRY(x)                 \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Segments run last to first.  Per segment j (buffer j mod 3):
//   recompute stream: waits for the weight-gradient pass that last used the
//     buffer, then records the segment;
//   caller stream: waits for the record, runs the reverse sweep (the
//     segment-to-segment adjoint carry keeps these in order);
//   weight-gradient stream: waits for the sweep, reduces the segment.
// So the recompute of the next segments and the weight gradients of the
// previous ones overlap the sweep.  The caller's stream finally waits for
// the last weight-gradient pass before the fixed-order partial sum.
// Overlap only pays while the sweep leaves compute units idle (fewer
// workgroups than CUs); for large batches the sweep (one wave per SIMD, most
// registers) fills the chip and everything stays on the caller's stream in
// order.
// nbuf: segment buffers to rotate (BWD_NBUF, or 1 for the serial order of
// the scratch-array variant, which also keeps every kernel on st).
static hipError_t backward_segments(const DevCfg& c, const SimBufs& b, const BwdBufs& bw, int nbuf,
                                    const float* W, const float* tape, int K, int T,
                                    const float* d_rewards, const float* d_states,
                                    float* grad_actor, float* grad_params, int* held,
                                    hipStream_t st) {
  const int N = c.n_envs;
  const size_t np = (size_t)bw.n_parts * DW_SLOT;
  hipLaunchKernelGGL(k_fill, dim3(nb((int)np, 256)), dim3(256), 0, st, bw.gpart, np, 0.0f);
  hipLaunchKernelGGL(k_bwd_init, dim3(nb(N, 256)), dim3(256), 0, st, N,
                     d_states ? d_states + (size_t)T * NS * N : nullptr, bw.lam, bw.gth);
  const bool overlap = nbuf == BWD_NBUF && (int)nb(N, 64) < bw.n_cu;
  hipStream_t s_rec = overlap ? bw.s_rec : st, s_dw = overlap ? bw.s_dw : st;
  if (overlap) {
    BWD_TRY(hipEventRecord(bw.e_init, st));
    BWD_TRY(hipStreamWaitEvent(s_rec, bw.e_init, 0));
    BWD_TRY(hipStreamWaitEvent(s_dw, bw.e_init, 0));
  }
  const int J = (T + K - 1) / K;
  int last = 0;
  for (int j = J - 1, idx = 0; j >= 0; --j, ++idx) {
    const int t0 = j * K;
    const int n = (T - t0) < K ? (T - t0) : K;
    const int buf = idx % nbuf;
    // the record may be in the buffer already: written by the taped rollout
    // (on the caller's stream, ahead of this call) or by a recompute of an
    // earlier backward on the same tape
    if (held && held[buf] == j) {
      // nothing to recompute
    } else {
      if (held) held[buf] = j;
      if (overlap && idx >= BWD_NBUF) BWD_TRY(hipStreamWaitEvent(s_rec, bw.e_dw[buf], 0));
      BWD_TRY(launch_recompute(c, b, W, n, tape + (size_t)j * CK_F * N, bw.seg[buf], s_rec));
      if (overlap) {
        BWD_TRY(hipEventRecord(bw.e_rec[buf], s_rec));
        BWD_TRY(hipStreamWaitEvent(st, bw.e_rec[buf], 0));
      }
    }
    if (taped_kernel(c) == TAPED_LANE)
      BWD_TRY(launch_reverse1(c, b.theta, W, tape + (size_t)j * CK_F * N, bw.seg[buf], n, t0,
                              d_rewards, d_states, bw.lam, bw.gth, bw.dz[buf], st));
    else if (N <= REVERSE_SPLIT_MAX_ENVS)
      hipLaunchKernelGGL(k_bwd_reverse<true>, dim3(nb(N, 16)), dim3(256), (R_TOTAL + R_XCH) * 4,
                         st, c, b.theta, W, tape + (size_t)j * CK_F * N, bw.seg[buf], n, t0,
                         d_rewards, d_states, bw.lam, bw.gth, bw.dz[buf]);
    else
      hipLaunchKernelGGL(k_bwd_reverse<false>, dim3(nb(N, 64)), dim3(256), R_TOTAL * 4, st, c,
                         b.theta, W, tape + (size_t)j * CK_F * N, bw.seg[buf], n, t0, d_rewards,
                         d_states, bw.lam, bw.gth, bw.dz[buf]);
    BWD_TRY(hipGetLastError());
    if (overlap) {
      BWD_TRY(hipEventRecord(bw.e_rev[buf], st));
      BWD_TRY(hipStreamWaitEvent(s_dw, bw.e_rev[buf], 0));
    }
    hipLaunchKernelGGL((c.flags & F_ACTOR_BF16) ? k_bwd_dw<true> : k_bwd_dw<false>,
                       dim3(bw.dw_gx, bw.dw_groups), dim3(512), 0, s_dw, N, bw.seg[buf],
                       bw.dz[buf], n, bw.dw_groups, bw.gpart);
    BWD_TRY(hipGetLastError());
    if (overlap) BWD_TRY(hipEventRecord(bw.e_dw[buf], s_dw));
    last = buf;
  }
  if (overlap) BWD_TRY(hipStreamWaitEvent(st, bw.e_dw[last], 0));
  hipLaunchKernelGGL(k_bwd_reduce, dim3(nb(NW, DR_OUT)), dim3(DR_OUT * DR_SPLIT), 0, st, bw.gpart,
                     bw.n_parts,
                     grad_actor ? grad_actor : bw.gsum);
  if (grad_params)
    hipLaunchKernelGGL(k_copy, dim3(nb(NP * N, 256)), dim3(256), 0, st, bw.gth, grad_params,
                       (size_t)NP * N);
  return hipGetLastError();
}

hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        int held[BWD_NBUF], hipStream_t st) {
  return backward_segments(c, b, bw, BWD_NBUF, W, tape, K, T, d_rewards, d_states, grad_actor,
                           grad_params, held, st);
}

// Layout of the scratch array in floats, every part starting on a 256-byte
// boundary: one segment record, its layer cotangents, the adjoint carry,
// the parameter gradients, the weight-gradient partials, the actor-gradient
// sink.
static inline size_t up64(size_t f) { return (f + 63) & ~(size_t)63; }

size_t bwd_scratch_floats(const BwdBufs& bw) {
  const int N = bw.N, K = bw.K;
  return up64(rec_floats(K, N)) + up64((size_t)K * DZ_F * rb_pad(N)) + up64((size_t)LAM_F * N) +
         up64((size_t)NP * N) + up64((size_t)bw.n_parts * DW_SLOT) + up64((size_t)NW);
}

hipError_t run_backward_in(const DevCfg& c, const SimBufs& b, const BwdBufs& bw, float* scratch,
                           const float* W, const float* tape, int K, int T,
                           const float* d_rewards, const float* d_states, float* grad_actor,
                           float* grad_params, hipStream_t st) {
  const int N = c.n_envs;
  BwdBufs sb = bw;  // shape, groups and device attributes of the handle's backward
  for (int i = 0; i < BWD_NBUF; ++i) sb.seg[i] = sb.dz[i] = nullptr;
  float* p = scratch;
  const size_t f_rec = rec_floats(K, N), f_dz = (size_t)K * DZ_F * rb_pad(N);
  sb.seg[0] = p;
  p += up64(f_rec);
  sb.dz[0] = p;
  p += up64(f_dz);
  sb.lam = p;
  p += up64((size_t)LAM_F * N);
  sb.gth = p;
  p += up64((size_t)NP * N);
  sb.gpart = p;
  p += up64((size_t)bw.n_parts * DW_SLOT);
  sb.gsum = p;
  // the array keeps whatever the last call on this device left in it; the
  // record and cotangent slots of envs >= N in the last 64-env block may go
  // unwritten here and must read as finite and zero
  // (k_fill: one float per thread; both sizes are below 2^31 by the
  // scratch bound the caller checked)
  hipLaunchKernelGGL(k_fill, dim3(nb((int)f_rec, 256)), dim3(256), 0, st, sb.seg[0], f_rec, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(nb((int)f_dz, 256)), dim3(256), 0, st, sb.dz[0], f_dz, 0.0f);
  BWD_TRY(hipGetLastError());
  return backward_segments(c, b, sb, 1, W, tape, K, T, d_rewards, d_states, grad_actor,
                           grad_params, nullptr, st);
}

}  // namespace qs
