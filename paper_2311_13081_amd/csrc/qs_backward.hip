// Discrete adjoint of a taped rollout.
//
// The taped forward stored checkpoints (state, history) every K steps.  The
// backward walks the segments last to first; per segment:
//   1. recompute: the fused MFMA kernel restarts from the checkpoint and
//      records x_t, a_t, the layer pre-activations z1, z2 and o_t per step;
//   2. reverse sweep (k_bwd_reverse): four lanes per env, the adjoints of
//      the state and of the action history in registers, stepping back
//      through reward, quaternion renormalisation, the four RK4 stages, the
//      action map, the actor (on MFMA) and the history shift; per-env
//      parameter gradients accumulate in registers; the layer cotangents
//      dz1, dz2, dz3 of every (step, env) go to scratch;
//   3. weight gradients (k_bwd_dw): sum over (step, env) rows of dz (x) input
//      on fp32 MFMA, one workgroup per 64-env chunk accumulating into its own
//      partial; biases come from a constant-one input column.
// Finally k_bwd_reduce adds the workgroup partials in ascending order, so
// the result does not depend on scheduling.
#include "qs_actor.h"
#include "qs_backward.h"
#include "qs_forward.h"

namespace qs {

constexpr int DZ_F = NHID + NHID + NA;  // dz1 | dz2 | dz3 per (step, env)
constexpr int LAM_F = NS + NH * NA;     // state and history adjoints

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

// Quarter-lane reverse sweep (16 envs per wave, lane L = j + 16 k: env j,
// quarter k), the adjoint of the quarter-lane forward kernel.  Per lane:
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

// Weight as the forward used it: rounded to bf16 under the bf16-actor flag.
__device__ inline float fwd_weight(float w, bool bf16) { return bf16 ? (float)(__bf16)w : w; }

__device__ inline void stage_reverse(const float* __restrict__ W, float* lds, bool bf16) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < NA * NHID; i += nt) lds[R_W3 + i] = fwd_weight(W[OFF_W3 + i], bf16);
  for (int idx = tid; idx < NHID * NHID; idx += nt) {
    const int v = idx & 3, i = (idx >> 2) & 15, m = (idx >> 6) & 3, g = (idx >> 8) & 3,
              n = idx >> 10;
    lds[R_W2P + idx] = fwd_weight(W[OFF_W2 + (16 * n + 4 * g + v) * NHID + 16 * m + i], bf16);
  }
  for (int idx = tid; idx < 10 * 16 * NHID; idx += nt) {
    const int v = idx & 3, i = (idx >> 2) & 15, rest = idx >> 6;  // rest = (m*4 + g)*10 + p
    const int p = rest % 10, g = (rest / 10) & 3, m = rest / 40;
    const int feat = r_phi(4 * p + (i & 3), i >> 2);
    lds[R_W1P + idx] =
        feat >= 0 ? fwd_weight(W[OFF_W1 + (16 * m + 4 * g + v) * NO + feat], bf16) : 0.0f;
  }
}

// Inputs of one reverse step: the recorded state and action, this lane's
// 16 layer-1 and layer-2 pre-activations (rows 16 q + 4 k + r), the reward
// and state cotangents.
struct StepIn {
  float x[NS], a[NA], z1[16], z2[16], dS[NS], dR;
};

__device__ inline void load_step(StepIn& in, const DevCfg& c, const float* __restrict__ rec,
                                 const float* __restrict__ d_rewards,
                                 const float* __restrict__ d_states, int tl, int t0, int N, int e,
                                 int k) {
  const uint32_t eo = opaque((uint32_t)e);
  const uint32_t roff = opaque((uint32_t)rb_at(e, REC_F));
  const uint32_t zoff = opaque((uint32_t)(rb_at(e, REC_F) + 4 * k * RB));
  const int t = t0 + tl;
  const float* rt = rec + (size_t)tl * REC_F * rb_pad(N);
#pragma unroll
  for (int i = 0; i < NS; ++i) in.x[i] = rt[(size_t)(REC_X + i) * RB + roff];
#pragma unroll
  for (int i = 0; i < NA; ++i) in.a[i] = rt[(size_t)(REC_A + i) * RB + roff];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      in.z1[4 * q + r] = rt[(size_t)(REC_Z1 + 16 * q + r) * RB + zoff];
      in.z2[4 * q + r] = rt[(size_t)(REC_Z2 + 16 * q + r) * RB + zoff];
    }
  in.dR = d_rewards ? d_rewards[(size_t)t * N + eo] : 1.0f;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    in.dS[i] = d_states ? d_states[((size_t)t * NS + i) * N + eo] : 0.0f;
}

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
  const int env0 = (blockIdx.x * blockDim.x + threadIdx.x - lane) / 4;
  if (env0 >= N) return;
  const int env = env0 + j;
  const bool active = env < N;
  const int e = active ? env : env0;

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
  const float h = c.dt;

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
  load_step(cur, c, rec, d_rewards, d_states, n - 1, t0, N, e, k);
  for (int tl = n - 1; tl >= 0; --tl) {
    __asm__ volatile("" ::: "memory");
    load_step(nxt, c, rec, d_rewards, d_states, tl > 0 ? tl - 1 : 0, t0, N, e, k);
    // blocked cotangent rows of this env: row k and row 4k
    const uint32_t koff = opaque((uint32_t)(rb_at(e, DZ_F) + k * RB));
    const uint32_t zoff = opaque((uint32_t)(rb_at(e, DZ_F) + 4 * k * RB));
    float* dzt = dz + (size_t)tl * DZ_F * rb_pad(N);
    float x[NS], a[NA], u[NA];
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = cur.x[i];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      a[i] = cur.a[i];
      u[i] = action_to_rpm(c, a[i]);
    }
    const float dR = cur.dR;

    // --- forward recompute of the RK4 stages -------------------------------
    float x2[NS], x3[NS], x4[NS], kd[NS], acc[NS];
    deriv<float>(B, c.arm, c.km, c.g, x, u, kd);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] = kd[i];
      x2[i] = x[i] + 0.5f * h * kd[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x2, u, kd);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] += 2.0f * kd[i];
      x3[i] = x[i] + 0.5f * h * kd[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x3, u, kd);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] += 2.0f * kd[i];
      x4[i] = x[i] + h * kd[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x4, u, kd);
    float sn[NS];  // post-step state (renormalised)
#pragma unroll
    for (int i = 0; i < NS; ++i) sn[i] = x[i] + (h / 6.0f) * (acc[i] + kd[i]);
    float rn = 1.0f;
    if (renorm) {
      // the forward's reciprocal square root (rk4_step)
      rn = rsqrt_r(sn[3] * sn[3] + sn[4] * sn[4] + sn[5] * sn[5] + sn[6] * sn[6]);
#pragma unroll
      for (int i = 0; i < 4; ++i) sn[3 + i] *= rn;
    }

    // --- reward and history coupling -----------------------------------------
    float g[NS], ga[NA];
#pragma unroll
    for (int i = 0; i < NS; ++i) g[i] = ls[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[i] += -2.0f * c.C_rp * sn[i] * dR;
      g[7 + i] += -2.0f * c.C_rv * sn[7 + i] * dR;
      g[10 + i] += -2.0f * c.C_rw * sn[10 + i] * dR;
    }
    g[3] += 2.0f * c.C_rq * sn[3] * dR;
    // newest history slot: component i lives in quarter i of the same env
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const float hn = __int_as_float(
          __builtin_amdgcn_ds_bpermute((j + 16 * i) << 2, __float_as_int(lH[NH - 1])));
      ga[i] = -2.0f * c.C_ra * (a[i] - c.C_rab) * dR + hn;
    }

    // --- renormalisation ------------------------------------------------------
    if (renorm) {
      const float d = sn[3] * g[3] + sn[4] * g[4] + sn[5] * g[5] + sn[6] * g[6];
#pragma unroll
      for (int i = 0; i < 4; ++i) g[3 + i] = (g[3 + i] - sn[3 + i] * d) * rn;
    }

    // --- RK4 stages in reverse ----------------------------------------------
    float gx[NS], gk[NS], gs[NS], gu[NA] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      gx[i] = g[i];
      gk[i] = (h / 6.0f) * g[i];
      gs[i] = 0.0f;
    }
    deriv_vjp(B, th, c.arm, c.km, x4, u, gk, gs, gu, gth);  // k4 = f(x4)
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      gx[i] += gs[i];
      gk[i] = (h / 3.0f) * g[i] + h * gs[i];
      gs[i] = 0.0f;
    }
    deriv_vjp(B, th, c.arm, c.km, x3, u, gk, gs, gu, gth);  // k3 = f(x3)
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      gx[i] += gs[i];
      gk[i] = (h / 3.0f) * g[i] + 0.5f * h * gs[i];
      gs[i] = 0.0f;
    }
    deriv_vjp(B, th, c.arm, c.km, x2, u, gk, gs, gu, gth);  // k2 = f(x2)
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      gx[i] += gs[i];
      gk[i] = (h / 6.0f) * g[i] + 0.5f * h * gs[i];
    }
    deriv_vjp(B, th, c.arm, c.km, x, u, gk, gx, gu, gth);   // k1 = f(x)
#pragma unroll
    for (int i = 0; i < NA; ++i) ga[i] += gu[i] * c.rpm_half_range;

    // --- actor VJP on matrix cores --------------------------------------------
    float d3[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) d3[i] = ga[i] * (1.0f - a[i] * a[i]);
    const float d3k = k == 0 ? d3[0] : k == 1 ? d3[1] : k == 2 ? d3[2] : d3[3];
    if (active) dzt[(size_t)(2 * NHID) * RB + koff] = d3k;
    // dz2 = (W3^T dz3) * [z2 > 0]: tile q rows 16q + 4k + r, env j
    f4 dz2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dz2[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(lds[R_W3 + k * NHID + 16 * q + j], d3k,
                                                    f4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z2 = cur.z2[4 * q + r];
        dz2[q][r] = z2 > 0.0f ? dz2[q][r] : 0.0f;
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
        const f4 w = *reinterpret_cast<const f4*>(
            &lds[R_W2P + (((q * 4 + k) * 4 + mt) * 16 + j) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          accm = __builtin_amdgcn_mfma_f32_16x16x4f32(w[v], dz2[q][v], accm, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z1 = cur.z1[4 * mt + r];
        dz1[mt][r] = z1 > 0.0f ? accm[r] : 0.0f;
        if (active) dzt[(size_t)(16 * mt + r) * RB + zoff] = dz1[mt][r];
      }
    }
    // do = W1^T dz1 in observation order: tile p, register r of quarter k is
    // the cotangent of feature PHI(4p + r, k)
    float dob[40];
#pragma unroll
    for (int p = 0; p < 10; ++p) {
      f4 accp = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const f4 w = *reinterpret_cast<const f4*>(
            &lds[R_W1P + (((mt * 4 + k) * 10 + p) * 16 + j) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          accp = __builtin_amdgcn_mfma_f32_16x16x4f32(w[v], dz1[mt][v], accp, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) dob[4 * p + r] = accp[r];
    }
    // history adjoint: H_t[s] feeds H_{t+1}[s-1]; descending s reads the
    // older adjoint before it is overwritten
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
    for (int i = 0; i < NS; ++i)
      ls[i] = gx[i] + cur.dS[i];
    cur = nxt;
  }
  if (!active) return;
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
// on fp32 MFMA (v_mfma_f32_16x16x4f32) with the rows as the K dimension:
// A[i][k] (lane i + 16 k) = dz of neuron 16 w + i at env e0 + k, B[k][j] =
// input column j of a 16-column tile at the same env; the result register r
// of a tile holds row 4 lg + r, column li.  Biases come from a constant-one
// input column (generated, not stored).
//
// One workgroup per (64-env block, step group), one wave per 16-neuron tile
// w.  The layer inputs of a step (o, relu(z1), relu(z2): 274 rows x 64 envs,
// read once from HBM as whole 256-byte block rows) are staged in LDS and
// shared by the four waves; the staging of step t + 1 is issued into
// registers before step t's matrix work and written to the other LDS buffer
// after it, so the loads' latency hides behind the MFMAs.  Each wave reads its
// own dz rows straight from the record, also one step ahead.  Layer 3 (4
// outputs) is split by column tiles: wave w takes tile w, wave 0 also tile 4
// (the bias column).  Each (block, step group) owns one partial slot,
// accumulated across segments.
constexpr int DW_ROWS = NO + 2 * NHID;  // staged input rows per step: o | z1 | z2
constexpr int DW_P = 68;                // LDS row pitch in floats (64 envs + 4)
constexpr int DW_BUF = DW_ROWS * DW_P;  // floats per staging buffer
constexpr int DW_LD = (DW_ROWS * 16 + 255) / 256;  // float4 staging loads per thread

// Four consecutive envs e..e+3 of one blocked row (p points at env e);
// envs >= N read as zero.
__device__ inline f4 dw_load(const float* __restrict__ p, int e, int N) {
  if (e + 4 <= N) return *reinterpret_cast<const f4*>(p);
  f4 v;
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = e + m < N ? p[m] : 0.0f;
  return v;
}

struct DwStage {
  f4 v[DW_LD];
};

// Issues the staging loads of one step (input row r, envs 4 c4 .. 4 c4 + 3
// for slot i of thread tid: r = tid / 16 + 16 i, c4 = tid % 16).
__device__ inline void dw_stage_load(DwStage& sg, const float* __restrict__ rt, int env0, int N,
                                     int tid) {
  const int c = (tid & 15) * 4;
#pragma unroll
  for (int i = 0; i < DW_LD; ++i) {
    const int r = (tid >> 4) + 16 * i;
    const int f = r < NO ? REC_O + r : REC_Z1 + (r - NO);  // z1 and z2 rows are adjacent
    sg.v[i] = r < DW_ROWS ? dw_load(rt + (size_t)f * RB + c, env0 + c, N)
                          : f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
}

// Writes staged rows to an LDS buffer: ReLU on the z rows, bf16 rounding of
// every input when the forward rounded it.
__device__ inline void dw_stage_store(const DwStage& sg, float* buf, int tid, int bf16) {
  const int c = (tid & 15) * 4;
#pragma unroll
  for (int i = 0; i < DW_LD; ++i) {
    const int r = (tid >> 4) + 16 * i;
    if (r < DW_ROWS) {
      f4 v = sg.v[i];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (r >= NO) v[m] = fmaxf(v[m], 0.0f);
        if (bf16) v[m] = (float)(__bf16)v[m];
      }
      *reinterpret_cast<f4*>(&buf[r * DW_P + c]) = v;
    }
  }
}

struct DwA {
  f4 a1[4], a2[4], a3[4];
};

__device__ inline void dw_a_load(DwA& A, const float* __restrict__ dzt, int env0, int N, int w,
                                 int li, int lg) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = 16 * q + 4 * lg;
    A.a1[q] = dw_load(dzt + (size_t)(16 * w + li) * RB + col, env0 + col, N);
    A.a2[q] = dw_load(dzt + (size_t)(NHID + 16 * w + li) * RB + col, env0 + col, N);
    A.a3[q] = li < NA ? dw_load(dzt + (size_t)(2 * NHID + li) * RB + col, env0 + col, N)
                      : f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
}

// B operand: input column `row` of a layer with n_in inputs whose staged
// rows start at LDS row `base`: the staged value, the bias column of ones
// (valid envs) at row == n_in, zeros beyond.
__device__ inline f4 dw_b(const float* buf, int base, int row, int n_in, int col, int env0,
                          int N) {
  if (row < n_in) return *reinterpret_cast<const f4*>(&buf[(base + row) * DW_P + col]);
  f4 v;
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = (row == n_in && env0 + col + m < N) ? 1.0f : 0.0f;
  return v;
}

__global__ void __launch_bounds__(256)
k_bwd_dw(int N, const float* __restrict__ rec, const float* __restrict__ dz, int n, int S,
         float* __restrict__ gpart, int bf16) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int chunk = blockIdx.x, w = tid >> 6, sg = blockIdx.y;
  const int env0 = chunk * RB;
  const int per = (n + S - 1) / S;
  const int t_begin = sg * per, t_end = (t_begin + per) < n ? (t_begin + per) : n;
  const size_t rstep = (size_t)REC_F * rb_pad(N), dstep = (size_t)DZ_F * rb_pad(N);
  const float* rblk = rec + (size_t)chunk * REC_F * RB;
  const float* dblk = dz + (size_t)chunk * DZ_F * RB;

  f4 acc1[10], acc2[5], acc3[2];
#pragma unroll
  for (int i = 0; i < 10; ++i) acc1[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < 5; ++i) acc2[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  acc3[0] = acc3[1] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  if (t_begin < t_end) {
    DwStage st;
    DwA A, An;
    dw_stage_load(st, rblk + (size_t)t_begin * rstep, env0, N, tid);
    dw_a_load(A, dblk + (size_t)t_begin * dstep, env0, N, w, li, lg);
    dw_stage_store(st, sm, tid, bf16);
    __syncthreads();
    for (int tl = t_begin; tl < t_end; ++tl) {
      const int cur = (tl - t_begin) & 1;
      const float* buf = sm + cur * DW_BUF;
      const bool more = tl + 1 < t_end;
      if (more) {  // next step's loads in flight during this step's MFMAs
        dw_stage_load(st, rblk + (size_t)(tl + 1) * rstep, env0, N, tid);
        dw_a_load(An, dblk + (size_t)(tl + 1) * dstep, env0, N, w, li, lg);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = 16 * q + 4 * lg;
        // independent accumulators innermost, so consecutive MFMAs never
        // wait on each other's results
        f4 bo[10], bh[5];
#pragma unroll
        for (int kt = 0; kt < 10; ++kt) bo[kt] = dw_b(buf, 0, 16 * kt + li, NO, col, env0, N);
#pragma unroll
        for (int kt = 0; kt < 5; ++kt) bh[kt] = dw_b(buf, NO, 16 * kt + li, NHID, col, env0, N);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
          for (int kt = 0; kt < 10; ++kt)
            acc1[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a1[q][m], bo[kt][m], acc1[kt], 0, 0, 0);
#pragma unroll
          for (int kt = 0; kt < 5; ++kt)
            acc2[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a2[q][m], bh[kt][m], acc2[kt], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (j == 1 && w != 0) break;
          const int kt = j == 0 ? w : 4;
          const f4 bh = dw_b(buf, NO + NHID, 16 * kt + li, NHID, col, env0, N);
#pragma unroll
          for (int m = 0; m < 4; ++m)
            acc3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a3[q][m], bh[m], acc3[j], 0, 0, 0);
        }
      }
      if (more) {
        dw_stage_store(st, sm + (cur ^ 1) * DW_BUF, tid, bf16);
        A = An;
      }
      __syncthreads();  // next buffer complete; this buffer free for reuse
    }
  }
  float* gp = gpart + ((size_t)chunk * S + sg) * NW;
#pragma unroll
  for (int kt = 0; kt < 10; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nrn = 16 * w + 4 * lg + r, col = 16 * kt + li;
      if (col < NO) gp[OFF_W1 + nrn * NO + col] += acc1[kt][r];
      else if (col == NO) gp[OFF_B1 + nrn] += acc1[kt][r];
    }
#pragma unroll
  for (int kt = 0; kt < 5; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nrn = 16 * w + 4 * lg + r, col = 16 * kt + li;
      if (col < NHID) gp[OFF_W2 + nrn * NHID + col] += acc2[kt][r];
      else if (col == NHID) gp[OFF_B2 + nrn] += acc2[kt][r];
    }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j == 1 && w != 0) break;
    const int kt = j == 0 ? w : 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * lg + r, col = 16 * kt + li;
      if (o < NA) {
        if (col < NHID) gp[OFF_W3 + o * NHID + col] += acc3[j][r];
        else if (col == NHID) gp[OFF_B3 + o] += acc3[j][r];
      }
    }
  }
}

// grad[i] = sum over workgroups of gpart[g][i], in ascending g.
__global__ void k_bwd_reduce(const float* __restrict__ gpart, int G, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NW) return;
  float s = 0.0f;
  for (int g = 0; g < G; ++g) s += gpart[(size_t)g * NW + i];
  out[i] = s;
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
  // Step groups of the weight-gradient pass: one workgroup per CU (the
  // double-buffered staging takes most of the LDS), so about n_cu workgroups.
  const int chunks = (int)nb(N, 64);
  int n_cu = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  int S = n_cu / chunks;
  if (S > K) S = K;
  if (S < 1) S = 1;
  bw.dw_groups = S;
  bw.n_parts = chunks * S;
  hipError_t e;
  for (int i = 0; i < BWD_NBUF; ++i) {
    if ((e = hipMalloc(&bw.seg[i], (size_t)K * REC_F * rb_pad(N) * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&bw.dz[i], (size_t)K * DZ_F * rb_pad(N) * 4)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&bw.e_rec[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&bw.e_rev[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&bw.e_dw[i], hipEventDisableTiming)) != hipSuccess) return e;
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
  if ((e = hipMalloc(&bw.gpart, (size_t)bw.n_parts * NW * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gsum, (size_t)NW * 4)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_bwd_reverse,
                               hipFuncAttributeMaxDynamicSharedMemorySize, R_TOTAL * 4)) !=
      hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_bwd_dw, hipFuncAttributeMaxDynamicSharedMemorySize,
                             2 * DW_BUF * 4);
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
hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        hipStream_t st) {
  const int N = c.n_envs;
  const size_t np = (size_t)bw.n_parts * NW;
  hipLaunchKernelGGL(k_fill, dim3(nb((int)np, 256)), dim3(256), 0, st, bw.gpart, np, 0.0f);
  hipLaunchKernelGGL(k_bwd_init, dim3(nb(N, 256)), dim3(256), 0, st, N,
                     d_states ? d_states + (size_t)T * NS * N : nullptr, bw.lam, bw.gth);
  const bool overlap = (int)nb(N, 64) < bw.n_cu;
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
    const int buf = idx % BWD_NBUF;
    if (overlap && idx >= BWD_NBUF) BWD_TRY(hipStreamWaitEvent(s_rec, bw.e_dw[buf], 0));
    BWD_TRY(launch_recompute(c, b, W, n, tape + (size_t)j * CK_F * N, bw.seg[buf], s_rec));
    if (overlap) {
      BWD_TRY(hipEventRecord(bw.e_rec[buf], s_rec));
      BWD_TRY(hipStreamWaitEvent(st, bw.e_rec[buf], 0));
    }
    hipLaunchKernelGGL(k_bwd_reverse, dim3(nb(N, 64)), dim3(256), R_TOTAL * 4, st, c, b.theta, W,
                       tape + (size_t)j * CK_F * N, bw.seg[buf], n, t0, d_rewards, d_states,
                       bw.lam, bw.gth, bw.dz[buf]);
    BWD_TRY(hipGetLastError());
    if (overlap) {
      BWD_TRY(hipEventRecord(bw.e_rev[buf], st));
      BWD_TRY(hipStreamWaitEvent(s_dw, bw.e_rev[buf], 0));
    }
    hipLaunchKernelGGL(k_bwd_dw, dim3(nb(N, 64), bw.dw_groups), dim3(256), 2 * DW_BUF * 4, s_dw, N,
                       bw.seg[buf], bw.dz[buf], n, bw.dw_groups, bw.gpart,
                       (c.flags & F_ACTOR_BF16) ? 1 : 0);
    BWD_TRY(hipGetLastError());
    if (overlap) BWD_TRY(hipEventRecord(bw.e_dw[buf], s_dw));
    last = buf;
  }
  if (overlap) BWD_TRY(hipStreamWaitEvent(st, bw.e_dw[last], 0));
  hipLaunchKernelGGL(k_bwd_reduce, dim3(nb(NW, 256)), dim3(256), 0, st, bw.gpart, bw.n_parts,
                     grad_actor ? grad_actor : bw.gsum);
  if (grad_params)
    hipLaunchKernelGGL(k_copy, dim3(nb(NP * N, 256)), dim3(256), 0, st, bw.gth, grad_params,
                       (size_t)NP * N);
  return hipGetLastError();
}

}  // namespace qs
