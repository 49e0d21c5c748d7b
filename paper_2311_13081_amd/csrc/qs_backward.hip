// Discrete adjoint of a taped rollout.
//
// The taped forward stored checkpoints (state, history) every K steps.  The
// backward walks the segments last to first; per segment:
//   1. recompute: the fused MFMA kernel restarts from the checkpoint and
//      records x_t, a_t, the layer pre-activations z1, z2 and o_t per step;
//   2. reverse sweep (k_bwd_reverse): one env per lane, the adjoints of the
//      state (17) and of the action history (128) in registers, stepping
//      back through reward, quaternion renormalisation, the four RK4 stages,
//      the action map, the actor and the history shift; per-env parameter
//      gradients accumulate in registers; the layer cotangents dz1, dz2, dz3
//      of every (step, env) go to scratch;
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

// LDS layout of the reverse kernel (floats).  Transposed weights packed so
// that each lane's MFMA A operand for 4 consecutive K-chunks is one 16-byte
// read:
//   R_W3: W3 row-major [4][64]; A of the 4-block 16x16x1 for dh2 = W3^T dz3.
//   R_W2P[((n*4 + g)*4 + m)*16 + i][v] = W2[16n + 4g + v][16m + i]  (dh1 = W2^T dz2)
//   R_W1P[((m*4 + g)*10 + f)*16 + i][v] = W1[16m + 4g + v][16f + i] (do = W1^T dz1),
//     zero for features 16f + i >= 146.
//   R_ST: per-wave 16 x 68 staging tile for moving do to one env per lane.
constexpr int R_W3 = 0, R_W2P = R_W3 + NA * NHID, R_W1P = R_W2P + NHID * NHID,
              R_ST = R_W1P + 10 * 16 * NHID, R_ST_P = 68, R_ST_SZ = 16 * R_ST_P,
              R_TOTAL = R_ST + 4 * R_ST_SZ;

__device__ inline void stage_reverse(const float* __restrict__ W, float* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < NA * NHID; i += nt) lds[R_W3 + i] = W[OFF_W3 + i];
  for (int idx = tid; idx < NHID * NHID; idx += nt) {
    const int v = idx & 3, i = (idx >> 2) & 15, m = (idx >> 6) & 3, g = (idx >> 8) & 3,
              n = idx >> 10;
    lds[R_W2P + idx] = W[OFF_W2 + (16 * n + 4 * g + v) * NHID + 16 * m + i];
  }
  for (int idx = tid; idx < 10 * 16 * NHID; idx += nt) {
    const int v = idx & 3, i = (idx >> 2) & 15, rest = idx >> 6;  // rest = (m*4 + g)*10 + f
    const int f = rest % 10, g = (rest / 10) & 3, m = rest / 40;
    const int feat = 16 * f + i;
    lds[R_W1P + idx] = feat < NO ? W[OFF_W1 + (16 * m + 4 * g + v) * NO + feat] : 0.0f;
  }
}

// Reverse sweep over steps t0 + n - 1 .. t0 of one segment.  One env per lane
// for the state adjoint, the history adjoint, the RK4/dynamics VJP and the
// parameter gradients; the actor VJP runs on fp32 matrix cores for the wave's
// 64 envs (the forward's layer chaining in reverse): dh2 = W3^T dz3 with the
// 4-block 16x16x1 MFMA from the per-lane dz3, dh1 = W2^T dz2 and
// do = W1^T dz1 with 16x16x4 MFMAs fed by the previous result registers.  do
// comes out as (feature, env) tiles; each 16-feature tile goes through a
// per-wave LDS tile to one env per lane, newest history feature first so the
// history-adjoint shift can run in place.  Inactive lanes of the last wave
// shadow the wave's first env (reads only).
__global__ void __launch_bounds__(256)
k_bwd_reverse(DevCfg c, const float* __restrict__ theta, const float* __restrict__ W,
              const float* __restrict__ rec, int n, int t0, const float* __restrict__ d_rewards,
              const float* __restrict__ d_states, float* __restrict__ lam,
              float* __restrict__ gth_io, float* __restrict__ dz) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  stage_reverse(W, lds);
  __syncthreads();
  const int N = c.n_envs;
  const int env = blockIdx.x * blockDim.x + threadIdx.x;
  const int first = env - (threadIdx.x & 63);
  if (first >= N) return;
  const bool active = env < N;
  const int e = active ? env : first;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  float* stg = lds + R_ST + (threadIdx.x >> 6) * R_ST_SZ;

  float th[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) th[i] = theta[(size_t)i * N + e];
  const Body<float> B = make_body<float>(th);
  const bool renorm = (c.flags & F_RENORM_Q) != 0;
  const float h = c.dt;

  float ls[NS], lH[NH * NA], gth[NP];
#pragma unroll
  for (int i = 0; i < NS; ++i) ls[i] = lam[(size_t)i * N + e];
#pragma unroll
  for (int i = 0; i < NH * NA; ++i) lH[i] = lam[(size_t)(NS + i) * N + e];
#pragma unroll
  for (int i = 0; i < NP; ++i) gth[i] = gth_io[(size_t)i * N + e];

  for (int tl = n - 1; tl >= 0; --tl) {
    __asm__ volatile("" ::: "memory");
    const uint32_t eo = opaque((uint32_t)e);
    const int t = t0 + tl;
    const float* rt = rec + (size_t)tl * REC_F * N;
    float* dzt = dz + (size_t)tl * DZ_F * N;
    float x[NS], a[NA], u[NA];
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = rt[(size_t)(REC_X + i) * N + eo];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      a[i] = rt[(size_t)(REC_A + i) * N + eo];
      u[i] = action_to_rpm(c, a[i]);
    }
    const float dR = d_rewards ? d_rewards[(size_t)t * N + eo] : 1.0f;

    // --- forward recompute of the RK4 stages -------------------------------
    float x2[NS], x3[NS], x4[NS], k[NS], acc[NS];
    deriv<float>(B, c.arm, c.km, c.g, x, u, k);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] = k[i];
      x2[i] = x[i] + 0.5f * h * k[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x2, u, k);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] += 2.0f * k[i];
      x3[i] = x[i] + 0.5f * h * k[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x3, u, k);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      acc[i] += 2.0f * k[i];
      x4[i] = x[i] + h * k[i];
    }
    deriv<float>(B, c.arm, c.km, c.g, x4, u, k);
    float sn[NS];  // post-step state (renormalised)
#pragma unroll
    for (int i = 0; i < NS; ++i) sn[i] = x[i] + (h / 6.0f) * (acc[i] + k[i]);
    float rn = 1.0f;
    if (renorm) {
      rn = 1.0f / sqrtf(sn[3] * sn[3] + sn[4] * sn[4] + sn[5] * sn[5] + sn[6] * sn[6]);
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
#pragma unroll
    for (int i = 0; i < NA; ++i)
      ga[i] = -2.0f * c.C_ra * (a[i] - c.C_rab) * dR + lH[(NH - 1) * NA + i];

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
    // Pre-activations of the wave's 64 envs in the (neuron, env) tile layout:
    // register r of tile q holds neuron 16q + 4lg + (r&3) of env
    // first + 16(r>>2) + li (clamped to the last env for the ragged tail).
    const int ed = opaque((uint32_t)(first + li));
    float m2[4][16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ee = min(ed + 16 * (r >> 2), N - 1);
        m2[q][r] = rt[(size_t)(REC_Z2 + 16 * q + 4 * lg + (r & 3)) * N + ee];
      }
    float d3[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      d3[i] = ga[i] * (1.0f - a[i] * a[i]);
      if (active) dzt[(size_t)(2 * NHID + i) * N + eo] = d3[i];
    }
    // dz2 = (W3^T dz3) * [z2 > 0]
    f16 dz2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int r = 0; r < 16; ++r) dz2[q][r] = 0.0f;
#pragma unroll
      for (int o = 0; o < NA; ++o)
        dz2[q] = __builtin_amdgcn_mfma_f32_16x16x1f32(lds[R_W3 + o * NHID + 16 * q + li], d3[o],
                                                      dz2[q], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        dz2[q][r] = m2[q][r] > 0.0f ? dz2[q][r] : 0.0f;
        const int ee = ed + 16 * (r >> 2);
        if (ee < N) dzt[(size_t)(NHID + 16 * q + 4 * lg + (r & 3)) * N + ee] = dz2[q][r];
      }
    }
    float m1[4][16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ee = min(ed + 16 * (r >> 2), N - 1);
        m1[q][r] = rt[(size_t)(REC_Z1 + 16 * q + 4 * lg + (r & 3)) * N + ee];
      }
    // dz1 = (W2^T dz2) * [z1 > 0]; tile m, env block b in dz1[m][4b .. 4b+3]
    f16 dz1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 accb[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) accb[bb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4 w = *reinterpret_cast<const f4*>(
            &lds[R_W2P + (((q * 4 + lg) * 4 + mt) * 16 + li) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            accb[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[v], dz2[q][4 * bb + v], accb[bb],
                                                            0, 0, 0);
      }
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float v = m1[mt][4 * bb + r] > 0.0f ? accb[bb][r] : 0.0f;
          dz1[mt][4 * bb + r] = v;
          const int ee = ed + 16 * bb;
          if (ee < N) dzt[(size_t)(16 * mt + 4 * lg + r) * N + ee] = v;
        }
    }
    // do = W1^T dz1, one 16-feature tile at a time, newest features first.
#pragma unroll
    for (int f = 9; f >= 0; --f) {
      f4 accb[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) accb[bb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const f4 w = *reinterpret_cast<const f4*>(
            &lds[R_W1P + (((mt * 4 + lg) * 10 + f) * 16 + li) * 4]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            accb[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[v], dz1[mt][4 * bb + v], accb[bb],
                                                            0, 0, 0);
      }
      // tile -> one env per lane: row 4lg + r, column 16bb + li
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int r = 0; r < 4; ++r) stg[(4 * lg + r) * R_ST_P + 16 * bb + li] = accb[bb][r];
      __builtin_amdgcn_wave_barrier();
      float dob[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) dob[r] = stg[r * R_ST_P + lane];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        const int kk = 16 * f + r;
        if (kk >= NO) continue;
        const float v = dob[r];
        if (kk >= 18) {
          // H_t[j] feeds H_{t+1}[j-1] (j >= 1); j descending keeps older
          // adjoints intact until read.
          const int jj = kk - 18;
          lH[jj] = (jj >= NA ? lH[jj - NA] : 0.0f) + v;
        } else if (kk < 3) {
          gx[kk] += v;
        } else if (kk < 12) {
          k[kk - 3] = v;  // rotation-matrix cotangent
        } else if (kk < 15) {
          gx[7 + kk - 12] += v;
        } else {
          gx[10 + kk - 15] += v;
        }
      }
    }
    {
      float gq[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      const float q[4] = {x[3], x[4], x[5], x[6]};
      rotmat_vjp(q, k, gq);
#pragma unroll
      for (int i = 0; i < 4; ++i) gx[3 + i] += gq[i];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
      ls[i] = gx[i] + (d_states ? d_states[((size_t)t * NS + i) * N + eo] : 0.0f);
  }
  if (!active) return;
  const uint32_t ef = opaque((uint32_t)e);
#pragma unroll
  for (int i = 0; i < NS; ++i) lam[(size_t)i * N + ef] = ls[i];
#pragma unroll
  for (int i = 0; i < NH * NA; ++i) lam[(size_t)(NS + i) * N + ef] = lH[i];
#pragma unroll
  for (int i = 0; i < NP; ++i) gth_io[(size_t)i * N + ef] = gth[i];
}

// Weight gradients of one segment: for every (step, env) row,
//   dW1 += dz1 o^T, dW2 += dz2 relu(z1)^T, dW3 += dz3 relu(z2)^T, db += dz,
// as MFMA reductions over 16 rows at a time.  Workgroup = 4 waves over a
// 64-env chunk; wave w owns neuron tile w of dW1 and dW2 and feature tile w
// of dW3 (wave 0 also tile 4).
constexpr int DW_P = 68;  // LDS row pitch (64 envs + 4)
constexpr int DW_O_ROWS = 160, DW_H_ROWS = 80;
constexpr int DW_D1 = 0, DW_D2 = DW_D1 + NHID * DW_P, DW_D3 = DW_D2 + NHID * DW_P,
              DW_O = DW_D3 + 16 * DW_P, DW_H1 = DW_O + DW_O_ROWS * DW_P,
              DW_H2 = DW_H1 + DW_H_ROWS * DW_P, DW_TOTAL = DW_H2 + DW_H_ROWS * DW_P;

__global__ void __launch_bounds__(256)
k_bwd_dw(int N, const float* __restrict__ rec, const float* __restrict__ dz, int n,
         float* __restrict__ gpart) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int env0 = blockIdx.x * 64;

  f4 acc1[10], acc2[5], acc3[2];
#pragma unroll
  for (int i = 0; i < 10; ++i) acc1[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < 5; ++i) acc2[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  acc3[0] = acc3[1] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  for (int tl = 0; tl < n; ++tl) {
    const float* rt = rec + (size_t)tl * REC_F * N;
    const float* dzt = dz + (size_t)tl * DZ_F * N;
    __syncthreads();  // previous step's tiles consumed
    // Stage the 64-env chunk: rows are features, columns envs.  Each thread
    // moves 4 consecutive envs of a row; the loads of one pass are issued
    // together (unrolled) so their latencies overlap.
    const bool full = (env0 + 64 <= N) && ((N & 3) == 0);
    const int c4 = (tid & 15) * 4;
#pragma unroll 4
    for (int row = tid >> 4; row < DW_TOTAL / DW_P; row += 16) {
      const float* src = nullptr;
      int kind = 0;  // 0: copy, 1: relu, 2: ones (valid envs), 3: zeros
      if (row < 2 * NHID) {
        src = dzt + (size_t)row * N;
      } else if (row < 2 * NHID + 16) {
        const int r = row - 2 * NHID;
        if (r < NA) src = dzt + (size_t)(2 * NHID + r) * N; else kind = 3;
      } else if (row < 2 * NHID + 16 + DW_O_ROWS) {
        const int r = row - (2 * NHID + 16);
        if (r < NO) src = rt + (size_t)(REC_O + r) * N; else kind = r == NO ? 2 : 3;
      } else if (row < 2 * NHID + 16 + DW_O_ROWS + DW_H_ROWS) {
        const int r = row - (2 * NHID + 16 + DW_O_ROWS);
        if (r < NHID) { src = rt + (size_t)(REC_Z1 + r) * N; kind = 1; } else kind = r == NHID ? 2 : 3;
      } else {
        const int r = row - (2 * NHID + 16 + DW_O_ROWS + DW_H_ROWS);
        if (r < NHID) { src = rt + (size_t)(REC_Z2 + r) * N; kind = 1; } else kind = r == NHID ? 2 : 3;
      }
      f4 v;
      if (src) {
        if (full) {
          v = *reinterpret_cast<const f4*>(src + env0 + c4);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = env0 + c4 + q < N ? src[env0 + c4 + q] : 0.0f;
        }
        if (kind == 1)
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q], 0.0f);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (kind == 2 && env0 + c4 + q < N) ? 1.0f : 0.0f;
      }
      *reinterpret_cast<f4*>(&sm[row * DW_P + c4]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = 16 * q + 4 * lg;  // this lane's 4 rows (envs) of the 16
      const f4 a1 = *reinterpret_cast<const f4*>(&sm[DW_D1 + (16 * wave + li) * DW_P + c0]);
      const f4 a2 = *reinterpret_cast<const f4*>(&sm[DW_D2 + (16 * wave + li) * DW_P + c0]);
      const f4 a3 = *reinterpret_cast<const f4*>(&sm[DW_D3 + li * DW_P + c0]);
#pragma unroll
      for (int kt = 0; kt < 10; ++kt) {
        const f4 bo = *reinterpret_cast<const f4*>(&sm[DW_O + (16 * kt + li) * DW_P + c0]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc1[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[m], bo[m], acc1[kt], 0, 0, 0);
      }
#pragma unroll
      for (int kt = 0; kt < 5; ++kt) {
        const f4 bh = *reinterpret_cast<const f4*>(&sm[DW_H1 + (16 * kt + li) * DW_P + c0]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc2[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[m], bh[m], acc2[kt], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int kt = j == 0 ? wave : 4;
        if (j == 1 && wave != 0) break;
        const f4 bh = *reinterpret_cast<const f4*>(&sm[DW_H2 + (16 * kt + li) * DW_P + c0]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[m], bh[m], acc3[j], 0, 0, 0);
      }
    }
  }
  // Result register r of a tile holds row 4 lg + r, column li.
  float* gp = gpart + (size_t)blockIdx.x * NW;
#pragma unroll
  for (int kt = 0; kt < 10; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nrn = 16 * wave + 4 * lg + r, col = 16 * kt + li;
      if (col < NO) gp[OFF_W1 + nrn * NO + col] += acc1[kt][r];
      else if (col == NO) gp[OFF_B1 + nrn] += acc1[kt][r];
    }
#pragma unroll
  for (int kt = 0; kt < 5; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nrn = 16 * wave + 4 * lg + r, col = 16 * kt + li;
      if (col < NHID) gp[OFF_W2 + nrn * NHID + col] += acc2[kt][r];
      else if (col == NHID) gp[OFF_B2 + nrn] += acc2[kt][r];
    }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j == 1 && wave != 0) break;
    const int kt = j == 0 ? wave : 4;
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
  bw.n_parts = (int)nb(N, 64);
  hipError_t e;
  if ((e = hipMalloc(&bw.seg, (size_t)K * REC_F * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.dz, (size_t)K * DZ_F * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.lam, (size_t)LAM_F * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gth, (size_t)NP * N * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gpart, (size_t)bw.n_parts * NW * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&bw.gsum, (size_t)NW * 4)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_bwd_reverse,
                               hipFuncAttributeMaxDynamicSharedMemorySize, R_TOTAL * 4)) !=
      hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_bwd_dw, hipFuncAttributeMaxDynamicSharedMemorySize,
                             DW_TOTAL * 4);
}

void bwd_free(BwdBufs& bw) {
  void* ptrs[] = {bw.seg, bw.dz, bw.lam, bw.gth, bw.gpart, bw.gsum};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  bw = BwdBufs{};
}

hipError_t run_backward(const DevCfg& c, const SimBufs& b, BwdBufs& bw, const float* W,
                        const float* tape, int K, int T, const float* d_rewards,
                        const float* d_states, float* grad_actor, float* grad_params,
                        hipStream_t st) {
  const int N = c.n_envs;
  const size_t np = (size_t)bw.n_parts * NW;
  hipLaunchKernelGGL(k_fill, dim3(nb((int)np, 256)), dim3(256), 0, st, bw.gpart, np, 0.0f);
  hipLaunchKernelGGL(k_bwd_init, dim3(nb(N, 256)), dim3(256), 0, st, N,
                     d_states ? d_states + (size_t)T * NS * N : nullptr, bw.lam, bw.gth);
  const int J = (T + K - 1) / K;
  for (int j = J - 1; j >= 0; --j) {
    const int t0 = j * K;
    const int n = (T - t0) < K ? (T - t0) : K;
    hipError_t e = launch_recompute(c, b, W, n, tape + (size_t)j * LAM_F * N, bw.seg, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bwd_reverse, dim3(nb(N, 256)), dim3(256), R_TOTAL * 4, st, c, b.theta, W,
                       bw.seg, n, t0, d_rewards, d_states, bw.lam, bw.gth, bw.dz);
    hipLaunchKernelGGL(k_bwd_dw, dim3(bw.n_parts), dim3(256), DW_TOTAL * 4, st, N, bw.seg, bw.dz,
                       n, bw.gpart);
  }
  hipLaunchKernelGGL(k_bwd_reduce, dim3(nb(NW, 256)), dim3(256), 0, st, bw.gpart, bw.n_parts,
                     grad_actor ? grad_actor : bw.gsum);
  if (grad_params)
    hipLaunchKernelGGL(k_copy, dim3(nb(NP * N, 256)), dim3(256), 0, st, bw.gth, grad_params,
                       (size_t)NP * N);
  return hipGetLastError();
}

}  // namespace qs
