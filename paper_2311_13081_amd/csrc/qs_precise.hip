// Double-precision forward path (config flag SIM_F_FP64).
//
// Same step as the single-precision kernels -- observation, actor, action map,
// RK4, renormalisation, reward, history push, termination, truncation, reset
// -- evaluated in double precision throughout, with the state, the action
// history and the per-env parameters stored in double.  The only float32
// decision is the termination box test, taken on the state rounded to float32
// (the precision the single-precision path decides in).  MI355X runs fp64
// vector FMAs at the fp32 rate, so the integrator costs about the same; the
// actor runs on the vector ALUs (no fp64 matrix-core path here).
//
// One env per lane; history ring in HBM (it does not fit in registers in
// double); weights staged in LDS as doubles, transposed so that every lane
// reads the same address.
#include <hip/hip_runtime.h>

#include "qs_device.h"
#include "qs_precise.h"

namespace qs {

constexpr int P_W1T = 0, P_B1 = P_W1T + NO * NHID, P_W2T = P_B1 + NHID,
              P_B2 = P_W2T + NHID * NHID, P_W3T = P_B2 + NHID, P_B3 = P_W3T + NHID * NA,
              P_TOTAL = P_B3 + NA;
static_assert(P_TOTAL * 8 == PRECISE_LDS_BYTES, "LDS layout must fill the launch's LDS");

__device__ inline void uniforms4_f64(uint32_t klo, uint32_t khi, uint32_t env, uint32_t episode,
                                     uint32_t block, uint32_t stream, double u[4]) {
  uint32_t c[4] = {env, episode, block, stream};
  philox4x32_10(c, klo, khi);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = ((double)(c[i] >> 9) + 0.5) * 0x1p-23;
}

__device__ inline void env_params64(const PreciseCfg& p, uint32_t env, double th[NP]) {
  double u[8];
  uniforms4_f64(p.dr_seed_lo, p.dr_seed_hi, env, 0, 0, STREAM_DR, u);
  uniforms4_f64(p.dr_seed_lo, p.dr_seed_hi, env, 0, 1, STREAM_DR, u + 4);
  for (int i = 0; i < NP; ++i) {
    const double f = p.dr_enable ? p.dr_lo[i] + (p.dr_hi[i] - p.dr_lo[i]) * u[i] : 1.0;
    th[i] = p.nominal[i] * f;
  }
}

// Episode disturbance and observation noise, as in the float path, in double.
__device__ inline void disturbance64(const PreciseCfg& p, uint32_t env, uint32_t episode,
                                     double d[6]) {
  for (int i = 0; i < 6; ++i) d[i] = 0.0;
  if (!(p.flags & F_DISTURB)) return;
  double u[8];
  uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, 0, STREAM_DIST, u);
  uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, 1, STREAM_DIST, u + 4);
  for (int i = 0; i < 3; ++i) {
    d[i] = p.dist_force * (2.0 * u[i] - 1.0);
    d[3 + i] = p.dist_torque * (2.0 * u[3 + i] - 1.0);
  }
}

__device__ inline void add_obs_noise64(const PreciseCfg& p, uint32_t env, uint32_t episode,
                                       int t_ep, double f[18]) {
  if (!(p.flags & F_OBS_NOISE)) return;
  double u[20];
  for (int bk = 0; bk < 5; ++bk)
    uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, (uint32_t)t_ep * 5u + (uint32_t)bk,
                  STREAM_NOISE, u + 4 * bk);
  for (int i = 0; i < 18; i += 2) {
    const double r = sqrt(-2.0 * log(u[i]));
    const double ph = 2.0 * 3.141592653589793 * u[i + 1];
    const int g0 = i < 3 ? 0 : i < 12 ? 1 : i < 15 ? 2 : 3;
    const int g1 = (i + 1) < 3 ? 0 : (i + 1) < 12 ? 1 : (i + 1) < 15 ? 2 : 3;
    f[i] += p.noise[g0] * r * cos(ph);
    f[i + 1] += p.noise[g1] * r * sin(ph);
  }
}

__device__ inline void set_disturbance64(Body<double>& B, const double d[6]) {
  B.ax = d[0] * B.inv_m;
  B.ay = d[1] * B.inv_m;
  B.az = d[2] * B.inv_m;
  B.dtx = d[3];
  B.dty = d[4];
  B.dtz = d[5];
}

__device__ inline double hover_rpm64(const PreciseCfg& p, const double th[NP]) {
  const double need = th[0] * p.g / 4.0 - th[4];
  if (th[6] == 0.0) return need / th[5];
  return (-th[5] + sqrt(th[5] * th[5] + 4.0 * th[6] * need)) / (2.0 * th[6]);
}

// Episode-start state and hover action (same distribution as the float path).
__device__ inline double reset64(const PreciseCfg& p, const double th[NP], uint32_t env,
                                 uint32_t episode, double s[NS]) {
  double u[12];
  uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, 0, STREAM_RESET, u);
  uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, 1, STREAM_RESET, u + 4);
  uniforms4_f64(p.seed_lo, p.seed_hi, env, episode, 2, STREAM_RESET, u + 8);
  for (int i = 0; i < 3; ++i) s[i] = p.init_pos * (2.0 * u[i] - 1.0);
  const double z = 2.0 * u[3] - 1.0;
  const double phi = 2.0 * 3.141592653589793 * u[4];
  const double alpha = p.init_angle * u[5];
  const double r = sqrt(fmax(0.0, 1.0 - z * z));
  const double sa = sin(0.5 * alpha);
  s[3] = cos(0.5 * alpha);
  s[4] = sa * r * cos(phi);
  s[5] = sa * r * sin(phi);
  s[6] = sa * z;
  for (int i = 0; i < 3; ++i) s[7 + i] = p.init_vel * (2.0 * u[6 + i] - 1.0);
  for (int i = 0; i < 3; ++i) s[10 + i] = p.init_angvel * (2.0 * u[9 + i] - 1.0);
  const double wh = hover_rpm64(p, th);
  for (int i = 0; i < 4; ++i) s[13 + i] = wh;
  return 2.0 * (wh - p.rpm_min) / (p.rpm_max - p.rpm_min) - 1.0;
}

__global__ void k_precise_init(PreciseCfg p, PreciseBufs b, int params) {
  const int N = p.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double th[NP], s[NS];
  if (params) {
    env_params64(p, (uint32_t)e, th);
    for (int i = 0; i < NP; ++i) b.theta[(size_t)i * N + e] = th[i];
  } else {
    for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  }
  const double ah = reset64(p, th, (uint32_t)e, 0u, s);
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = s[i];
  for (int i = 0; i < NH * NA; ++i) b.ring[(size_t)i * N + e] = ah;
  b.head[e] = 0;
  b.t_ep[e] = 0;
  b.ep[e] = 0;
  b.ret[e] = 0.0;
  b.ret[(size_t)N + e] = 0.0;
  b.last_len[e] = 0;
}

// T steps; outputs indexed by t_base + t, states rounded to float.
__global__ void __launch_bounds__(256)
k_precise(PreciseCfg p, PreciseBufs b, const float* __restrict__ W, const float* __restrict__ ext,
          int T, int t_base, float* __restrict__ rewards, uint8_t* __restrict__ dones,
          float* __restrict__ states) {
  extern __shared__ double lds[];
  if (W) {
    for (int i = threadIdx.x; i < NO * NHID; i += blockDim.x) {
      const int k = i / NHID, n = i % NHID;
      lds[P_W1T + i] = (double)W[OFF_W1 + n * NO + k];
    }
    for (int i = threadIdx.x; i < NHID * NHID; i += blockDim.x) {
      const int k = i / NHID, n = i % NHID;
      lds[P_W2T + i] = (double)W[OFF_W2 + n * NHID + k];
    }
    for (int i = threadIdx.x; i < NHID * NA; i += blockDim.x) {
      const int k = i / NA, n = i % NA;
      lds[P_W3T + i] = (double)W[OFF_W3 + n * NHID + k];
    }
    for (int i = threadIdx.x; i < NHID; i += blockDim.x) {
      lds[P_B1 + i] = (double)W[OFF_B1 + i];
      lds[P_B2 + i] = (double)W[OFF_B2 + i];
    }
    for (int i = threadIdx.x; i < NA; i += blockDim.x) lds[P_B3 + i] = (double)W[OFF_B3 + i];
  }
  __syncthreads();
  const int N = p.n_envs;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double th[NP], x[NS];
  for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  for (int i = 0; i < NS; ++i) x[i] = b.state[(size_t)i * N + e];
  Body<double> B;
  B.inv_m = 1.0 / th[0];
  B.Jx = th[1];
  B.Jy = th[2];
  B.Jz = th[3];
  B.inv_Jx = 1.0 / th[1];
  B.inv_Jy = 1.0 / th[2];
  B.inv_Jz = 1.0 / th[3];
  B.c0 = th[4];
  B.c1 = th[5];
  B.c2 = th[6];
  B.inv_Tm = 1.0 / th[7];
  int head = b.head[e], t_ep = b.t_ep[e], ep = b.ep[e];
  double ret_cur = b.ret[e], ret_last = b.ret[(size_t)N + e];
  int len_last = b.last_len[e];
  {
    double d[6];
    disturbance64(p, (uint32_t)e, (uint32_t)ep, d);
    set_disturbance64(B, d);
  }
  const bool renorm = (p.flags & F_RENORM_Q) != 0;
  if (states && t_base == 0)
    for (int i = 0; i < NS; ++i) states[(size_t)i * N + e] = (float)x[i];
  for (int t = 0; t < T; ++t) {
    const int gt = t_base + t;
    double a[NA];
    if (ext) {
      for (int i = 0; i < NA; ++i) a[i] = (double)ext[((size_t)t * NA + i) * N + e];
    } else {
      // observation: p, R(q/|q|) row-major, v, w, history oldest first
      double o18[18];
      {
        const double n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
        const double nn = sqrt(n2);
        const double w = x[3] / nn, qx = x[4] / nn, qy = x[5] / nn, qz = x[6] / nn;
        o18[0] = x[0];
        o18[1] = x[1];
        o18[2] = x[2];
        o18[3] = 1 - 2 * (qy * qy + qz * qz);
        o18[4] = 2 * (qx * qy - w * qz);
        o18[5] = 2 * (qx * qz + w * qy);
        o18[6] = 2 * (qx * qy + w * qz);
        o18[7] = 1 - 2 * (qx * qx + qz * qz);
        o18[8] = 2 * (qy * qz - w * qx);
        o18[9] = 2 * (qx * qz - w * qy);
        o18[10] = 2 * (qy * qz + w * qx);
        o18[11] = 1 - 2 * (qx * qx + qy * qy);
        for (int i = 0; i < 3; ++i) {
          o18[12 + i] = x[7 + i];
          o18[15 + i] = x[10 + i];
        }
        add_obs_noise64(p, (uint32_t)e, (uint32_t)ep, t_ep, o18);
      }
      double z1[NHID];
#pragma unroll
      for (int n = 0; n < NHID; ++n) z1[n] = lds[P_B1 + n];
#pragma unroll
      for (int k = 0; k < 18; ++k)
#pragma unroll
        for (int n = 0; n < NHID; ++n) z1[n] = fma(lds[P_W1T + k * NHID + n], o18[k], z1[n]);
      for (int k = 18; k < NO; ++k) {
        const int sl = (k - 18) >> 2, c = (k - 18) & 3;
        const double v = b.ring[(size_t)((((head + sl) & (NH - 1)) * NA) + c) * N + e];
#pragma unroll
        for (int n = 0; n < NHID; ++n) z1[n] = fma(lds[P_W1T + k * NHID + n], v, z1[n]);
      }
      // layers 2 and 3 in chunks of 16 hidden units, so only one chunk of the
      // second hidden layer is live next to the first
#pragma unroll
      for (int n = 0; n < NA; ++n) a[n] = lds[P_B3 + n];
#pragma unroll
      for (int cb = 0; cb < NHID; cb += 16) {
        double z2[16];
#pragma unroll
        for (int n = 0; n < 16; ++n) z2[n] = lds[P_B2 + cb + n];
#pragma unroll
        for (int k = 0; k < NHID; ++k) {
          const double v = z1[k] > 0.0 ? z1[k] : 0.0;
#pragma unroll
          for (int n = 0; n < 16; ++n) z2[n] = fma(lds[P_W2T + k * NHID + cb + n], v, z2[n]);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const double v = z2[k] > 0.0 ? z2[k] : 0.0;
#pragma unroll
          for (int n = 0; n < NA; ++n) a[n] = fma(lds[P_W3T + (cb + k) * NA + n], v, a[n]);
        }
      }
      for (int n = 0; n < NA; ++n) a[n] = tanh(a[n]);
    }
    double u[NA];
    for (int i = 0; i < NA; ++i) u[i] = p.rpm_min + 0.5 * (a[i] + 1.0) * (p.rpm_max - p.rpm_min);
    rk4_step<double>(B, p.arm, p.km, p.g, p.dt, renorm, x, u);
    double pp = 0, vv = 0, ww = 0, aa = 0;
    for (int i = 0; i < 3; ++i) {
      pp += x[i] * x[i];
      vv += x[7 + i] * x[7 + i];
      ww += x[10 + i] * x[10 + i];
    }
    for (int i = 0; i < NA; ++i) aa += (a[i] - p.C_rab) * (a[i] - p.C_rab);
    const double r = -p.C_rp * pp - p.C_rq * (1.0 - x[3] * x[3]) - p.C_rv * vv - p.C_rw * ww -
                     p.C_ra * aa + p.C_rs;
    // history push into the ring
    for (int i = 0; i < NA; ++i) b.ring[(size_t)(head * NA + i) * N + e] = a[i];
    head = (head + 1) & (NH - 1);
    ++t_ep;
    uint32_t term = 0;
    if (p.flags & F_TERMINATE) {
      bool out = false, finite = true;
      for (int i = 0; i < 3; ++i) {
        out |= fabsf((float)x[i]) > (float)p.pos_limit;
        out |= fabsf((float)x[7 + i]) > (float)p.vel_limit;
      }
      for (int i = 0; i < NS; ++i) finite &= isfinite(x[i]);
      term = (out || !finite) ? 1u : 0u;
    }
    const uint32_t trunc = (!term && p.max_steps > 0 && t_ep >= p.max_steps) ? 2u : 0u;
    const uint32_t d = term | trunc;
    ret_cur += r;
    if (d && (p.flags & F_AUTORESET)) {
      ret_last = ret_cur;
      len_last = t_ep;
      ret_cur = 0.0;
      ++ep;
      t_ep = 0;
      const double ah = reset64(p, th, (uint32_t)e, (uint32_t)ep, x);
      for (int i = 0; i < NH * NA; ++i) b.ring[(size_t)i * N + e] = ah;
      head = 0;
      double d[6];
      disturbance64(p, (uint32_t)e, (uint32_t)ep, d);
      set_disturbance64(B, d);
    }
    if (rewards) rewards[(size_t)gt * N + e] = (float)r;
    if (dones) dones[(size_t)gt * N + e] = (uint8_t)d;
    if (states)
      for (int i = 0; i < NS; ++i) states[((size_t)(gt + 1) * NS + i) * N + e] = (float)x[i];
  }
  for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = x[i];
  b.head[e] = head;
  b.t_ep[e] = t_ep;
  b.ep[e] = ep;
  b.ret[e] = ret_cur;
  b.ret[(size_t)N + e] = ret_last;
  b.last_len[e] = len_last;
}

// ---------------------------------------------------------------------------
// Quarter-lane kernel of the FP64 path: the actor on fp64 matrix cores.
//
// Each env occupies 4 lanes (lane L = j + 16 k: env j of the wave, quarter
// k); register c of quarter k holds observation feature q_phi(c, k) in
// double: chunk c < 5 state feature 4c + k (two padding slots), chunk c >= 5
// history slot c - 5, component k.  That is the B operand of
// v_mfma_f64_16x16x4_f64 for 16 envs with K-chunk c (B[k][j] in lane
// j + 16 k), so layer 1 is 37 x 4 products against W1 columns taken in the
// same order (A[i][k] in lane i + 16 k).  The result register r of a tile
// holds row 4 r + g in lane group g (the fp64 layout differs from the fp32
// one), i.e. exactly the B operand of the next layer for the K-chunk of
// neurons {16 n + 4 r + g}; the weights of layers 2 and 3 are staged in the
// order each lane reads them, so every LDS read is one contiguous 512-byte
// row.  Layer 3 fills rows 0..3 of one tile; output o then sits in register
// 0 of lane group o and is broadcast to the env's 4 lanes.  The dynamics,
// reward, termination and reset run replicated on the 4 lanes, in double, as
// in k_precise; the history stays in the HBM ring as there (in double it
// does not fit in registers next to the RK4 stages), each lane loading its
// component of the 32 slots per step.  fp64 products have no faster matrix
// rate than vector FMAs
// on this part, but the matrix operands come from registers and
// lane-distinct LDS rows, not from one broadcast LDS read per FMA pair.
// ---------------------------------------------------------------------------
typedef double d4p __attribute__((ext_vector_type(4)));

constexpr int PQ_C = 37;                          // K-chunks of layer 1
constexpr int PQ_W1 = 0;                          // [n 4][c 37][lane 64]
constexpr int PQ_W2 = PQ_W1 + 4 * PQ_C * 64;      // [n2 4][n 4][r 4][lane 64]
constexpr int PQ_W3 = PQ_W2 + 4 * 4 * 4 * 64;     // [n2 4][r 4][lane 64]
constexpr int PQ_B1 = PQ_W3 + 4 * 4 * 64;         // [64]
constexpr int PQ_B2 = PQ_B1 + NHID;               // [64]
constexpr int PQ_B3 = PQ_B2 + NHID;               // [4]
constexpr int PQ_TOTAL = PQ_B3 + NA;              // doubles
constexpr int PQ_LDS_BYTES = PQ_TOTAL * 8;

__host__ __device__ constexpr int pq_phi(int c, int k) {
  return c < 5 ? (4 * c + k < 18 ? 4 * c + k : -1) : 18 + 4 * (c - 5) + k;
}

__device__ inline void stage_pq(const float* __restrict__ W, double* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < 4 * PQ_C * 64; idx += nt) {
    const int L = idx % 64, c = (idx / 64) % PQ_C, n = idx / (64 * PQ_C);
    const int f = pq_phi(c, L >> 4);
    lds[PQ_W1 + idx] = f >= 0 ? (double)W[OFF_W1 + (16 * n + (L & 15)) * NO + f] : 0.0;
  }
  for (int idx = tid; idx < 4 * 4 * 4 * 64; idx += nt) {
    const int L = idx % 64, r = (idx / 64) % 4, n = (idx / 256) % 4, n2 = idx / 1024;
    lds[PQ_W2 + idx] = (double)W[OFF_W2 + (16 * n2 + (L & 15)) * NHID + 16 * n + 4 * r + (L >> 4)];
  }
  for (int idx = tid; idx < 4 * 4 * 64; idx += nt) {
    const int L = idx % 64, r = (idx / 64) % 4, n2 = idx / 256;
    const int o = L & 15;
    lds[PQ_W3 + idx] = o < NA ? (double)W[OFF_W3 + o * NHID + 16 * n2 + 4 * r + (L >> 4)] : 0.0;
  }
  for (int i = tid; i < NHID; i += nt) {
    lds[PQ_B1 + i] = (double)W[OFF_B1 + i];
    lds[PQ_B2 + i] = (double)W[OFF_B2 + i];
  }
  for (int i = tid; i < NA; i += nt) lds[PQ_B3 + i] = (double)W[OFF_B3 + i];
}

__device__ inline double relu64(double v) { return v > 0.0 ? v : 0.0; }

// The actor for the wave's 16 envs: returns the 4 pre-tanh outputs of the
// lane's env in every lane.
__device__ inline void actor_pq(const double* lds, const double F[PQ_C], double z3[NA]) {
  const int L = threadIdx.x & 63, g = L >> 4;
  // The weight reads are pipelined one K-chunk ahead by hand; the empty asm
  // statements keep the compiler from hoisting all of them to the top (which
  // would hold 148 doubles per lane and spill).
  d4p acc1[4];
  double wn[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) wn[n] = lds[PQ_W1 + (n * PQ_C) * 64 + L];
#pragma unroll
  for (int c = 0; c < PQ_C; ++c) {
    double w[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) w[n] = wn[n];
    __asm__ volatile("" ::: "memory");
    if (c + 1 < PQ_C) {
#pragma unroll
      for (int n = 0; n < 4; ++n) wn[n] = lds[PQ_W1 + (n * PQ_C + c + 1) * 64 + L];
    }
    // four independent chains, one per 16-neuron tile
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      d4p b;
      if (c == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = lds[PQ_B1 + 16 * n + 4 * r + g];
      }
      acc1[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[n], F[c], c == 0 ? b : acc1[n], 0, 0, 0);
    }
  }
  d4p acc2[4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    d4p b;
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = lds[PQ_B2 + 16 * n2 + 4 * r + g];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc2[n2] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            lds[PQ_W2 + ((n2 * 4 + n) * 4 + r) * 64 + L], relu64(acc1[n][r]),
            (n == 0 && r == 0) ? b : acc2[n2], 0, 0, 0);
    }
  }
  d4p acc3;
  {
    d4p b = {0.0, 0.0, 0.0, 0.0};
    b[0] = lds[PQ_B3 + g];  // row g of register 0 is output g
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(lds[PQ_W3 + (n2 * 4 + r) * 64 + L],
                                                    relu64(acc2[n2][r]),
                                                    (n2 == 0 && r == 0) ? b : acc3, 0, 0, 0);
  }
  // output o of env j sits in register 0 of lane j + 16 o
  const int j = L & 15;
  const long long v = __double_as_longlong(acc3[0]);
  const int lo = (int)(v & 0xffffffffll), hi = (int)(v >> 32);
#pragma unroll
  for (int o = 0; o < NA; ++o) {
    const int src = (j + 16 * o) << 2;
    const unsigned l2 = (unsigned)__builtin_amdgcn_ds_bpermute(src, lo);
    const unsigned h2 = (unsigned)__builtin_amdgcn_ds_bpermute(src, hi);
    z3[o] = __longlong_as_double((long long)(((unsigned long long)h2 << 32) | l2));
  }
}

// T steps of the FP64 path with the quarter-lane actor (256 threads = 64
// envs per workgroup); outputs indexed by t_base + t, states rounded to
// float.  Same step as k_precise.
__global__ void __launch_bounds__(256)
k_precise4(PreciseCfg p, PreciseBufs b, const float* __restrict__ W, int T, int t_base,
           float* __restrict__ rewards, uint8_t* __restrict__ dones,
           float* __restrict__ states) {
  extern __shared__ double lds[];
  const int N = p.n_envs;
  stage_pq(W, lds);
  __syncthreads();
  const int L = threadIdx.x & 63, j = L & 15, k = L >> 4;
  const int env0 = (blockIdx.x * blockDim.x + threadIdx.x - L) / 4;  // first env of the wave
  if (env0 >= N) return;
  const int env = env0 + j;
  const bool active = env < N;
  const int e = active ? env : env0;

  double th[NP], x[NS];
  for (int i = 0; i < NP; ++i) th[i] = b.theta[(size_t)i * N + e];
  for (int i = 0; i < NS; ++i) x[i] = b.state[(size_t)i * N + e];
  Body<double> B;
  B.inv_m = 1.0 / th[0];
  B.Jx = th[1];
  B.Jy = th[2];
  B.Jz = th[3];
  B.inv_Jx = 1.0 / th[1];
  B.inv_Jy = 1.0 / th[2];
  B.inv_Jz = 1.0 / th[3];
  B.c0 = th[4];
  B.c1 = th[5];
  B.c2 = th[6];
  B.inv_Tm = 1.0 / th[7];
  int head = b.head[e], t_ep = b.t_ep[e], ep = b.ep[e];
  double ret_cur = b.ret[e], ret_last = b.ret[(size_t)N + e];
  int len_last = b.last_len[e];
  {
    double d[6];
    disturbance64(p, (uint32_t)e, (uint32_t)ep, d);
    set_disturbance64(B, d);
  }
  const bool renorm = (p.flags & F_RENORM_Q) != 0;
  if (states && t_base == 0 && active)
    for (int i = 0; i < NS; ++i)
      if ((i & 3) == k) states[(size_t)i * N + e] = (float)x[i];
  for (int t = 0; t < T; ++t) {
    const int gt = t_base + t;
    double F[PQ_C];
    // history, oldest first: component k of each slot
#pragma unroll
    for (int sl = 0; sl < NH; ++sl)
      F[5 + sl] = b.ring[(size_t)((((head + sl) & (NH - 1)) * NA) + k) * N + e];
    // observation state part, as in k_precise; this quarter keeps 4c + k
    {
      double o18[20];
      const double n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
      const double nn = sqrt(n2);
      const double w = x[3] / nn, qx = x[4] / nn, qy = x[5] / nn, qz = x[6] / nn;
      o18[0] = x[0];
      o18[1] = x[1];
      o18[2] = x[2];
      o18[3] = 1 - 2 * (qy * qy + qz * qz);
      o18[4] = 2 * (qx * qy - w * qz);
      o18[5] = 2 * (qx * qz + w * qy);
      o18[6] = 2 * (qx * qy + w * qz);
      o18[7] = 1 - 2 * (qx * qx + qz * qz);
      o18[8] = 2 * (qy * qz - w * qx);
      o18[9] = 2 * (qx * qz - w * qy);
      o18[10] = 2 * (qy * qz + w * qx);
      o18[11] = 1 - 2 * (qx * qx + qy * qy);
      for (int i = 0; i < 3; ++i) {
        o18[12 + i] = x[7 + i];
        o18[15 + i] = x[10 + i];
      }
      o18[18] = 0.0;
      o18[19] = 0.0;
      add_obs_noise64(p, (uint32_t)e, (uint32_t)ep, t_ep, o18);
#pragma unroll
      for (int cc = 0; cc < 5; ++cc)
        F[cc] = k == 0 ? o18[4 * cc] : k == 1 ? o18[4 * cc + 1] : k == 2 ? o18[4 * cc + 2]
                                                                          : o18[4 * cc + 3];
    }
    double z3[NA], a[NA];
    actor_pq(lds, F, z3);
    for (int n = 0; n < NA; ++n) a[n] = tanh(z3[n]);
    double u[NA];
    for (int i = 0; i < NA; ++i) u[i] = p.rpm_min + 0.5 * (a[i] + 1.0) * (p.rpm_max - p.rpm_min);
    rk4_step<double>(B, p.arm, p.km, p.g, p.dt, renorm, x, u);
    double pp = 0, vv = 0, ww = 0, aa = 0;
    for (int i = 0; i < 3; ++i) {
      pp += x[i] * x[i];
      vv += x[7 + i] * x[7 + i];
      ww += x[10 + i] * x[10 + i];
    }
    for (int i = 0; i < NA; ++i) aa += (a[i] - p.C_rab) * (a[i] - p.C_rab);
    const double r = -p.C_rp * pp - p.C_rq * (1.0 - x[3] * x[3]) - p.C_rv * vv - p.C_rw * ww -
                     p.C_ra * aa + p.C_rs;
    // history push into the ring (component k), as in k_precise
    if (active)
      b.ring[(size_t)(head * NA + k) * N + e] = k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
    head = (head + 1) & (NH - 1);
    ++t_ep;
    uint32_t term = 0;
    if (p.flags & F_TERMINATE) {
      bool out = false, finite = true;
      for (int i = 0; i < 3; ++i) {
        out |= fabsf((float)x[i]) > (float)p.pos_limit;
        out |= fabsf((float)x[7 + i]) > (float)p.vel_limit;
      }
      for (int i = 0; i < NS; ++i) finite &= isfinite(x[i]);
      term = (out || !finite) ? 1u : 0u;
    }
    const uint32_t trunc = (!term && p.max_steps > 0 && t_ep >= p.max_steps) ? 2u : 0u;
    const uint32_t d = term | trunc;
    ret_cur += r;
    if (d && (p.flags & F_AUTORESET)) {
      ret_last = ret_cur;
      len_last = t_ep;
      ret_cur = 0.0;
      ++ep;
      t_ep = 0;
      const double ah = reset64(p, th, (uint32_t)e, (uint32_t)ep, x);
      if (active)
        for (int sl = 0; sl < NH; ++sl) b.ring[(size_t)(sl * NA + k) * N + e] = ah;
      head = 0;
      double dd[6];
      disturbance64(p, (uint32_t)e, (uint32_t)ep, dd);
      set_disturbance64(B, dd);
    }
    if (active) {
      if (k == 0 && rewards) rewards[(size_t)gt * N + e] = (float)r;
      if (k == 1 && dones) dones[(size_t)gt * N + e] = (uint8_t)d;
      if (states)
        for (int i = 0; i < NS; ++i)
          if ((i & 3) == k) states[((size_t)(gt + 1) * NS + i) * N + e] = (float)x[i];
    }
  }
  if (!active) return;
  for (int i = 0; i < NS; ++i)
    if ((i & 3) == k) b.state[(size_t)i * N + e] = x[i];
  if (k == 0) {
    b.head[e] = head;
    b.t_ep[e] = t_ep;
    b.ep[e] = ep;
    b.ret[e] = ret_cur;
    b.ret[(size_t)N + e] = ret_last;
    b.last_len[e] = len_last;
  }
}

// Float32 snapshots of the double state (history in logical order).
__global__ void k_precise_get(PreciseBufs b, int N, float* state, float* hist, int32_t* t_ep,
                              int32_t* ep, float* theta, float* ret, int32_t* last_len) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state)
    for (int i = 0; i < NS; ++i) state[(size_t)i * N + e] = (float)b.state[(size_t)i * N + e];
  if (hist) {
    const int h = b.head[e];
    for (int s = 0; s < NH; ++s)
      for (int a = 0; a < NA; ++a)
        hist[(size_t)(s * NA + a) * N + e] =
            (float)b.ring[(size_t)((((h + s) & (NH - 1)) * NA) + a) * N + e];
  }
  if (t_ep) t_ep[e] = b.t_ep[e];
  if (ep) ep[e] = b.ep[e];
  if (theta)
    for (int i = 0; i < NP; ++i) theta[(size_t)i * N + e] = (float)b.theta[(size_t)i * N + e];
  if (ret) {
    ret[e] = (float)b.ret[e];
    ret[(size_t)N + e] = (float)b.ret[(size_t)N + e];
  }
  if (last_len) last_len[e] = b.last_len[e];
}

__global__ void k_precise_set(PreciseBufs b, int N, const float* state, const float* hist,
                              const int32_t* t_ep, const int32_t* ep, const float* theta,
                              const float* ret, const int32_t* last_len) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (state)
    for (int i = 0; i < NS; ++i) b.state[(size_t)i * N + e] = (double)state[(size_t)i * N + e];
  if (hist) {
    for (int i = 0; i < NH * NA; ++i) b.ring[(size_t)i * N + e] = (double)hist[(size_t)i * N + e];
    b.head[e] = 0;
  }
  if (t_ep) b.t_ep[e] = t_ep[e];
  if (ep) b.ep[e] = ep[e];
  if (theta)
    for (int i = 0; i < NP; ++i) b.theta[(size_t)i * N + e] = (double)theta[(size_t)i * N + e];
  if (ret) {
    b.ret[e] = (double)ret[e];
    b.ret[(size_t)N + e] = (double)ret[(size_t)N + e];
  }
  if (last_len) b.last_len[e] = last_len[e];
}

static inline unsigned pb(int n) { return (unsigned)((n + 255) / 256); }

hipError_t precise_prepare() {
  hipError_t e = hipFuncSetAttribute((const void*)k_precise,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, PRECISE_LDS_BYTES);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_precise4, hipFuncAttributeMaxDynamicSharedMemorySize,
                             PQ_LDS_BYTES);
}

hipError_t precise_init(const PreciseCfg& p, const PreciseBufs& b, int params, hipStream_t st) {
  hipLaunchKernelGGL(k_precise_init, dim3(pb(p.n_envs)), dim3(256), 0, st, p, b, params);
  return hipGetLastError();
}

hipError_t precise_run(const PreciseCfg& p, const PreciseBufs& b, const float* W,
                       const float* ext, int T, int t_base, float* rewards, uint8_t* dones,
                       float* states, hipStream_t st) {
  if (W && !ext) {
    // the actor on fp64 matrix cores, 4 lanes per env
    const unsigned grid = (unsigned)((p.n_envs + 63) / 64);
    hipLaunchKernelGGL(k_precise4, dim3(grid), dim3(256), PQ_LDS_BYTES, st, p, b, W, T, t_base,
                       rewards, dones, states);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_precise, dim3(pb(p.n_envs)), dim3(256), PRECISE_LDS_BYTES, st, p, b, W,
                     ext, T, t_base, rewards, dones, states);
  return hipGetLastError();
}

hipError_t precise_get(const PreciseBufs& b, int N, float* state, float* hist, int32_t* t_ep,
                       int32_t* ep, float* theta, float* ret, int32_t* last_len, hipStream_t st) {
  hipLaunchKernelGGL(k_precise_get, dim3(pb(N)), dim3(256), 0, st, b, N, state, hist, t_ep, ep,
                     theta, ret, last_len);
  return hipGetLastError();
}

hipError_t precise_set(const PreciseBufs& b, int N, const float* state, const float* hist,
                       const int32_t* t_ep, const int32_t* ep, const float* theta,
                       const float* ret, const int32_t* last_len, hipStream_t st) {
  hipLaunchKernelGGL(k_precise_set, dim3(pb(N)), dim3(256), 0, st, b, N, state, hist, t_ep, ep,
                     theta, ret, last_len);
  return hipGetLastError();
}

}  // namespace qs
