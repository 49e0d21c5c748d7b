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
    if (d && (p.flags & F_AUTORESET)) {
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
}

// Float32 snapshots of the double state (history in logical order).
__global__ void k_precise_get(PreciseBufs b, int N, float* state, float* hist, int32_t* t_ep,
                              int32_t* ep, float* theta) {
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
}

__global__ void k_precise_set(PreciseBufs b, int N, const float* state, const float* hist,
                              const int32_t* t_ep, const int32_t* ep, const float* theta) {
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
}

static inline unsigned pb(int n) { return (unsigned)((n + 255) / 256); }

hipError_t precise_prepare() {
  return hipFuncSetAttribute((const void*)k_precise, hipFuncAttributeMaxDynamicSharedMemorySize,
                             PRECISE_LDS_BYTES);
}

hipError_t precise_init(const PreciseCfg& p, const PreciseBufs& b, int params, hipStream_t st) {
  hipLaunchKernelGGL(k_precise_init, dim3(pb(p.n_envs)), dim3(256), 0, st, p, b, params);
  return hipGetLastError();
}

hipError_t precise_run(const PreciseCfg& p, const PreciseBufs& b, const float* W,
                       const float* ext, int T, int t_base, float* rewards, uint8_t* dones,
                       float* states, hipStream_t st) {
  hipLaunchKernelGGL(k_precise, dim3(pb(p.n_envs)), dim3(256), PRECISE_LDS_BYTES, st, p, b, W,
                     ext, T, t_base, rewards, dones, states);
  return hipGetLastError();
}

hipError_t precise_get(const PreciseBufs& b, int N, float* state, float* hist, int32_t* t_ep,
                       int32_t* ep, float* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_precise_get, dim3(pb(N)), dim3(256), 0, st, b, N, state, hist, t_ep, ep,
                     theta);
  return hipGetLastError();
}

hipError_t precise_set(const PreciseBufs& b, int N, const float* state, const float* hist,
                       const int32_t* t_ep, const int32_t* ep, const float* theta,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_precise_set, dim3(pb(N)), dim3(256), 0, st, b, N, state, hist, t_ep, ep,
                     theta);
  return hipGetLastError();
}

}  // namespace qs
