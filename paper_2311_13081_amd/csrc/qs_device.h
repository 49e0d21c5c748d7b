// Device-side pieces shared by every kernel of the library: the per-launch
// configuration, the counter RNG, the reset distribution, the quadrotor
// dynamics, RK4, reward and termination.  One env is one lane; everything here
// is scalar per env.  Equations: "Learning to Fly in Seconds", Sec. IV.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

constexpr int NS = 17, NH = 32, NA = 4, NO = 146, NHID = 64, NP = 8, NW = 13828;
constexpr int OFF_W1 = 0, OFF_B1 = NHID * NO, OFF_W2 = OFF_B1 + NHID, OFF_B2 = OFF_W2 + NHID * NHID,
              OFF_W3 = OFF_B2 + NHID, OFF_B3 = OFF_W3 + NA * NHID;
constexpr int F_TERMINATE = 1, F_AUTORESET = 2, F_RENORM_Q = 4, F_ACTOR_BF16 = 16,
              F_DISTURB = 32, F_OBS_NOISE = 64;
constexpr uint32_t STREAM_RESET = 0, STREAM_DR = 1, STREAM_DIST = 2, STREAM_NOISE = 3;

// Everything a kernel needs from the configuration, in single precision,
// passed by value.
struct DevCfg {
  int n_envs, max_steps, flags, dr_enable;
  float dt, g, arm, km, rpm_min, rpm_half_range;
  float pos_limit, vel_limit, init_pos, init_angle, init_vel, init_angvel;
  float C_rp, C_rq, C_rv, C_rw, C_ra, C_rab, C_rs;
  float nominal[NP], dr_lo[NP], dr_hi[NP];
  uint32_t seed_lo, seed_hi, dr_seed_lo, dr_seed_hi;
  float dist_force, dist_torque;  // per-component bounds of the episode disturbance
  float noise[4];                 // observation noise std: p, R entries, v, w
  // Set-point shift of the actor's observation ([6][N]: position and
  // velocity set points per env; NULL = none): the actor sees p - p_sp and
  // v - v_sp, each component clipped to +-pos_clip, +-vel_clip.
  const float* target;
  float pos_clip, vel_clip;
};

// Set point of env e (zeros without a target), loaded once per launch.
struct SetPoint {
  float p[3], v[3];
  __device__ inline void load(const DevCfg& c, int N, int e) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p[i] = c.target ? c.target[(size_t)i * N + e] : 0.0f;
      v[i] = c.target ? c.target[(size_t)(3 + i) * N + e] : 0.0f;
    }
  }
  // Shifts the observed position f[0..2] and velocity f[12..14] of the 18
  // state features (Sec. IV: a position controller follows a moving set point
  // through this offset; clipping keeps the errors within the trained range).
  __device__ inline void apply(const DevCfg& c, float f[18]) const {
    if (!c.target) return;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      f[i] = fminf(fmaxf(f[i] - p[i], -c.pos_clip), c.pos_clip);
      f[12 + i] = fminf(fmaxf(f[12 + i] - v[i], -c.vel_clip), c.vel_clip);
    }
  }
};

// Device state of the batch, struct-of-arrays, N = n_envs.
struct SimBufs {
  float* state;    // [17][N]
  float* ring;     // [32][4][N] action history ring; logical slot s at (head+s)&31
  int32_t* head;   // [N]
  int32_t* t_ep;   // [N] steps in the current episode
  int32_t* ep;     // [N] episode index
  float* theta;    // [8][N] m, Jxx, Jyy, Jzz, c0, c1, c2, Tm
  float* ret;      // [2][N] return of the current episode so far; of the last finished one
  int32_t* last_len;  // [N] steps of the last finished episode (0 until one finishes)
};

// Episode accumulators of one env (Sec. V: episode return and length are
// the training measures).  An episode closes when the env is reset inside
// the step: its return and length become the "last" values and the running
// return restarts at zero.  Without in-step resets the running return keeps
// summing.
struct EpAcc {
  float cur, last;
  int len;
  __device__ inline void load(const SimBufs& b, int N, int e) {
    cur = b.ret[e];
    last = b.ret[(size_t)N + e];
    len = b.last_len[e];
  }
  // after the step's reward r; t_ep = steps of the episode including this one
  __device__ inline void add(float r, bool rst, int t_ep) {
    cur += r;
    last = rst ? cur : last;
    len = rst ? t_ep : len;
    cur = rst ? 0.0f : cur;
  }
  __device__ inline void store(const SimBufs& b, int N, uint32_t e) const {
    b.ret[e] = cur;
    b.ret[(size_t)N + e] = last;
    b.last_len[e] = len;
  }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 counter RNG (Salmon et al., SC'11).  Counter (env, episode,
// block, stream), key = 64-bit seed.  Uniform u = (2k+1) 2^-24, k the top 23
// bits, exact in float.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline void uniforms4(uint32_t klo, uint32_t khi, uint32_t env, uint32_t episode,
                                 uint32_t block, uint32_t stream, float u[4]) {
  uint32_t c[4] = {env, episode, block, stream};
  philox4x32_10(c, klo, khi);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = ((float)(c[i] >> 9) + 0.5f) * 0x1p-23f;
}

// Per-env parameters: nominal times U(lo, hi) factors when randomised.
__device__ inline void env_params(const DevCfg& c, uint32_t env, float th[NP]) {
  float u[8];
  uniforms4(c.dr_seed_lo, c.dr_seed_hi, env, 0, 0, STREAM_DR, u);
  uniforms4(c.dr_seed_lo, c.dr_seed_hi, env, 0, 1, STREAM_DR, u + 4);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const float f = c.dr_enable ? c.dr_lo[i] + (c.dr_hi[i] - c.dr_lo[i]) * u[i] : 1.0f;
    th[i] = c.nominal[i] * f;
  }
}

// Hover rotor speed: positive root of c2 w^2 + c1 w + c0 = m g / 4, in the
// cancellation-free form 2 need / (c1 + sqrt(c1^2 + 4 c2 need)).
__device__ inline float hover_rpm(const DevCfg& c, float m, float c0, float c1, float c2) {
  const float need = m * c.g * 0.25f - c0;
  return 2.0f * need / (c1 + sqrtf(c1 * c1 + 4.0f * c2 * need));
}

__device__ inline float rpm_to_action(const DevCfg& c, float w) {
  return (w - c.rpm_min) / c.rpm_half_range - 1.0f;
}

// Episode disturbance {f_r (world frame), tau_r (body frame)} of (env,
// episode): each component uniform in [-F, F] resp. [-T, T], held for the
// episode (Sec. IV, asymmetric actor-critic paragraph); zero with the flag off.
__device__ inline void disturbance(const DevCfg& c, uint32_t env, uint32_t episode, float d[6]) {
  if (!(c.flags & F_DISTURB)) {
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = 0.0f;
    return;
  }
  float u[8];
  uniforms4(c.seed_lo, c.seed_hi, env, episode, 0, STREAM_DIST, u);
  uniforms4(c.seed_lo, c.seed_hi, env, episode, 1, STREAM_DIST, u + 4);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    d[i] = c.dist_force * (2.0f * u[i] - 1.0f);
    d[3 + i] = c.dist_torque * (2.0f * u[3 + i] - 1.0f);
  }
}

// Adds the actor's observation noise to the 18 state features f (p, R
// row-major, v, w) of step t_ep of an episode: f_i += sigma_g z_i, z standard
// normal by Box-Muller on consecutive uniform pairs of stream STREAM_NOISE,
// blocks 5 t_ep .. 5 t_ep + 4.  No-op with the flag off.
__device__ inline void add_obs_noise(const DevCfg& c, uint32_t env, uint32_t episode, int t_ep,
                                     float f[18]) {
  if (!(c.flags & F_OBS_NOISE)) return;
  float u[20];
#pragma unroll
  for (int bk = 0; bk < 5; ++bk)
    uniforms4(c.seed_lo, c.seed_hi, env, episode, (uint32_t)t_ep * 5u + (uint32_t)bk,
              STREAM_NOISE, u + 4 * bk);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float r = sqrtf(-2.0f * logf(u[2 * i]));
    float sn, cs;
    sincosf(6.283185307179586f * u[2 * i + 1], &sn, &cs);
    const int g0 = (2 * i) < 3 ? 0 : (2 * i) < 12 ? 1 : (2 * i) < 15 ? 2 : 3;
    const int g1 = (2 * i + 1) < 3 ? 0 : (2 * i + 1) < 12 ? 1 : (2 * i + 1) < 15 ? 2 : 3;
    f[2 * i] += c.noise[g0] * r * cs;
    f[2 * i + 1] += c.noise[g1] * r * sn;
  }
}

// Episode-start state for (env, episode): p, attitude (angle about a uniform
// axis), v, w uniform in their ranges, rotors at the env's hover speed wh
// (constant per env, so loops compute it once).
__device__ inline void reset_draw(const DevCfg& c, uint32_t env, uint32_t episode, float wh,
                                  float s[NS]) {
  float u[12];
  uniforms4(c.seed_lo, c.seed_hi, env, episode, 0, STREAM_RESET, u);
  uniforms4(c.seed_lo, c.seed_hi, env, episode, 1, STREAM_RESET, u + 4);
  uniforms4(c.seed_lo, c.seed_hi, env, episode, 2, STREAM_RESET, u + 8);
#pragma unroll
  for (int i = 0; i < 3; ++i) s[i] = c.init_pos * (2.0f * u[i] - 1.0f);
  const float z = 2.0f * u[3] - 1.0f;
  const float phi = 6.283185307179586f * u[4];
  const float half = 0.5f * c.init_angle * u[5];
  const float r = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  float sp, cp, sa, ca;
  sincosf(phi, &sp, &cp);
  sincosf(half, &sa, &ca);
  s[3] = ca;
  s[4] = sa * r * cp;
  s[5] = sa * r * sp;
  s[6] = sa * z;
#pragma unroll
  for (int i = 0; i < 3; ++i) s[7 + i] = c.init_vel * (2.0f * u[6 + i] - 1.0f);
#pragma unroll
  for (int i = 0; i < 3; ++i) s[10 + i] = c.init_angvel * (2.0f * u[9 + i] - 1.0f);
#pragma unroll
  for (int i = 0; i < 4; ++i) s[13 + i] = wh;
}

// Start states drawn ahead.  In a wave of many envs, drawing at the moment
// of a reset runs the draw in every step in which any of the envs resets
// (most steps).  The fused kernels instead keep each env's next start state
// (all but the rotor speeds, which start at the hover speed) in registers:
// a reset takes it, and the envs that used theirs draw the following one
// together every RESERVE_PERIOD steps.  An env that resets again before its
// refill draws in place.  The draws are the same counter-based ones either
// way, so results do not depend on when they are made.
constexpr int RESERVE_PERIOD = 16;  // power of 2
constexpr int NRES = NS - NA;      // drawn-ahead state values

__device__ inline void draw_ahead(const DevCfg& c, uint32_t env, uint32_t episode, float wh,
                                  float nx[NRES]) {
  float s0[NS];
  reset_draw(c, env, episode, wh, s0);
#pragma unroll
  for (int i = 0; i < NRES; ++i) nx[i] = s0[i];
}

// Start state of episode `episode`: the reserve if there is one, else drawn.
__device__ inline void reset_from_reserve(const DevCfg& c, uint32_t env, uint32_t episode,
                                          float wh, const float nx[NRES], bool& have,
                                          float s[NS]) {
  if (have) {
#pragma unroll
    for (int i = 0; i < NRES; ++i) s[i] = nx[i];
#pragma unroll
    for (int i = NRES; i < NS; ++i) s[i] = wh;
    have = false;
  } else {
    reset_draw(c, env, episode, wh, s);
  }
}

// reset_draw with the hover speed of parameters (m, c0, c1, c2); returns the
// hover action that fills the history.
__device__ inline float reset_state(const DevCfg& c, uint32_t env, uint32_t episode, float m,
                                    float c0, float c1, float c2, float s[NS]) {
  const float wh = hover_rpm(c, m, c0, c1, c2);
  reset_draw(c, env, episode, wh, s);
  return rpm_to_action(c, wh);
}

// ---------------------------------------------------------------------------
// Dynamics, templated on the arithmetic type R of the integrator.
// Rotor i sits at (sx_i l, sy_i l, 0) with spin sign d_i:
//   sx = (+,-,-,+), sy = (-,-,+,+), d = (-,+,-,+).
// ---------------------------------------------------------------------------
template <typename R>
struct Body {
  R inv_m, Jx, Jy, Jz, inv_Jx, inv_Jy, inv_Jz, c0, c1, c2, inv_Tm;
  R ax, ay, az;     // episode disturbance force over mass (world frame)
  R dtx, dty, dtz;  // episode disturbance torque (body frame)
};

template <typename R>
__device__ inline Body<R> make_body(const float th[NP]) {
  Body<R> b;
  b.inv_m = R(1) / R(th[0]);
  b.Jx = R(th[1]);
  b.Jy = R(th[2]);
  b.Jz = R(th[3]);
  b.inv_Jx = R(1) / b.Jx;
  b.inv_Jy = R(1) / b.Jy;
  b.inv_Jz = R(1) / b.Jz;
  b.c0 = R(th[4]);
  b.c1 = R(th[5]);
  b.c2 = R(th[6]);
  b.inv_Tm = R(1) / R(th[7]);
  b.ax = b.ay = b.az = R(0);
  b.dtx = b.dty = b.dtz = R(0);
  return b;
}

// Sets the episode disturbance d = {f_r, tau_r} of a body.
template <typename R>
__device__ inline void set_disturbance(Body<R>& b, const float d[6]) {
  b.ax = R(d[0]) * b.inv_m;
  b.ay = R(d[1]) * b.inv_m;
  b.az = R(d[2]) * b.inv_m;
  b.dtx = R(d[3]);
  b.dty = R(d[4]);
  b.dtz = R(d[5]);
}

__device__ inline float rsqrt_r(float x) { return __frsqrt_rn(x); }
__device__ inline double rsqrt_r(double x) { return 1.0 / sqrt(x); }
// 1/x: the hardware reciprocal (within 1 ulp) in single precision, a
// correctly rounded division in double precision.
__device__ inline float recip_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip_r(double x) { return 1.0 / x; }

// dx = f(x, u) for the 17-state (Newton-Euler with motor lag, z up).  DIST:
// include the body's episode disturbance (compile-time, so kernels without
// the training extras carry no extra arithmetic).
template <typename R, bool DIST = true>
__device__ inline void deriv(const Body<R>& B, R arm, R km, R g, const R x[NS], const R u[4],
                             R dx[NS]) {
  const R w0 = x[13], w1 = x[14], w2 = x[15], w3 = x[16];
  const R T0 = B.c0 + w0 * (B.c1 + B.c2 * w0);
  const R T1 = B.c0 + w1 * (B.c1 + B.c2 * w1);
  const R T2 = B.c0 + w2 * (B.c1 + B.c2 * w2);
  const R T3 = B.c0 + w3 * (B.c1 + B.c2 * w3);
  const R F = (T0 + T1) + (T2 + T3);
  const R tx = arm * ((T2 + T3) - (T0 + T1));
  const R ty = arm * ((T1 + T2) - (T0 + T3));
  const R tz = km * ((T1 + T3) - (T0 + T2));
  const R qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  // third column of R(q/|q|) times F/m: (2(xz+wy), 2(yz-wx), 1-2(x^2+y^2)) / |q|^2
  const R n2 = qw * qw + qx * qx + qy * qy + qz * qz;
  const R s = F * B.inv_m * recip_r(n2);
  dx[0] = x[7];
  dx[1] = x[8];
  dx[2] = x[9];
  const R ox = x[10], oy = x[11], oz = x[12];
  dx[3] = R(-0.5) * (qx * ox + qy * oy + qz * oz);
  dx[4] = R(0.5) * (qw * ox + qy * oz - qz * oy);
  dx[5] = R(0.5) * (qw * oy + qz * ox - qx * oz);
  dx[6] = R(0.5) * (qw * oz + qx * oy - qy * ox);
  const R ax = DIST ? B.ax : R(0), ay = DIST ? B.ay : R(0), az = DIST ? B.az : R(0);
  dx[7] = R(2) * (qx * qz + qw * qy) * s;
  dx[8] = R(2) * (qy * qz - qw * qx) * s;
  dx[9] = (n2 - R(2) * (qx * qx + qy * qy)) * s;
  if (DIST) {
    dx[7] += ax;
    dx[8] += ay;
    dx[9] += az;
  }
  dx[9] -= g;
  // Euler: J wdot = tau + tau_r - w x (J w)
  const R ttx = DIST ? tx + B.dtx : tx, tty = DIST ? ty + B.dty : ty,
          ttz = DIST ? tz + B.dtz : tz;
  dx[10] = (ttx - (B.Jz - B.Jy) * oy * oz) * B.inv_Jx;
  dx[11] = (tty - (B.Jx - B.Jz) * oz * ox) * B.inv_Jy;
  dx[12] = (ttz - (B.Jy - B.Jx) * ox * oy) * B.inv_Jz;
  dx[13] = (u[0] - w0) * B.inv_Tm;
  dx[14] = (u[1] - w1) * B.inv_Tm;
  dx[15] = (u[2] - w2) * B.inv_Tm;
  dx[16] = (u[3] - w3) * B.inv_Tm;
}

// One classical RK4 step, set points held.  Optional renormalisation of q.
template <typename R, bool DIST = true>
__device__ inline void rk4_step(const Body<R>& B, R arm, R km, R g, R h, bool renorm, R x[NS],
                                const R u[4]) {
  R k[NS], acc[NS], t[NS];
  deriv<R, DIST>(B, arm, km, g, x, u, k);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    acc[i] = k[i];
    t[i] = x[i] + R(0.5) * h * k[i];
  }
  deriv<R, DIST>(B, arm, km, g, t, u, k);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    acc[i] += R(2) * k[i];
    t[i] = x[i] + R(0.5) * h * k[i];
  }
  deriv<R, DIST>(B, arm, km, g, t, u, k);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    acc[i] += R(2) * k[i];
    t[i] = x[i] + h * k[i];
  }
  deriv<R, DIST>(B, arm, km, g, t, u, k);
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = x[i] + (h / R(6)) * (acc[i] + k[i]);
  // a select rather than a branch: multiplying by exactly 1 leaves q as it
  // is, and the state stays in the same registers on both sides
  const R rq = rsqrt_r(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
  const R r = renorm ? rq : R(1);
  x[3] *= r;
  x[4] *= r;
  x[5] *= r;
  x[6] *= r;
}

// Row-major rotation matrix of q/|q| (Hamilton, body to world).
__device__ inline void rotmat(const float q[4], float Rm[9]) {
  const float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const float s = 2.0f * recip_r(n2);
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  Rm[0] = 1.0f - s * (y * y + z * z);
  Rm[1] = s * (x * y - w * z);
  Rm[2] = s * (x * z + w * y);
  Rm[3] = s * (x * y + w * z);
  Rm[4] = 1.0f - s * (x * x + z * z);
  Rm[5] = s * (y * z - w * x);
  Rm[6] = s * (x * z - w * y);
  Rm[7] = s * (y * z + w * x);
  Rm[8] = 1.0f - s * (x * x + y * y);
}

__device__ inline float reward(const DevCfg& c, const float s[NS], const float a[NA]) {
  const float pp = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
  const float vv = s[7] * s[7] + s[8] * s[8] + s[9] * s[9];
  const float ww = s[10] * s[10] + s[11] * s[11] + s[12] * s[12];
  float aa = 0.0f;
#pragma unroll
  for (int i = 0; i < NA; ++i) aa += (a[i] - c.C_rab) * (a[i] - c.C_rab);
  return -c.C_rp * pp - c.C_rq * (1.0f - s[3] * s[3]) - c.C_rv * vv - c.C_rw * ww - c.C_ra * aa +
         c.C_rs;
}

// bit0: terminated (box or non-finite, if enabled); bit1: truncated.
__device__ inline uint32_t episode_end(const DevCfg& c, const float s[NS], int t_ep) {
  uint32_t term = 0;
  if (c.flags & F_TERMINATE) {
    bool out = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      out |= fabsf(s[i]) > c.pos_limit;
      out |= fabsf(s[7 + i]) > c.vel_limit;
    }
    // s*0 is NaN exactly when s is infinite or NaN, else a zero: the sum
    // stays zero only when every state value is finite
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < NS; ++i) z = fmaf(s[i], 0.0f, z);
    const bool finite = z == 0.0f;
    term = (out || !finite) ? 1u : 0u;
  }
  const uint32_t trunc = (!term && c.max_steps > 0 && t_ep >= c.max_steps) ? 2u : 0u;
  return term | trunc;
}

// Returns v unchanged but hides its value from the optimiser.  Loop bodies
// index SoA rows as row*N + opaque(e): the row part stays scalar and the
// per-lane part is one register, instead of the compiler hoisting one live
// 64-bit address per row out of the loop.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

// Stages weights into LDS: dst[i] = W[src] with src = index(i) (rounded to
// bf16 when bf16), or 0 where index(i) < 0, for i < n; the workgroup's
// threads stride over i, eight elements at a time: each thread issues its
// eight (unconditional, in-bounds) loads before it waits for the first,
// instead of one load and one wait per element.
template <typename Index>
__device__ inline void stage_lds(float* dst, int n, const float* __restrict__ W, Index index,
                                 bool bf16 = false) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int base = tid; base < n; base += 8 * nt) {
    float v[8];
    int src[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j * nt;
      src[j] = index(i < n ? i : n - 1);
      v[j] = W[src[j] >= 0 ? src[j] : 0];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j * nt;
      const float w = bf16 ? (float)(__bf16)v[j] : v[j];
      if (i < n) dst[i] = src[j] >= 0 ? w : 0.0f;
    }
  }
}

// Raw buffer view of a device span below 4 GiB: a load or store takes a
// 32-bit per-lane byte offset and a wave-uniform byte offset, so the per-row
// and per-step parts of an address stay in scalar registers and no 64-bit
// address is formed per access.
__device__ inline __amdgpu_buffer_rsrc_t span_rsrc(const float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
__device__ inline float bld1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline void bst1(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// tanh of the actor output without branches: tanh|x| = (1 - e) / (1 + e),
// e = exp(-2|x|), on the hardware exponential and reciprocal; absolute error
// about 2e-7 over the whole range.
__device__ inline float tanh_act(float x) {
  const float e = __expf(-2.0f * fabsf(x));
  const float t = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
  return copysignf(t, x);
}

// ReLU as a signed-integer maximum of the bit pattern: negative floats (and
// -0) are negative integers, so they become +0 and the rest pass through.
// One instruction; the float maximum would first quieten its operand.
__device__ __forceinline__ float relu_bits(float x) {
  return __int_as_float(max(__float_as_int(x), 0));
}

__device__ inline float action_to_rpm(const DevCfg& c, float a) {
  return c.rpm_min + (a + 1.0f) * c.rpm_half_range;
}


// ---------------------------------------------------------------------------
// Vector-Jacobian products (discrete adjoint) of the maps above, single
// precision.  Gradients with respect to the body parameters accumulate in
// gth = d/d(m, Jxx, Jyy, Jzz, c0, c1, c2, Tm).
// ---------------------------------------------------------------------------

// VJP of deriv() at (x, u) with cotangent gd of dx: accumulates gx, gu, gth.
__device__ inline void deriv_vjp(const Body<float>& B, const float th[NP], float arm, float km,
                                 const float x[NS], const float u[4], const float gd[NS],
                                 float gx[NS], float gu[4], float gth[NP]) {
  const float w[4] = {x[13], x[14], x[15], x[16]};
  float T[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) T[i] = B.c0 + w[i] * (B.c1 + B.c2 * w[i]);
  const float F = (T[0] + T[1]) + (T[2] + T[3]);
  const float tx = arm * ((T[2] + T[3]) - (T[0] + T[1]));
  const float ty = arm * ((T[1] + T[2]) - (T[0] + T[3]));
  const float tz = km * ((T[1] + T[3]) - (T[0] + T[2]));
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float ox = x[10], oy = x[11], oz = x[12];
  const float n2 = qw * qw + qx * qx + qy * qy + qz * qz;
  const float inv_n2 = recip_r(n2);
  const float sc = F * B.inv_m * inv_n2;
  // p' = v
  gx[7] += gd[0];
  gx[8] += gd[1];
  gx[9] += gd[2];
  // q' = 1/2 q (x) (0, w)
  const float g3 = gd[3], g4 = gd[4], g5 = gd[5], g6 = gd[6];
  gx[3] += 0.5f * (g4 * ox + g5 * oy + g6 * oz);
  gx[4] += 0.5f * (-g3 * ox - g5 * oz + g6 * oy);
  gx[5] += 0.5f * (-g3 * oy + g4 * oz - g6 * ox);
  gx[6] += 0.5f * (-g3 * oz - g4 * oy + g5 * ox);
  gx[10] += 0.5f * (-g3 * qx + g4 * qw + g5 * qz - g6 * qy);
  gx[11] += 0.5f * (-g3 * qy - g4 * qz + g5 * qw + g6 * qx);
  gx[12] += 0.5f * (-g3 * qz + g4 * qy - g5 * qx + g6 * qw);
  // v' = sc * P(q) - g e_z,  P = (2(xz+wy), 2(yz-wx), |q|^2 - 2(x^2+y^2))
  const float g7 = gd[7], g8 = gd[8], g9 = gd[9];
  const float P0 = 2.0f * (qx * qz + qw * qy), P1 = 2.0f * (qy * qz - qw * qx),
              P2 = n2 - 2.0f * (qx * qx + qy * qy);
  const float gsc = g7 * P0 + g8 * P1 + g9 * P2;
  const float k2 = 2.0f * gsc * sc * inv_n2;  // from sc's 1/|q|^2
  gx[3] += 2.0f * sc * (g7 * qy - g8 * qx + g9 * qw) - k2 * qw;
  gx[4] += 2.0f * sc * (g7 * qz - g8 * qw - g9 * qx) - k2 * qx;
  gx[5] += 2.0f * sc * (g7 * qw + g8 * qz - g9 * qy) - k2 * qy;
  gx[6] += 2.0f * sc * (g7 * qx + g8 * qy + g9 * qz) - k2 * qz;
  const float gF = gsc * B.inv_m * inv_n2;
  gth[0] += -(gsc * sc + g7 * B.ax + g8 * B.ay + g9 * B.az) * B.inv_m;
  // w' = J^-1 (tau - w x J w)
  const float hx = gd[10] * B.inv_Jx, hy = gd[11] * B.inv_Jy, hz = gd[12] * B.inv_Jz;
  const float dwx = (tx + B.dtx - (B.Jz - B.Jy) * oy * oz) * B.inv_Jx;
  const float dwy = (ty + B.dty - (B.Jx - B.Jz) * oz * ox) * B.inv_Jy;
  const float dwz = (tz + B.dtz - (B.Jy - B.Jx) * ox * oy) * B.inv_Jz;
  gth[1] += -hx * dwx;
  gth[2] += -hy * dwy;
  gth[3] += -hz * dwz;
  gx[11] += -hx * (B.Jz - B.Jy) * oz;
  gx[12] += -hx * (B.Jz - B.Jy) * oy;
  gth[3] += -hx * oy * oz;
  gth[2] += hx * oy * oz;
  gx[12] += -hy * (B.Jx - B.Jz) * ox;
  gx[10] += -hy * (B.Jx - B.Jz) * oz;
  gth[1] += -hy * oz * ox;
  gth[3] += hy * oz * ox;
  gx[10] += -hz * (B.Jy - B.Jx) * oy;
  gx[11] += -hz * (B.Jy - B.Jx) * ox;
  gth[2] += -hz * ox * oy;
  gth[1] += hz * ox * oy;
  // torques and collective thrust -> rotor thrusts
  float gT[4];
  gT[0] = gF - arm * (hx + hy) - km * hz;
  gT[1] = gF - arm * hx + arm * hy + km * hz;
  gT[2] = gF + arm * (hx + hy) - km * hz;
  gT[3] = gF + arm * hx - arm * hy + km * hz;
  // thrust curve T = c0 + c1 w + c2 w^2, motor lag w' = (u - w) / Tm
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gth[4] += gT[i];
    gth[5] += gT[i] * w[i];
    gth[6] += gT[i] * w[i] * w[i];
    const float gm = gd[13 + i];
    gx[13 + i] += gT[i] * (B.c1 + 2.0f * B.c2 * w[i]) - gm * B.inv_Tm;
    gu[i] += gm * B.inv_Tm;
    gth[7] += -gm * (u[i] - w[i]) * B.inv_Tm * B.inv_Tm;
  }
  (void)th;
}

// VJP of rotmat(q) (R of q/|q|, row-major) with cotangent G: accumulates gq.
__device__ inline void rotmat_vjp(const float q[4], const float G[9], float gq[4]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  const float n2 = w * w + x * x + y * y + z * z;
  const float inv_n2 = recip_r(n2);
  const float s = 2.0f * inv_n2;
  const float dw = -z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7];
  const float dx = y * G[1] + z * G[2] + y * G[3] - 2.0f * x * G[4] - w * G[5] + z * G[6] +
                   w * G[7] - 2.0f * x * G[8];
  const float dy = -2.0f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] +
                   z * G[7] - 2.0f * y * G[8];
  const float dz = -2.0f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0f * z * G[4] +
                   y * G[5] + x * G[6] + y * G[7];
  const float GP = -(y * y + z * z) * G[0] + (x * y - w * z) * G[1] + (x * z + w * y) * G[2] +
                   (x * y + w * z) * G[3] - (x * x + z * z) * G[4] + (y * z - w * x) * G[5] +
                   (x * z - w * y) * G[6] + (y * z + w * x) * G[7] - (x * x + y * y) * G[8];
  const float k = 2.0f * s * GP * inv_n2;
  gq[0] += s * dw - k * w;
  gq[1] += s * dx - k * x;
  gq[2] += s * dy - k * y;
  gq[3] += s * dz - k * z;
}

}  // namespace qs
