/*
 * FP64 CPU oracle for the batched quadrotor environment step.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * GPU library is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. The GPU library never includes,
 * links or calls anything here, and nothing here includes a GPU header.
 *
 * What it computes follows "Learning to Fly in Seconds" (Eschmann, Albani,
 * Loianno, IEEE RA-L 2024), Sec. IV (Methodology):
 *   - state s = {p, q, v, w, w_m}, 17 values, quaternion attitude (w,x,y,z);
 *   - rigid-body quadrotor dynamics with first-order motor lag (Sec. IV and the
 *     taxonomy of Sec. II, levels 2.1 mass, 3.1 rotational kinematics,
 *     4.1 inertia, 4.2 geometry, 4.3 thrust curve, 5.1 motor delay);
 *   - actor observation {p, R(q), v, w, H} of size 18 + 4 N_H (Sec. IV);
 *   - actions = RPM setpoints (Sec. IV);
 *   - reward = negative squared cost plus survival constant (Sec. IV, reward
 *     equation);
 *   - termination when leaving a box around the origin (Sec. V, Training);
 *   - the training extras of the asymmetric actor-critic paragraph (Sec. IV):
 *     a random force and torque disturbance drawn per episode, additive noise
 *     on the actor's observation, and the 28-value critic observation
 *     {p, R, v, w, w_m, f_r, tau_r}.
 * The integrator is classical 4-stage Runge-Kutta at 100 Hz (Sec. V,
 * Simulation, gives the 100 Hz rate).  Every choice the paper leaves open
 * (constants, rotor layout, reset distribution, RNG) is a stated reading; the
 * values arrive in the config struct.
 *
 * Everything is evaluated in double precision except two decisions that map
 * floating point to an integer: the termination box test is taken in single
 * precision (the kernel's precision), and the counter RNG produces 23-bit
 * uniforms that are exact in both precisions.
 *
 * The adjoint below is a hand-derived discrete adjoint of exactly this
 * forward map (the RK4 stages, the quaternion normalisation inside R and after
 * the step, the action map and the MLP with ReLU subgradient 0 at 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define NS 17     /* state size, Sec. IV                                   */
#define NH 32     /* action history length N_H                              */
#define NA 4      /* actions: 4 RPM setpoints, Sec. IV                      */
#define NO 146    /* actor observation 18 + 4*32, Sec. IV                   */
#define NHID 64   /* hidden width of the 146-64-64-4 actor                  */
#define NP 8      /* dynamics parameters m, Jxx, Jyy, Jzz, c0, c1, c2, T_m  */
#define NW 13828  /* actor parameter count                                  */

/* Flat actor layout: torch.nn.Linear weight [out][in] and bias, concatenated. */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NHID * NO)
#define OFF_W2 (OFF_B1 + NHID)
#define OFF_B2 (OFF_W2 + NHID * NHID)
#define OFF_W3 (OFF_B2 + NHID)
#define OFF_B3 (OFF_W3 + NA * NHID)

#define F_TERMINATE 1
#define F_AUTORESET 2
#define F_RENORM_Q 4
#define F_DISTURB 32
#define F_OBS_NOISE 64

/* Mirrors the config the Python side builds; own definition, no shared header. */
typedef struct {
  double dt, g, arm, k_m, rpm_min, rpm_max;
  double nominal[NP], dr_lo[NP], dr_hi[NP];
  double pos_limit, vel_limit;
  double init_pos, init_angle, init_vel, init_angvel;
  double C_rp, C_rq, C_rv, C_rw, C_ra, C_rab, C_rs;
  int32_t max_episode_steps, flags, dr_enable, pad_;
  uint64_t seed, dr_seed;
  double dist_force, dist_torque; /* per-component bounds of the episode disturbance */
  double obs_noise[4];            /* noise std on p, R entries, v, w of the actor observation */
} orc_cfg;

/* ------------------------------------------------------------------------- */
/* Counter-based RNG: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;  /* Weyl key schedule */
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four uniforms in (0,1): counter (env, episode, block, stream), key = seed.
 * u = (2k+1) 2^-24 with k the top 23 bits, exact in float and double. */
static void uniforms4(uint64_t seed, uint32_t env, uint32_t episode, uint32_t block,
                      uint32_t stream, double u[4]) {
  uint32_t ctr[4] = {env, episode, block, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  for (int i = 0; i < 4; ++i) u[i] = ((double)(x[i] >> 9) + 0.5) * (1.0 / 8388608.0);
}

void orc_uniforms(uint64_t seed, uint32_t env, uint32_t episode, uint32_t block, uint32_t stream,
                  double* u4) {
  uniforms4(seed, env, episode, block, stream, u4);
}

enum { STREAM_RESET = 0, STREAM_DR = 1, STREAM_DIST = 2, STREAM_NOISE = 3 };

/* Episode disturbance (Sec. IV, asymmetric actor-critic paragraph: a random
 * force and torque drawn at the start of every episode).  Reading: the force
 * acts in the world frame and the torque in the body frame, each component
 * uniform in [-F, F] and [-T, T]; the draw is keyed by (env, episode), so it
 * holds for the whole episode.  d = {f_r, tau_r}; zero with the flag off. */
static void disturbance(const orc_cfg* c, uint32_t env, uint32_t episode, double d[6]) {
  if (!(c->flags & F_DISTURB)) {
    for (int i = 0; i < 6; ++i) d[i] = 0.0;
    return;
  }
  double u[8];
  uniforms4(c->seed, env, episode, 0, STREAM_DIST, u);
  uniforms4(c->seed, env, episode, 1, STREAM_DIST, u + 4);
  for (int i = 0; i < 3; ++i) {
    d[i] = c->dist_force * (2.0 * u[i] - 1.0);
    d[3 + i] = c->dist_torque * (2.0 * u[3 + i] - 1.0);
  }
}

/* 18 standard normal draws for the observation of step t_ep of an episode:
 * Box-Muller (Box and Muller, 1958) on consecutive uniform pairs,
 * z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2). */
static void normals18(const orc_cfg* c, uint32_t env, uint32_t episode, int32_t t_ep,
                      double z[18]) {
  double u[20];
  for (int b = 0; b < 5; ++b)
    uniforms4(c->seed, env, episode, (uint32_t)t_ep * 5u + (uint32_t)b, STREAM_NOISE, u + 4 * b);
  for (int i = 0; i < 9; ++i) {
    double r = sqrt(-2.0 * log(u[2 * i]));
    z[2 * i] = r * cos(2.0 * M_PI * u[2 * i + 1]);
    z[2 * i + 1] = r * sin(2.0 * M_PI * u[2 * i + 1]);
  }
}

/* Sensor noise on the actor observation (Sec. IV; the scales are in the
 * missing parameter sheet, so they are configuration): o_i += sigma_g z_i on
 * the 18 state features, groups p, R, v, w; the action history is the agent's
 * own output and stays clean. */
static void add_obs_noise(const orc_cfg* c, uint32_t env, uint32_t episode, int32_t t_ep,
                          double o[NO]) {
  if (!(c->flags & F_OBS_NOISE)) return;
  double z[18];
  normals18(c, env, episode, t_ep, z);
  for (int i = 0; i < 18; ++i) {
    const int g = i < 3 ? 0 : i < 12 ? 1 : i < 15 ? 2 : 3;
    o[i] += c->obs_noise[g] * z[i];
  }
}

/* ------------------------------------------------------------------------- */
/* Parameters, hover point, reset distribution                               */
/* ------------------------------------------------------------------------- */

/* Per-env dynamics parameters: nominal values times independent uniform factors
 * (domain randomisation), fixed for the life of the env. */
static void env_params(const orc_cfg* c, uint32_t env, double th[NP]) {
  double u[8];
  uniforms4(c->dr_seed, env, 0, 0, STREAM_DR, u);
  uniforms4(c->dr_seed, env, 0, 1, STREAM_DR, u + 4);
  for (int i = 0; i < NP; ++i) {
    double f = c->dr_enable ? c->dr_lo[i] + (c->dr_hi[i] - c->dr_lo[i]) * u[i] : 1.0;
    th[i] = c->nominal[i] * f;
  }
}

/* Rotor speed at which the four rotors together carry the weight:
 * the positive root of c2 w^2 + c1 w + c0 = m g / 4. */
double orc_hover_rpm(const orc_cfg* c, const double th[NP]) {
  double need = th[0] * c->g / 4.0 - th[4];
  double c1 = th[5], c2 = th[6];
  if (c2 == 0.0) return need / c1;
  return (-c1 + sqrt(c1 * c1 + 4.0 * c2 * need)) / (2.0 * c2);
}

static double rpm_to_action(const orc_cfg* c, double w) {
  return 2.0 * (w - c->rpm_min) / (c->rpm_max - c->rpm_min) - 1.0;
}

/* Initial-state distribution (Sec. IV asks for diverse positions, attitudes,
 * velocities, angular velocities).  Reading: p ~ U(-P,P)^3; attitude = rotation
 * by angle U(0, A) about an axis uniform on the sphere; v ~ U(-V,V)^3;
 * w ~ U(-W,W)^3; rotors at hover; history filled with the hover action. */
static void reset_env(const orc_cfg* c, const double th[NP], uint32_t env, uint32_t episode,
                      double s[NS], double H[NH * NA]) {
  double u[12];
  uniforms4(c->seed, env, episode, 0, STREAM_RESET, u);
  uniforms4(c->seed, env, episode, 1, STREAM_RESET, u + 4);
  uniforms4(c->seed, env, episode, 2, STREAM_RESET, u + 8);
  for (int i = 0; i < 3; ++i) s[i] = c->init_pos * (2.0 * u[i] - 1.0);
  double z = 2.0 * u[3] - 1.0;
  double phi = 2.0 * M_PI * u[4];
  double alpha = c->init_angle * u[5];
  double r = sqrt(fmax(0.0, 1.0 - z * z));
  double sa = sin(0.5 * alpha);
  s[3] = cos(0.5 * alpha);
  s[4] = sa * r * cos(phi);
  s[5] = sa * r * sin(phi);
  s[6] = sa * z;
  for (int i = 0; i < 3; ++i) s[7 + i] = c->init_vel * (2.0 * u[6 + i] - 1.0);
  for (int i = 0; i < 3; ++i) s[10 + i] = c->init_angvel * (2.0 * u[9 + i] - 1.0);
  double wh = orc_hover_rpm(c, th);
  for (int i = 0; i < 4; ++i) s[13 + i] = wh;
  double ah = rpm_to_action(c, wh);
  for (int i = 0; i < NH * NA; ++i) H[i] = ah;
}

/* ------------------------------------------------------------------------- */
/* Dynamics f(x, u; theta)                                                    */
/* ------------------------------------------------------------------------- */

/* Rotor layout (reading of the vehicle geometry): rotor i sits at
 * (sx_i * l, sy_i * l, 0) in the body frame and spins with sign d_i. */
static const double RSX[4] = {+1, -1, -1, +1};
static const double RSY[4] = {-1, -1, +1, +1};
static const double RD[4] = {-1, +1, -1, +1};

/* Rotation matrix of the unit quaternion (w,x,y,z), Hamilton convention,
 * body to world, row-major. */
static void rotmat(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void normalize4(const double q[4], double out[4]) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) out[i] = q[i] / n;
}

/* Time derivative of the 17-state.  u = RPM setpoints held over the step;
 * d = episode disturbance {f_r (world), tau_r (body)} or NULL. */
static void dynamics(const orc_cfg* c, const double th[NP], const double x[NS], const double u[4],
                     const double* d, double dx[NS]) {
  const double m = th[0], J[3] = {th[1], th[2], th[3]}, c0 = th[4], c1 = th[5], c2 = th[6],
               Tm = th[7];
  const double* q = x + 3;
  const double* v = x + 7;
  const double* w = x + 10;
  const double* wm = x + 13;
  double T[4], F = 0.0;
  for (int i = 0; i < 4; ++i) {
    T[i] = c0 + c1 * wm[i] + c2 * wm[i] * wm[i];
    F += T[i];
  }
  double tau[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i) {
    tau[0] += c->arm * RSY[i] * T[i];
    tau[1] += -c->arm * RSX[i] * T[i];
    tau[2] += c->k_m * RD[i] * T[i];
  }
  double qn[4], R[9];
  normalize4(q, qn);
  rotmat(qn, R);
  /* position */
  for (int i = 0; i < 3; ++i) dx[i] = v[i];
  /* attitude: qdot = 1/2 q (x) (0, w), w in the body frame */
  dx[3] = 0.5 * (-q[1] * w[0] - q[2] * w[1] - q[3] * w[2]);
  dx[4] = 0.5 * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);
  dx[5] = 0.5 * (q[0] * w[1] + q[3] * w[0] - q[1] * w[2]);
  dx[6] = 0.5 * (q[0] * w[2] + q[1] * w[1] - q[2] * w[0]);
  /* linear velocity: rotated body thrust and disturbance force over mass,
   * plus gravity (z up) */
  for (int i = 0; i < 3; ++i) dx[7 + i] = (R[3 * i + 2] * F + (d ? d[i] : 0.0)) / m;
  dx[9] -= c->g;
  /* angular velocity: Euler's equation J wdot = tau - w x (J w) */
  double Jw[3] = {J[0] * w[0], J[1] * w[1], J[2] * w[2]};
  double cr[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],
                  w[0] * Jw[1] - w[1] * Jw[0]};
  for (int i = 0; i < 3; ++i) dx[10 + i] = (tau[i] + (d ? d[3 + i] : 0.0) - cr[i]) / J[i];
  /* motors: first-order low-pass towards the setpoint */
  for (int i = 0; i < 4; ++i) dx[13 + i] = (u[i] - wm[i]) / Tm;
}

/* One classical RK4 step with the setpoint held (zero-order hold). */
static void rk4(const orc_cfg* c, const double th[NP], const double x[NS], const double u[4],
                const double* d, double xn[NS]) {
  const double h = c->dt;
  double k1[NS], k2[NS], k3[NS], k4[NS], t[NS];
  dynamics(c, th, x, u, d, k1);
  for (int i = 0; i < NS; ++i) t[i] = x[i] + 0.5 * h * k1[i];
  dynamics(c, th, t, u, d, k2);
  for (int i = 0; i < NS; ++i) t[i] = x[i] + 0.5 * h * k2[i];
  dynamics(c, th, t, u, d, k3);
  for (int i = 0; i < NS; ++i) t[i] = x[i] + h * k3[i];
  dynamics(c, th, t, u, d, k4);
  for (int i = 0; i < NS; ++i) xn[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* ------------------------------------------------------------------------- */
/* Observation, actor, action map, reward                                    */
/* ------------------------------------------------------------------------- */

/* o = {p, R(q) row-major, v, w, H oldest..newest}; 18 + 128 = 146. */
static void observe(const double s[NS], const double H[NH * NA], double o[NO]) {
  double qn[4], R[9];
  normalize4(s + 3, qn);
  rotmat(qn, R);
  for (int i = 0; i < 3; ++i) o[i] = s[i];
  for (int i = 0; i < 9; ++i) o[3 + i] = R[i];
  for (int i = 0; i < 3; ++i) o[12 + i] = s[7 + i];
  for (int i = 0; i < 3; ++i) o[15 + i] = s[10 + i];
  for (int i = 0; i < NH * NA; ++i) o[18 + i] = H[i];
}

/* a = tanh(W3 relu(W2 relu(W1 o + b1) + b2) + b3).  Pre-activations kept for
 * the adjoint when z1/z2/z3 are non-NULL. */
static void actor(const double* W, const double o[NO], double a[NA], double* z1o, double* z2o,
                  double* z3o) {
  double z1[NHID], h1[NHID], z2[NHID], h2[NHID], z3[NA];
  for (int n = 0; n < NHID; ++n) {
    double acc = W[OFF_B1 + n];
    for (int k = 0; k < NO; ++k) acc += W[OFF_W1 + n * NO + k] * o[k];
    z1[n] = acc;
    h1[n] = acc > 0.0 ? acc : 0.0;
  }
  for (int n = 0; n < NHID; ++n) {
    double acc = W[OFF_B2 + n];
    for (int k = 0; k < NHID; ++k) acc += W[OFF_W2 + n * NHID + k] * h1[k];
    z2[n] = acc;
    h2[n] = acc > 0.0 ? acc : 0.0;
  }
  for (int n = 0; n < NA; ++n) {
    double acc = W[OFF_B3 + n];
    for (int k = 0; k < NHID; ++k) acc += W[OFF_W3 + n * NHID + k] * h2[k];
    z3[n] = acc;
    a[n] = tanh(acc);
  }
  if (z1o) memcpy(z1o, z1, sizeof z1);
  if (z2o) memcpy(z2o, z2, sizeof z2);
  if (z3o) memcpy(z3o, z3, sizeof z3);
}

/* Normalised action in [-1,1] to RPM setpoint. */
static void action_to_rpm(const orc_cfg* c, const double a[NA], double u[NA]) {
  for (int i = 0; i < NA; ++i) u[i] = c->rpm_min + 0.5 * (a[i] + 1.0) * (c->rpm_max - c->rpm_min);
}

/* r = -Crp|p|^2 - Crq(1 - qw^2) - Crv|v|^2 - Crw|w|^2 - Cra|a - Crab|^2 + Crs,
 * evaluated on the post-step state and the normalised action (Sec. IV). */
static double reward(const orc_cfg* c, const double s[NS], const double a[NA]) {
  double pp = 0, vv = 0, ww = 0, aa = 0;
  for (int i = 0; i < 3; ++i) {
    pp += s[i] * s[i];
    vv += s[7 + i] * s[7 + i];
    ww += s[10 + i] * s[10 + i];
  }
  for (int i = 0; i < NA; ++i) aa += (a[i] - c->C_rab) * (a[i] - c->C_rab);
  return -c->C_rp * pp - c->C_rq * (1.0 - s[3] * s[3]) - c->C_rv * vv - c->C_rw * ww -
         c->C_ra * aa + c->C_rs;
}

/* ------------------------------------------------------------------------- */
/* One environment step                                                       */
/* ------------------------------------------------------------------------- */

/* Advances one env: observation, actor (or the given action), RK4, optional
 * quaternion renormalisation, reward, history push, episode bookkeeping and,
 * when the episode ended and auto-reset is on, the reset.  The reward and done
 * flags returned belong to the transition; the state left behind is the reset
 * state when a reset happened.  done: bit0 terminated, bit1 truncated. */
static void env_step(const orc_cfg* c, const double* W, const double* a_ext, const double th[NP],
                     uint32_t env, double s[NS], double H[NH * NA], int32_t* t_ep, int32_t* ep,
                     double* r_out, uint8_t* done_out, double* a_out) {
  double o[NO], a[NA], u[NA], sn[NS], d[6];
  disturbance(c, env, (uint32_t)*ep, d);
  if (a_ext) {
    memcpy(a, a_ext, sizeof a);
  } else {
    observe(s, H, o);
    add_obs_noise(c, env, (uint32_t)*ep, *t_ep, o);
    actor(W, o, a, NULL, NULL, NULL);
  }
  action_to_rpm(c, a, u);
  rk4(c, th, s, u, d, sn);
  if (c->flags & F_RENORM_Q) {
    double qn[4];
    normalize4(sn + 3, qn);
    memcpy(sn + 3, qn, sizeof qn);
  }
  double r = reward(c, sn, a);
  memmove(H, H + NA, sizeof(double) * (NH - 1) * NA);
  memcpy(H + (NH - 1) * NA, a, sizeof a);
  *t_ep += 1;
  int term = 0;
  if (c->flags & F_TERMINATE) {
    const float pl = (float)c->pos_limit, vl = (float)c->vel_limit;
    for (int i = 0; i < 3; ++i) {
      if (fabsf((float)sn[i]) > pl) term = 1;
      if (fabsf((float)sn[7 + i]) > vl) term = 1;
    }
    for (int i = 0; i < NS; ++i)
      if (!isfinite(sn[i])) term = 1;
  }
  int trunc = !term && c->max_episode_steps > 0 && *t_ep >= c->max_episode_steps;
  memcpy(s, sn, sizeof sn);
  if ((term || trunc) && (c->flags & F_AUTORESET)) {
    *ep += 1;
    *t_ep = 0;
    reset_env(c, th, env, (uint32_t)*ep, s, H);
  }
  if (r_out) *r_out = r;
  if (done_out) *done_out = (uint8_t)(term | (trunc << 1));
  if (a_out) memcpy(a_out, a, sizeof a);
}

/* ------------------------------------------------------------------------- */
/* Exported batch API (AoS layouts: s[n][17], H[n][32][4], theta[n][8])       */
/* ------------------------------------------------------------------------- */

static uint32_t env_id(const uint32_t* ids, int i) { return ids ? ids[i] : (uint32_t)i; }

/* Per-env parameters and episode-0 reset for n envs (env ids default 0..n-1). */
void orc_init(const orc_cfg* c, int n, const uint32_t* ids, double* theta, double* s, double* H,
              int32_t* t_ep, int32_t* ep) {
  for (int i = 0; i < n; ++i) {
    uint32_t e = env_id(ids, i);
    env_params(c, e, theta + (size_t)i * NP);
    reset_env(c, theta + (size_t)i * NP, e, 0, s + (size_t)i * NS, H + (size_t)i * NH * NA);
    t_ep[i] = 0;
    ep[i] = 0;
  }
}

void orc_env_params(const orc_cfg* c, int n, const uint32_t* ids, double* theta) {
  for (int i = 0; i < n; ++i) env_params(c, env_id(ids, i), theta + (size_t)i * NP);
}

void orc_reset_state(const orc_cfg* c, int n, const uint32_t* ids, const int32_t* episode,
                     const double* theta, double* s, double* H) {
  for (int i = 0; i < n; ++i)
    reset_env(c, theta + (size_t)i * NP, env_id(ids, i), (uint32_t)episode[i],
              s + (size_t)i * NS, H + (size_t)i * NH * NA);
}

void orc_dynamics(const orc_cfg* c, const double* th, const double* x, const double* u,
                  const double* d, double* dx) {
  dynamics(c, th, x, u, d, dx);
}

void orc_rk4(const orc_cfg* c, const double* th, const double* x, const double* u,
             const double* d, double* xn) {
  rk4(c, th, x, u, d, xn);
}

void orc_observe(const double* s, const double* H, double* o) { observe(s, H, o); }

void orc_disturbance(const orc_cfg* c, uint32_t env, uint32_t episode, double* d) {
  disturbance(c, env, episode, d);
}

void orc_normals18(const orc_cfg* c, uint32_t env, uint32_t episode, int32_t t_ep, double* z) {
  normals18(c, env, episode, t_ep, z);
}

/* Actor observation of an env at step t_ep of its episode: o with noise. */
void orc_observe_noisy(const orc_cfg* c, uint32_t env, uint32_t episode, int32_t t_ep,
                       const double* s, const double* H, double* o) {
  observe(s, H, o);
  add_obs_noise(c, env, episode, t_ep, o);
}

/* Critic observation (Sec. IV): {p, R(q) row-major, v, w, w_m, f_r, tau_r},
 * 3 + 9 + 3 + 3 + 4 + 3 + 3 = 28, ground truth (no noise). */
void orc_critic_obs(const orc_cfg* c, uint32_t env, uint32_t episode, const double* s,
                    double* oc) {
  double qn[4], R[9], d[6];
  normalize4(s + 3, qn);
  rotmat(qn, R);
  disturbance(c, env, episode, d);
  for (int i = 0; i < 3; ++i) oc[i] = s[i];
  for (int i = 0; i < 9; ++i) oc[3 + i] = R[i];
  for (int i = 0; i < 3; ++i) oc[12 + i] = s[7 + i];
  for (int i = 0; i < 3; ++i) oc[15 + i] = s[10 + i];
  for (int i = 0; i < 4; ++i) oc[18 + i] = s[13 + i];
  for (int i = 0; i < 6; ++i) oc[22 + i] = d[i];
}

void orc_actor(const double* W, const double* o, double* a) { actor(W, o, a, NULL, NULL, NULL); }

void orc_rotmat(const double* q, double* R) {
  double qn[4];
  normalize4(q, qn);
  rotmat(qn, R);
}

double orc_reward(const orc_cfg* c, const double* s, const double* a) { return reward(c, s, a); }

typedef struct {
  const orc_cfg* c;
  const uint32_t* ids;
  const double* W;
  const double* actions;
  int n, T, i0, i1;
  double *s, *H, *theta, *rewards, *states, *acts;
  int32_t *t_ep, *ep;
  uint8_t* dones;
} roll_job;

static void* roll_worker(void* arg) {
  roll_job* j = (roll_job*)arg;
  for (int i = j->i0; i < j->i1; ++i) {
    uint32_t e = env_id(j->ids, i);
    double* s = j->s + (size_t)i * NS;
    double* H = j->H + (size_t)i * NH * NA;
    if (j->states) memcpy(j->states + (size_t)i * NS, s, sizeof(double) * NS);
    for (int t = 0; t < j->T; ++t) {
      const double* ax = j->actions ? j->actions + ((size_t)t * j->n + i) * NA : NULL;
      double r;
      uint8_t d;
      double a[NA];
      env_step(j->c, j->W, ax, j->theta + (size_t)i * NP, e, s, H, j->t_ep + i, j->ep + i, &r, &d,
               a);
      if (j->rewards) j->rewards[(size_t)t * j->n + i] = r;
      if (j->dones) j->dones[(size_t)t * j->n + i] = d;
      if (j->acts) memcpy(j->acts + ((size_t)t * j->n + i) * NA, a, sizeof a);
      if (j->states) memcpy(j->states + ((size_t)(t + 1) * j->n + i) * NS, s, sizeof(double) * NS);
    }
  }
  return NULL;
}

/* T steps for n envs.  W (actor, 13828 values) is used unless actions
 * ([T][n][4]) is given.  Outputs are optional: rewards [T][n], dones [T][n],
 * states [T+1][n][17] (states[0] = start state), acts [T][n][4].  Envs are
 * independent; nthreads > 1 splits them over POSIX threads. */
void orc_rollout(const orc_cfg* c, int n, const uint32_t* ids, const double* W,
                 const double* actions, int T, double* s, double* H, int32_t* t_ep, int32_t* ep,
                 const double* theta, double* rewards, uint8_t* dones, double* states, double* acts,
                 int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n) nthreads = n > 0 ? n : 1;
  roll_job jobs[256];
  pthread_t th[256];
  if (nthreads > 256) nthreads = 256;
  for (int k = 0; k < nthreads; ++k) {
    roll_job j = {c, ids, W, actions, n, T, (int)((long)n * k / nthreads),
                  (int)((long)n * (k + 1) / nthreads), s, H, (double*)theta, rewards, states, acts,
                  t_ep, ep, dones};
    jobs[k] = j;
  }
  if (nthreads == 1) {
    roll_worker(&jobs[0]);
    return;
  }
  for (int k = 0; k < nthreads; ++k) pthread_create(&th[k], NULL, roll_worker, &jobs[k]);
  for (int k = 0; k < nthreads; ++k) pthread_join(th[k], NULL);
}

/* ========================================================================= */
/* Discrete adjoint (differentiable mode: no termination, no reset)           */
/* ========================================================================= */

/* Back-propagates the cotangent g of q_hat = q/|q| to q. */
static void normalize4_vjp(const double q[4], const double gqn[4], double gq[4]) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double qn[4], d = 0.0;
  for (int i = 0; i < 4; ++i) qn[i] = q[i] / n;
  for (int i = 0; i < 4; ++i) d += qn[i] * gqn[i];
  for (int i = 0; i < 4; ++i) gq[i] += (gqn[i] - qn[i] * d) / n;
}

/* Cotangent of R (row-major, from the unit quaternion qn) to qn. */
static void rotmat_vjp(const double qn[4], const double G[9], double gqn[4]) {
  double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  gqn[0] = 2 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  gqn[1] = 2 * (y * G[1] + z * G[2] + y * G[3] - 2 * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                2 * x * G[8]);
  gqn[2] = 2 * (-2 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                2 * y * G[8]);
  gqn[3] = 2 * (-2 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2 * z * G[4] + y * G[5] +
                x * G[6] + y * G[7]);
}

/* VJP of f at (x, u, theta) with cotangent gd (17): accumulates into gx (17),
 * gu (4) and gth (8). */
static void dynamics_vjp(const orc_cfg* c, const double th[NP], const double x[NS],
                         const double u[4], const double* d, const double gd[NS], double gx[NS],
                         double gu[4], double gth[NP]) {
  const double m = th[0], J[3] = {th[1], th[2], th[3]}, c0 = th[4], c1 = th[5], c2 = th[6],
               Tm = th[7];
  const double* q = x + 3;
  const double* w = x + 10;
  const double* wm = x + 13;
  double T[4], F = 0.0;
  for (int i = 0; i < 4; ++i) {
    T[i] = c0 + c1 * wm[i] + c2 * wm[i] * wm[i];
    F += T[i];
  }
  double tau[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i) {
    tau[0] += c->arm * RSY[i] * T[i];
    tau[1] += -c->arm * RSX[i] * T[i];
    tau[2] += c->k_m * RD[i] * T[i];
  }
  double qn[4], R[9];
  normalize4(q, qn);
  rotmat(qn, R);
  const double* gp = gd;
  const double* gq = gd + 3;
  const double* gv = gd + 7;
  const double* gw = gd + 10;
  const double* gm = gd + 13;
  double gT[4] = {0, 0, 0, 0};

  /* pdot = v */
  for (int i = 0; i < 3; ++i) gx[7 + i] += gp[i];

  /* vdot = R[:,2] F / m - g e_z */
  double G[9] = {0};
  double gF = 0.0;
  for (int i = 0; i < 3; ++i) {
    G[3 * i + 2] = gv[i] * F / m;
    gF += gv[i] * R[3 * i + 2] / m;
    gth[0] += -gv[i] * (R[3 * i + 2] * F + (d ? d[i] : 0.0)) / (m * m);
  }
  double gqn[4];
  rotmat_vjp(qn, G, gqn);
  normalize4_vjp(q, gqn, gx + 3);

  /* qdot = 1/2 q (x) (0, w) */
  gx[3] += 0.5 * (gq[1] * w[0] + gq[2] * w[1] + gq[3] * w[2]);
  gx[4] += 0.5 * (-gq[0] * w[0] - gq[2] * w[2] + gq[3] * w[1]);
  gx[5] += 0.5 * (-gq[0] * w[1] + gq[1] * w[2] - gq[3] * w[0]);
  gx[6] += 0.5 * (-gq[0] * w[2] - gq[1] * w[1] + gq[2] * w[0]);
  gx[10] += 0.5 * (-gq[0] * q[1] + gq[1] * q[0] + gq[2] * q[3] - gq[3] * q[2]);
  gx[11] += 0.5 * (-gq[0] * q[2] - gq[1] * q[3] + gq[2] * q[0] + gq[3] * q[1]);
  gx[12] += 0.5 * (-gq[0] * q[3] + gq[1] * q[2] - gq[2] * q[1] + gq[3] * q[0]);

  /* wdot_i = (tau_i - cr_i) / J_i,  cr = w x (J w) */
  double Jw[3] = {J[0] * w[0], J[1] * w[1], J[2] * w[2]};
  double cr[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],
                  w[0] * Jw[1] - w[1] * Jw[0]};
  double hq[3], gtau[3];
  for (int i = 0; i < 3; ++i) {
    hq[i] = gw[i] / J[i];
    gtau[i] = hq[i];
    gth[1 + i] += -gw[i] * (tau[i] + (d ? d[3 + i] : 0.0) - cr[i]) / (J[i] * J[i]);
  }
  /* cr_x = (Jz - Jy) wy wz, cr_y = (Jx - Jz) wz wx, cr_z = (Jy - Jx) wx wy */
  gx[11] += -hq[0] * (J[2] - J[1]) * w[2];
  gx[12] += -hq[0] * (J[2] - J[1]) * w[1];
  gth[3] += -hq[0] * w[1] * w[2];
  gth[2] += hq[0] * w[1] * w[2];
  gx[12] += -hq[1] * (J[0] - J[2]) * w[0];
  gx[10] += -hq[1] * (J[0] - J[2]) * w[2];
  gth[1] += -hq[1] * w[2] * w[0];
  gth[3] += hq[1] * w[2] * w[0];
  gx[10] += -hq[2] * (J[1] - J[0]) * w[1];
  gx[11] += -hq[2] * (J[1] - J[0]) * w[0];
  gth[2] += -hq[2] * w[0] * w[1];
  gth[1] += hq[2] * w[0] * w[1];
  for (int i = 0; i < 4; ++i)
    gT[i] += c->arm * RSY[i] * gtau[0] - c->arm * RSX[i] * gtau[1] + c->k_m * RD[i] * gtau[2];

  /* F = sum T_i */
  for (int i = 0; i < 4; ++i) gT[i] += gF;

  /* T_i = c0 + c1 w_i + c2 w_i^2 */
  for (int i = 0; i < 4; ++i) {
    gth[4] += gT[i];
    gth[5] += gT[i] * wm[i];
    gth[6] += gT[i] * wm[i] * wm[i];
    gx[13 + i] += gT[i] * (c1 + 2.0 * c2 * wm[i]);
  }

  /* wm_dot = (u - wm) / Tm */
  for (int i = 0; i < 4; ++i) {
    gu[i] += gm[i] / Tm;
    gx[13 + i] += -gm[i] / Tm;
    gth[7] += -gm[i] * (u[i] - wm[i]) / (Tm * Tm);
  }
}

/* VJP of one RK4 step: cotangent g of x_next -> gx, gu, gth (accumulated). */
static void rk4_vjp(const orc_cfg* c, const double th[NP], const double x[NS], const double u[4],
                    const double* d, const double g[NS], double gx[NS], double gu[4],
                    double gth[NP]) {
  const double h = c->dt;
  double k1[NS], k2[NS], k3[NS], x2[NS], x3[NS], x4[NS];
  dynamics(c, th, x, u, d, k1);
  for (int i = 0; i < NS; ++i) x2[i] = x[i] + 0.5 * h * k1[i];
  dynamics(c, th, x2, u, d, k2);
  for (int i = 0; i < NS; ++i) x3[i] = x[i] + 0.5 * h * k2[i];
  dynamics(c, th, x3, u, d, k3);
  for (int i = 0; i < NS; ++i) x4[i] = x[i] + h * k3[i];

  double gk1[NS], gk2[NS], gk3[NS], gk4[NS], gx2[NS], gx3[NS], gx4[NS];
  for (int i = 0; i < NS; ++i) {
    gx[i] += g[i];
    gk1[i] = h / 6.0 * g[i];
    gk2[i] = h / 3.0 * g[i];
    gk3[i] = h / 3.0 * g[i];
    gk4[i] = h / 6.0 * g[i];
    gx2[i] = gx3[i] = gx4[i] = 0.0;
  }
  dynamics_vjp(c, th, x4, u, d, gk4, gx4, gu, gth);
  for (int i = 0; i < NS; ++i) {
    gx[i] += gx4[i];
    gk3[i] += h * gx4[i];
  }
  dynamics_vjp(c, th, x3, u, d, gk3, gx3, gu, gth);
  for (int i = 0; i < NS; ++i) {
    gx[i] += gx3[i];
    gk2[i] += 0.5 * h * gx3[i];
  }
  dynamics_vjp(c, th, x2, u, d, gk2, gx2, gu, gth);
  for (int i = 0; i < NS; ++i) {
    gx[i] += gx2[i];
    gk1[i] += 0.5 * h * gx2[i];
  }
  dynamics_vjp(c, th, x, u, d, gk1, gx, gu, gth);
}

/* VJP of the actor at o with cotangent ga of a: accumulates gW, returns go. */
static void actor_vjp(const double* W, const double o[NO], const double ga[NA], double* gW,
                      double go[NO]) {
  double z1[NHID], z2[NHID], z3[NA], a[NA], h1[NHID], h2[NHID];
  actor(W, o, a, z1, z2, z3);
  for (int n = 0; n < NHID; ++n) {
    h1[n] = z1[n] > 0.0 ? z1[n] : 0.0;
    h2[n] = z2[n] > 0.0 ? z2[n] : 0.0;
  }
  double gz3[NA], gh2[NHID] = {0}, gz2[NHID], gh1[NHID] = {0}, gz1[NHID];
  for (int n = 0; n < NA; ++n) gz3[n] = ga[n] * (1.0 - a[n] * a[n]);
  for (int n = 0; n < NA; ++n) {
    gW[OFF_B3 + n] += gz3[n];
    for (int k = 0; k < NHID; ++k) {
      gW[OFF_W3 + n * NHID + k] += gz3[n] * h2[k];
      gh2[k] += W[OFF_W3 + n * NHID + k] * gz3[n];
    }
  }
  for (int n = 0; n < NHID; ++n) gz2[n] = z2[n] > 0.0 ? gh2[n] : 0.0;
  for (int n = 0; n < NHID; ++n) {
    gW[OFF_B2 + n] += gz2[n];
    for (int k = 0; k < NHID; ++k) {
      gW[OFF_W2 + n * NHID + k] += gz2[n] * h1[k];
      gh1[k] += W[OFF_W2 + n * NHID + k] * gz2[n];
    }
  }
  for (int n = 0; n < NHID; ++n) gz1[n] = z1[n] > 0.0 ? gh1[n] : 0.0;
  for (int k = 0; k < NO; ++k) go[k] = 0.0;
  for (int n = 0; n < NHID; ++n) {
    gW[OFF_B1 + n] += gz1[n];
    for (int k = 0; k < NO; ++k) {
      gW[OFF_W1 + n * NO + k] += gz1[n] * o[k];
      go[k] += W[OFF_W1 + n * NO + k] * gz1[n];
    }
  }
}

/* VJP of the observation map: go (146) -> gs (17), gH (128), accumulated. */
static void observe_vjp(const double s[NS], const double go[NO], double gs[NS], double gH[NH * NA]) {
  for (int i = 0; i < 3; ++i) {
    gs[i] += go[i];
    gs[7 + i] += go[12 + i];
    gs[10 + i] += go[15 + i];
  }
  double qn[4], gqn[4];
  normalize4(s + 3, qn);
  rotmat_vjp(qn, go + 3, gqn);
  normalize4_vjp(s + 3, gqn, gs + 3);
  for (int i = 0; i < NH * NA; ++i) gH[i] += go[18 + i];
}

/* Reward VJP: cotangent gr of r -> gs (post-step state), ga. */
static void reward_vjp(const orc_cfg* c, const double s[NS], const double a[NA], double gr,
                       double gs[NS], double ga[NA]) {
  for (int i = 0; i < 3; ++i) {
    gs[i] += -2.0 * c->C_rp * s[i] * gr;
    gs[7 + i] += -2.0 * c->C_rv * s[7 + i] * gr;
    gs[10 + i] += -2.0 * c->C_rw * s[10 + i] * gr;
  }
  gs[3] += 2.0 * c->C_rq * s[3] * gr;
  for (int i = 0; i < NA; ++i) ga[i] += -2.0 * c->C_ra * (a[i] - c->C_rab) * gr;
}

/* Differentiable rollout of one env from (s0, H0) for T steps without
 * termination or reset.  Loss J = sum_t dR[t] r_t + sum_{t=0..T} dS[t].s_t.
 * Returns J; if gW / gth are non-NULL, accumulates dJ/dW (13828) into gW and
 * writes dJ/dtheta (8) to gth, holding (s0, H0) fixed. */
static double env_grad(const orc_cfg* c, const double* W, const double th[NP], uint32_t env,
                       uint32_t episode, int32_t t_ep0, const double s0[NS],
                       const double H0[NH * NA], int T, const double* dR, size_t dR_stride,
                       const double* dS, size_t dS_stride, double* gW, double* gth) {
  double d[6];
  disturbance(c, env, episode, d);
  double* S = (double*)malloc(sizeof(double) * (size_t)(T + 1) * NS);
  double* Hs = (double*)malloc(sizeof(double) * (size_t)(T + 1) * NH * NA);
  double* A = (double*)malloc(sizeof(double) * (size_t)T * NA);
  memcpy(S, s0, sizeof(double) * NS);
  memcpy(Hs, H0, sizeof(double) * NH * NA);
  double J = 0.0;
  if (dS)
    for (int i = 0; i < NS; ++i) J += dS[i] * S[i];
  for (int t = 0; t < T; ++t) {
    const double* s = S + (size_t)t * NS;
    const double* H = Hs + (size_t)t * NH * NA;
    double* sn = S + (size_t)(t + 1) * NS;
    double* Hn = Hs + (size_t)(t + 1) * NH * NA;
    double o[NO], u[NA];
    double* a = A + (size_t)t * NA;
    observe(s, H, o);
    add_obs_noise(c, env, episode, t_ep0 + t, o);
    actor(W, o, a, NULL, NULL, NULL);
    action_to_rpm(c, a, u);
    rk4(c, th, s, u, d, sn);
    if (c->flags & F_RENORM_Q) {
      double qn[4];
      normalize4(sn + 3, qn);
      memcpy(sn + 3, qn, sizeof qn);
    }
    double r = reward(c, sn, a);
    J += (dR ? dR[(size_t)t * dR_stride] : 1.0) * r;
    if (dS)
      for (int i = 0; i < NS; ++i) J += dS[(size_t)(t + 1) * dS_stride + i] * sn[i];
    memcpy(Hn, H + NA, sizeof(double) * (NH - 1) * NA);
    memcpy(Hn + (NH - 1) * NA, a, sizeof(double) * NA);
  }
  if (gW || gth) {
    double ls[NS], lH[NH * NA];
    double gth_loc[NP] = {0};
    for (int i = 0; i < NS; ++i) ls[i] = dS ? dS[(size_t)T * dS_stride + i] : 0.0;
    for (int i = 0; i < NH * NA; ++i) lH[i] = 0.0;
    double* gW_loc = gW;
    double gW_dummy_needed = (gW == NULL);
    double* scratchW = NULL;
    if (gW_dummy_needed) {
      scratchW = (double*)calloc(NW, sizeof(double));
      gW_loc = scratchW;
    }
    for (int t = T - 1; t >= 0; --t) {
      const double* s = S + (size_t)t * NS;
      const double* H = Hs + (size_t)t * NH * NA;
      const double* sn = S + (size_t)(t + 1) * NS;
      const double* a = A + (size_t)t * NA;
      double gsn[NS], ga[NA] = {0, 0, 0, 0}, graw[NS], gs[NS], gu[NA] = {0, 0, 0, 0}, go[NO];
      double gH[NH * NA];
      memcpy(gsn, ls, sizeof gsn);
      reward_vjp(c, sn, a, dR ? dR[(size_t)t * dR_stride] : 1.0, gsn, ga);
      /* H_{t+1} = [H_t[1..31], a_t] */
      for (int i = 0; i < NA; ++i) ga[i] += lH[(NH - 1) * NA + i];
      /* renormalisation after the step */
      double u[NA], xr[NS];
      action_to_rpm(c, a, u);
      memcpy(graw, gsn, sizeof graw);
      if (c->flags & F_RENORM_Q) {
        rk4(c, th, s, u, d, xr);
        double gq[4] = {0, 0, 0, 0};
        normalize4_vjp(xr + 3, gsn + 3, gq);
        memcpy(graw + 3, gq, sizeof gq);
      }
      for (int i = 0; i < NS; ++i) gs[i] = 0.0;
      rk4_vjp(c, th, s, u, d, graw, gs, gu, gth_loc);
      for (int i = 0; i < NA; ++i) ga[i] += gu[i] * 0.5 * (c->rpm_max - c->rpm_min);
      double o[NO];
      observe(s, H, o);
      add_obs_noise(c, env, episode, t_ep0 + t, o);  /* additive: the VJP to s is unchanged */
      actor_vjp(W, o, ga, gW_loc, go);
      for (int i = 0; i < NH * NA; ++i) gH[i] = 0.0;
      observe_vjp(s, go, gs, gH);
      /* history adjoint: H_t[k] feeds H_{t+1}[k-1] for k >= 1 */
      for (int k = NH * NA - 1; k >= NA; --k) gH[k] += lH[k - NA];
      memcpy(lH, gH, sizeof lH);
      for (int i = 0; i < NS; ++i) ls[i] = gs[i] + (dS ? dS[(size_t)t * dS_stride + i] : 0.0);
    }
    if (gth) memcpy(gth, gth_loc, sizeof gth_loc);
    free(scratchW);
  }
  free(S);
  free(Hs);
  free(A);
  return J;
}

typedef struct {
  const orc_cfg* c;
  const double *W, *theta, *s0, *H0, *dR, *dS;
  const uint32_t* ids;
  const int32_t *t_ep0, *ep;
  int n, T, i0, i1, want_grad;
  double *gW_part, *gth, *J_part;
} grad_job;

static void* grad_worker(void* arg) {
  grad_job* j = (grad_job*)arg;
  double Jsum = 0.0;
  for (int i = j->i0; i < j->i1; ++i) {
    const double* dR = j->dR ? j->dR + i : NULL;
    const double* dS = j->dS ? j->dS + (size_t)i * NS : NULL;
    Jsum += env_grad(j->c, j->W, j->theta + (size_t)i * NP, env_id(j->ids, i),
                     j->ep ? (uint32_t)j->ep[i] : 0u, j->t_ep0 ? j->t_ep0[i] : 0,
                     j->s0 + (size_t)i * NS,
                     j->H0 + (size_t)i * NH * NA, j->T, dR, (size_t)j->n, dS, (size_t)j->n * NS,
                     j->want_grad ? j->gW_part : NULL,
                     j->want_grad ? j->gth + (size_t)i * NP : NULL);
  }
  *j->J_part = Jsum;
  return NULL;
}

/* Batched loss and gradient.  dR: [T][n] (NULL = all ones); dS: [T+1][n][17]
 * (NULL = zeros).  gW (13828) receives the sum over envs; gth: [n][8]. Either
 * may be NULL only together (loss only).  ids, t_ep0, ep: env ids, step within
 * the episode and episode at the start (NULL = i, 0, 0), which key the
 * disturbance and the observation noise.  Returns J.  Thread partial sums of
 * gW are added in thread order, so results do not depend on scheduling. */
double orc_grad(const orc_cfg* c, int n, const uint32_t* ids, const int32_t* t_ep0,
                const int32_t* ep, const double* W, const double* theta, const double* s0,
                const double* H0, int T, const double* dR, const double* dS, double* gW,
                double* gth, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n) nthreads = n > 0 ? n : 1;
  if (nthreads > 256) nthreads = 256;
  int want = gW != NULL && gth != NULL;
  grad_job jobs[256];
  pthread_t th[256];
  double Jp[256];
  double* parts = want ? (double*)calloc((size_t)nthreads * NW, sizeof(double)) : NULL;
  for (int k = 0; k < nthreads; ++k) {
    grad_job j = {c, W, theta, s0, H0, dR, dS, ids, t_ep0, ep, n, T, (int)((long)n * k / nthreads),
                  (int)((long)n * (k + 1) / nthreads), want,
                  want ? parts + (size_t)k * NW : NULL, gth, &Jp[k]};
    jobs[k] = j;
  }
  if (nthreads == 1) {
    grad_worker(&jobs[0]);
  } else {
    for (int k = 0; k < nthreads; ++k) pthread_create(&th[k], NULL, grad_worker, &jobs[k]);
    for (int k = 0; k < nthreads; ++k) pthread_join(th[k], NULL);
  }
  double J = 0.0;
  for (int k = 0; k < nthreads; ++k) J += Jp[k];
  if (want) {
    for (int i = 0; i < NW; ++i) gW[i] = 0.0;
    for (int k = 0; k < nthreads; ++k)
      for (int i = 0; i < NW; ++i) gW[i] += parts[(size_t)k * NW + i];
    free(parts);
  }
  return J;
}
