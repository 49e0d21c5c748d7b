/*
 * quadsim.h -- C ABI of the MI355X batched quadrotor environment.
 *
 * The library advances N independent quadrotors.  Each one is the Markov
 * decision process of "Learning to Fly in Seconds" (Eschmann, Albani,
 * Loianno, IEEE RA-L 2024), Sec. IV (Methodology):
 *   state s = {p, q, v, w, w_m} (17 floats: position, unit quaternion
 *     (w,x,y,z), linear velocity, body angular velocity, 4 rotor speeds in
 *     RPM), integrated with classical RK4 at the configured dt (100 Hz in
 *     Sec. V, Simulation);
 *   actor observation {p, R(q) row-major, v, w, H} with H the last 32 actions
 *     oldest first, 18 + 4*32 = 146 inputs (Sec. IV);
 *   actor MLP 146-64-64-4, ReLU, ReLU, tanh; action a in (-1,1)^4 mapped to
 *     RPM set points u = rpm_min + (a+1)/2 (rpm_max - rpm_min) (Sec. IV);
 *   rotors: thrust c0 + c1 w + c2 w^2, first-order lag with time constant T_m
 *     (Sec. IV and the taxonomy of Sec. II, levels 4.3 and 5.1);
 *   reward r = -C_rp|p|^2 - C_rq(1-q_w^2) - C_rv|v|^2 - C_rw|w|^2
 *              - C_ra|a - C_rab|^2 + C_rs on the post-step state (Sec. IV);
 *   termination when any |p_i| > pos_limit, any |v_i| > vel_limit or the state
 *     is not finite (the box around the origin of Sec. V, Training);
 *     truncation at max_episode_steps; optional in-kernel reset.
 *
 * Conventions for every call:
 *   - Pointers named "dev" are device pointers on the handle's device; all
 *     device buffers use struct-of-arrays layouts: element (k, env) of a
 *     [K][N] array is at k*N + env.
 *   - The caller owns every pointer it passes; the library never frees them
 *     and keeps none after the call returns.  The handle owns all internal
 *     device memory (state, history, parameters, tape, scratch).
 *   - Every call returns SIM_OK (0) or a negative sim_status and never throws.
 *     Argument errors are detected before any work is queued.  Device errors
 *     (including asynchronous ones from earlier work) map to SIM_E_DEVICE.
 *     sim_last_error() gives a message for the calling thread's last error.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *     All work is queued on it and calls return without synchronising, except
 *     sim_create, sim_destroy and sim_autotune, which synchronise.
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef QUADSIM_H
#define QUADSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SIM_NSTATE = 17,   /* p(3) q(4) v(3) w(3) w_m(4)                                  */
  SIM_NHIST = 32,    /* action history length N_H                                   */
  SIM_NACT = 4,      /* normalised actions / RPM set points                         */
  SIM_NOBS = 146,    /* 18 + 4 * N_H                                                */
  SIM_NHID = 64,     /* hidden width                                                */
  SIM_NPARAM = 8,    /* m, Jxx, Jyy, Jzz, c0, c1, c2, T_m                            */
  SIM_NACTOR = 13828 /* [W1 64x146 | b1 64 | W2 64x64 | b2 64 | W3 4x64 | b3 4]      */
};

typedef enum sim_status {
  SIM_OK = 0,
  SIM_E_INVAL = -1,       /* bad argument                                        */
  SIM_E_NOMEM = -2,       /* device allocation failed                            */
  SIM_E_DEVICE = -3,      /* HIP error, no device, or a launch failed            */
  SIM_E_STATE = -4,       /* call not valid in the handle's current state        */
  SIM_E_UNSUPPORTED = -5  /* option not available for this handle or library    */
} sim_status;

enum {
  SIM_F_TERMINATE = 1,  /* end episodes that leave the box or become non-finite */
  SIM_F_AUTORESET = 2,  /* reset ended episodes inside the step                  */
  SIM_F_RENORM_Q = 4,   /* renormalise the quaternion after each step           */
  SIM_F_FP64 = 8,       /* whole forward step in double precision: state, history
                           and parameters stored in double, observation, actor,
                           RK4, reward and reset draws evaluated in double (the
                           termination box test stays in float32).  Forward only:
                           such a handle records no tape; float32 interfaces
                           (states, snapshots, parameters) round on output and
                           widen on input.  Fixed at creation.                  */
  SIM_F_ACTOR_BF16 = 16, /* actor layers on bf16 matrix cores: weights and layer
                           inputs rounded to bf16 (nearest even), fp32
                           accumulation, biases and activations; the dynamics
                           stay fp32.  Policy steps and rollouts then run on
                           the matrix-core kernels only (SIM_V_AUTO,
                           SIM_V_FUSED_MFMA4 -- the default until tuned -- or
                           SIM_V_FUSED_MFMA; the two sum the bf16 products
                           in different orders); taped rollouts and their
                           backward recompute use the quarter-lane bf16
                           forward, the reverse sweep differentiates it with
                           bf16-rounded weights.  Not combinable with SIM_F_FP64.  Fixed
                           at creation.  (A precision option, not the
                           reference arithmetic: the FP64 oracle stays the
                           reference, and the error against it is larger.)   */
  SIM_F_DISTURB = 32,   /* per-episode disturbance (Sec. IV, asymmetric
                           actor-critic paragraph): a force in the world frame
                           and a torque in the body frame, each component
                           uniform in [-dist_force, dist_force] and
                           [-dist_torque, dist_torque], drawn at every reset
                           from the reset seed and the (env, episode) counter
                           and held for the episode.                          */
  SIM_F_OBS_NOISE = 64  /* additive Gaussian noise on the actor's observation
                           (Sec. IV): the 18 state features p, R, v, w get
                           obs_noise[0..3] times a standard normal drawn per
                           (env, episode, step); the action history and the
                           critic observation stay clean.  Noise is additive,
                           so gradients to the state are unchanged.           */
};

/* Execution variants of the forward step. */
enum {
  SIM_V_AUTO = 0,        /* the autotuned choice (fused MFMA until tuned)         */
  SIM_V_PLAIN = 1,       /* five kernels per step, intermediates through HBM      */
  SIM_V_FUSED_VALU = 2,  /* one fused kernel, actor on the vector ALUs            */
  SIM_V_FUSED_MFMA = 3,  /* one fused kernel, actor on fp32 matrix cores, one env
                            per lane (64 envs per wave)                           */
  SIM_V_FUSED_MFMA4 = 4, /* one fused kernel, actor on fp32 matrix cores, four
                            lanes per env (16 envs per wave); also the kernel of
                            taped rollouts and of the backward recompute          */
  SIM_V_FUSED_SPLIT = 5  /* one fused kernel, the quarter-lane actor split by
                            neuron tile over the 4 waves of a workgroup (16 envs
                            per workgroup, 16 lanes per env): four times the
                            waves of SIM_V_FUSED_MFMA4 for small batches; fp32
                            actor only, untaped rollouts and steps           */
};

typedef struct sim_config {
  int32_t n_envs;            /* 1 <= N <= 2^24 (16 777 216)                          */
  int32_t max_episode_steps; /* truncation cap (0 = none)                            */
  int32_t flags;             /* SIM_F_*                                              */
  int32_t dr_enable;         /* 1: per-env parameters = nominal * U(dr_lo, dr_hi)    */
  int32_t max_tape_horizon;  /* longest differentiable rollout (0 = none)            */
  int32_t ckpt_every;        /* checkpoint interval K of the tape (>= 1)             */
  int32_t reserved0, reserved1;
  double dt, g, arm, k_m, rpm_min, rpm_max; /* s, m/s^2, m, m (yaw moment / thrust), RPM */
  double nominal[SIM_NPARAM];   /* m, Jxx, Jyy, Jzz, c0, c1, c2, T_m                  */
  double dr_lo[SIM_NPARAM], dr_hi[SIM_NPARAM]; /* randomisation factor ranges          */
  double pos_limit, vel_limit;  /* termination box (per axis)                          */
  double init_pos, init_angle, init_vel, init_angvel; /* reset ranges                  */
  double C_rp, C_rq, C_rv, C_rw, C_ra, C_rab, C_rs;   /* reward constants              */
  uint64_t seed;             /* reset-state seed (also keys disturbances and noise)  */
  uint64_t dr_seed;          /* domain-randomisation seed                            */
  double dist_force;         /* N, bound per component (SIM_F_DISTURB)               */
  double dist_torque;        /* N m, bound per component (SIM_F_DISTURB)             */
  double obs_noise[4];       /* noise std on p (m), R entries, v (m/s), w (rad/s)    */
} sim_config;

typedef struct sim_handle sim_handle;

/* Creates a simulator for cfg->n_envs envs on HIP device `device`, allocates
 * all device memory (including the tape for max_tape_horizon steps), draws the
 * per-env parameters from dr_seed and resets every env to episode 0 from
 * cfg->seed.  Synchronises.  *out is NULL on failure.  A differentiable handle
 * (max_tape_horizon > 0) needs the backward's per-segment record, about
 * (128 + 171 ckpt_every) x 4 bytes per env, below 4 GiB (SIM_E_INVAL
 * otherwise). */
int sim_create(const sim_config* cfg, int device, sim_handle** out);

/* Frees everything the handle owns.  Synchronises.  NULL is allowed. */
int sim_destroy(sim_handle* h);

/* Resets every env to episode 0 with reset seed `seed` (Sec. IV initial-state
 * distribution): p ~ U(-init_pos, init_pos)^3, attitude rotated by an angle
 * U(0, init_angle) about a uniformly random axis, v, w uniform in their
 * ranges, rotors at the hover speed of the env's parameters, history filled
 * with the hover action, episode counters zero. */
int sim_reset(sim_handle* h, uint64_t seed, void* stream);

/* One step of every env.  actor: dev [13828] weights; if NULL, actions
 * (dev [4][N], values in [-1,1]) are applied instead of the policy.
 * reward: dev [N] or NULL; done: dev [N] or NULL, bit0 terminated, bit1
 * truncated.  Reward and done describe the transition; with SIM_F_AUTORESET
 * the state left behind for a finished env is its next episode's start. */
int sim_step(sim_handle* h, const float* actor, const float* actions, float* reward,
             uint8_t* done, void* stream);

/* T >= 1 steps of every env under the actor (dev [13828], required).
 * Optional outputs (NULL to skip): rewards dev [T][N], dones dev [T][N],
 * states dev [T+1][17][N] with states[0] the start state.
 * record_tape != 0 stores checkpoints for sim_backward; it requires
 * T <= max_tape_horizon and flags without TERMINATE and AUTORESET, else
 * SIM_E_STATE / SIM_E_INVAL.  A taped rollout runs on the kernel its
 * backward recomputes with (split-actor below 16384 envs with the fp32
 * actor, one env per lane from 65536 envs with the fp32 actor, else
 * quarter-lane), whatever variant is set or tuned, and also writes the
 * backward's records of its last segments (the last one on the split-actor
 * kernel, else up to four), whose recomputes the next sim_backward skips. */
int sim_rollout(sim_handle* h, const float* actor, int32_t T, float* rewards, uint8_t* dones,
                float* states, int32_t record_tape, void* stream);

/* Observations of the current state, for a caller that runs its own policy
 * or critic (Sec. IV, asymmetric actor-critic): actor_obs dev [146][N] = {p,
 * R(q) row-major, v, w, action history oldest first}, with the noise of the
 * coming step under SIM_F_OBS_NOISE (exactly what the next policy step
 * feeds the actor); critic_obs dev [28][N] = {p, R, v, w, rotor speeds, f_r,
 * tau_r}, ground truth.  Either may be NULL.  Not available on SIM_F_FP64
 * handles. */
int sim_observe(sim_handle* h, float* actor_obs, float* critic_obs, void* stream);

/* Dynamics-only rollout: T >= 1 steps with the policy replaced by given
 * normalised actions -- the simulator alone, as in the throughput experiment
 * of Sec. V (Simulation).  actions: dev [4][N] held for every step
 * (actions_per_step == 0) or dev [T][4][N] (actions_per_step != 0).  Outputs
 * as in sim_rollout.  Reward, termination, truncation and reset behave as in
 * sim_step; the action history is left exactly as T single steps would leave
 * it.  Not available on SIM_F_FP64 handles. */
int sim_rollout_actions(sim_handle* h, const float* actions, int32_t actions_per_step, int32_t T,
                        float* rewards, uint8_t* dones, float* states, void* stream);

/* Vector-Jacobian product of the last taped rollout (discrete adjoint through
 * the observation, actor, action map, RK4 stages, quaternion normalisation and
 * history shift).  Cotangents: d_rewards dev [T][N] (NULL = all ones),
 * d_states dev [T+1][17][N] (NULL = zeros).  Outputs: grad_actor dev [13828]
 * (summed over envs and steps, reduced in a fixed order), grad_params dev
 * [8][N] (per env).  Either output may be NULL.  The start state of the
 * rollout is held fixed.  Must use the same actor as the taped rollout.
 * SIM_E_STATE if no tape is recorded. */
int sim_backward(sim_handle* h, const float* actor, const float* d_rewards,
                 const float* d_states, float* grad_actor, float* grad_params, void* stream);

/* sim_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors as sim_backward, but every
 * intermediate of the backward (one segment's record and layer cotangents,
 * the adjoint carry, parameter gradients, weight-gradient partials) lives in
 * a static device array of the library, 32 MiB on each device, held until
 * the process ends; it calls no allocator.  The kernels run in order on
 * `stream` and recompute every segment.  SIM_E_INVAL when the handle's
 * shape needs more than 32 MiB (about 28 KB per env at ckpt_every 16: up to
 * 1024 envs there, 3584 at ckpt_every 4).
 * All calls on one device share the array: calls that overlap in time on
 * one device (other streams, other threads) race and must not be issued. */
int sim_backward_noalloc(sim_handle* h, const float* actor, const float* d_rewards,
                         const float* d_states, float* grad_actor, float* grad_params,
                         void* stream);

/* Snapshot of the per-env state: state dev [17][N], hist dev [32][4][N]
 * (oldest first), t_ep dev [N], episode dev [N], and the episode
 * accumulators (Sec. V, Training: episode return and length are the measures
 * of training progress): returns dev [2][N] = {return of the current episode
 * so far, return of the last finished episode}, last_len dev [N] = steps of
 * the last finished episode (0 until one finishes).  An episode finishes when
 * the step resets the env (SIM_F_AUTORESET): its summed rewards and its
 * length become the "last" values and the running return restarts at 0;
 * without in-step resets the running return keeps summing.  sim_create and
 * sim_reset zero them.  Any pointer may be NULL. */
int sim_get_state(sim_handle* h, float* state, float* hist, int32_t* t_ep, int32_t* episode,
                  float* returns, int32_t* last_len, void* stream);

/* Restores a snapshot (same layouts).  NULL pointers leave that part as is.
 * Invalidates the tape. */
int sim_set_state(sim_handle* h, const float* state, const float* hist, const int32_t* t_ep,
                  const int32_t* episode, const float* returns, const int32_t* last_len,
                  void* stream);

/* Replaces the reward constants C = host {C_rp, C_rq, C_rv, C_rw, C_ra,
 * C_rab, C_rs} (the reward equation of Sec. IV) without touching any env:
 * steps queued after the call use the new values.  This is the hook of a
 * reward curriculum (Sec. IV: the penalty weights grow during training).
 * Values must be finite.  Host-side only (nothing is queued); drops a
 * captured rollout graph. */
int sim_set_reward(sim_handle* h, const double* C);

/* Set point of the actor's observation (Sec. IV: the position controller is
 * steered to any position or velocity by shifting the observed position and
 * velocity, with clipping to keep the errors in the trained range; Sec. VI
 * tracks a trajectory this way): target dev [6][N] = {p_sp (3), v_sp (3)}
 * per env, copied into the handle (stream-ordered); from the next step on
 * the actor observes clip(p - p_sp, +-pos_clip) and clip(v - v_sp,
 * +-vel_clip) in place of p and v (before its observation noise).  The
 * dynamics, reward, termination box and the critic observation keep the
 * absolute state.  target == NULL removes the set point (the clips are then
 * ignored).  Forward only: a taped rollout with a set point in force returns
 * SIM_E_STATE; not available on SIM_F_FP64 handles.  Drops a captured
 * rollout graph and the tape. */
int sim_set_target(sim_handle* h, const float* target, double pos_clip, double vel_clip,
                   void* stream);

/* Ends the episodes of the envs with mask[e] != 0 (mask dev uint8 [N]) and
 * starts their next ones exactly as an in-step reset would (episode + 1,
 * step 0, the counter-RNG start state of (env, episode + 1), history filled
 * with the hover action, episode accumulators closed).  For a caller that
 * steps without SIM_F_AUTORESET so it can read every transition's post-step
 * state before restarting the finished envs.  Not available on SIM_F_FP64
 * handles.  Invalidates the tape. */
int sim_reset_envs(sim_handle* h, const uint8_t* mask, void* stream);

/* Rewards of M given transitions under the handle's current reward
 * constants: rewards dev [M] = r(s', a) for post-step states dev [17][M] and
 * normalised actions dev [4][M] (the reward equation of Sec. IV), e.g. to
 * re-score a replay buffer after sim_set_reward.  M >= 0; with M == 0 the
 * pointers are not used (may be NULL). */
int sim_reward(sim_handle* h, const float* states, const float* actions, int32_t M,
               float* rewards, void* stream);

/* Per-env dynamics parameters theta dev [8][N] (m, Jxx, Jyy, Jzz, c0, c1, c2,
 * T_m).  set: values must be finite with m, J, T_m > 0 and c2 >= 0 (checked
 * on the device at the next step: offending envs produce non-finite states). */
int sim_get_params(sim_handle* h, float* theta, void* stream);
int sim_set_params(sim_handle* h, const float* theta, void* stream);

/* Chooses the forward variant (SIM_V_*), steps per launch for the fused
 * variants (0 = whole rollout in one launch) and whether multi-launch
 * rollouts are replayed from a captured hipGraph (use_graph != 0).  Taped
 * rollouts ignore the variant: they run on the kernel the backward pass
 * recomputes segments with (see sim_rollout). */
int sim_set_variant(sim_handle* h, int variant, int steps_per_launch, int use_graph);
int sim_get_variant(const sim_handle* h, int* variant, int* steps_per_launch, int* use_graph);

/* Times every variant and launch shape on a T-step rollout with HIP events,
 * keeps the fastest (ties go to the earlier candidate), restores the env state
 * afterwards.  Writes the chosen variant and its time to *variant_out and
 * *ms_out (either may be NULL).  Synchronises.  On failure the tuned choice
 * and the variant settings are left as they were, the temporary snapshot is
 * freed, and the env state is unspecified. */
int sim_autotune(sim_handle* h, const float* actor, int32_t T, void* stream, int* variant_out,
                 float* ms_out);

/* Average duration (ms) of the dominant kernel over the last sim_rollout call,
 * from HIP events recorded on the call's stream, and the number of launches
 * it made.  Valid after the stream has completed the rollout. */
int sim_last_rollout_timing(sim_handle* h, float* ms_per_launch, int* launches);

int sim_n_envs(const sim_handle* h);

/* Message for the calling thread's last failed call ("" if none). */
const char* sim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QUADSIM_H */
