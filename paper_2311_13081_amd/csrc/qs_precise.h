// Double-precision forward path (qs_precise.hip), selected by SIM_F_FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

struct PreciseCfg {
  int n_envs, max_steps, flags, dr_enable;
  double dt, g, arm, km, rpm_min, rpm_max;
  double pos_limit, vel_limit, init_pos, init_angle, init_vel, init_angvel;
  double C_rp, C_rq, C_rv, C_rw, C_ra, C_rab, C_rs;
  double nominal[8], dr_lo[8], dr_hi[8];
  uint32_t seed_lo, seed_hi, dr_seed_lo, dr_seed_hi;
  double dist_force, dist_torque, noise[4];
};

struct PreciseBufs {
  double* state;   // [17][N]
  double* ring;    // [32][4][N], logical slot s at (head+s)&31
  int32_t* head;   // [N]
  int32_t* t_ep;   // [N]
  int32_t* ep;     // [N]
  double* theta;   // [8][N]
  double* ret;     // [2][N] return of the current episode so far; of the last finished one
  int32_t* last_len;  // [N] steps of the last finished episode
};

constexpr int PRECISE_LDS_BYTES = 13828 * 8;

hipError_t precise_prepare();
hipError_t precise_init(const PreciseCfg& p, const PreciseBufs& b, int params, hipStream_t st);
hipError_t precise_run(const PreciseCfg& p, const PreciseBufs& b, const float* W,
                       const float* ext, int T, int t_base, float* rewards, uint8_t* dones,
                       float* states, hipStream_t st);
// Float32 snapshots; ret [2][N] and last_len [N] are the episode
// accumulators.  Any pointer may be NULL.
hipError_t precise_get(const PreciseBufs& b, int N, float* state, float* hist, int32_t* t_ep,
                       int32_t* ep, float* theta, float* ret, int32_t* last_len, hipStream_t st);
hipError_t precise_set(const PreciseBufs& b, int N, const float* state, const float* hist,
                       const int32_t* t_ep, const int32_t* ep, const float* theta,
                       const float* ret, const int32_t* last_len, hipStream_t st);

}  // namespace qs
