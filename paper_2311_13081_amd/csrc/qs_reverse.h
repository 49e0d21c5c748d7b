// Reverse of one env step's dynamics, shared by the reverse sweeps of every
// lane layout (qs_backward.hip, qs_reverse1.hip).
#pragma once
#include "qs_device.h"

namespace qs {

constexpr int DZ_F = NHID + NHID + NA;  // layer cotangents dz1 | dz2 | dz3 per (step, env)
constexpr int LAM_F = NS + NH * NA;     // state and history adjoints carried between segments

// Weight as the forward used it: rounded to bf16 under the bf16-actor flag.
__device__ inline float fwd_weight(float w, bool bf16) { return bf16 ? (float)(__bf16)w : w; }

// Reverse of one step's dynamics: recomputes the RK4 stages from the recorded
// state x and action a, then steps back through the reward, the quaternion
// renormalisation and the four stages.  In: ls (state adjoint after the
// step), hn (adjoint of the newest history slot, i.e. of a).
// Out: gx (state adjoint before the step, without the observation's share),
// ga (action adjoint, the history coupling included); gth accumulates the
// parameter gradients.
__device__ __forceinline__ void reverse_dynamics(const DevCfg& c, const Body<float>& B,
                                                 const float th[NP], bool renorm, const float x[NS],
                                                 const float a[NA], float dR, const float ls[NS],
                                                 const float hn[NA], float gx[NS], float ga[NA],
                                                 float gth[NP]) {
  const float h = c.dt;
  float u[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) u[i] = action_to_rpm(c, a[i]);
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
  float g[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) g[i] = ls[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[i] += -2.0f * c.C_rp * sn[i] * dR;
    g[7 + i] += -2.0f * c.C_rv * sn[7 + i] * dR;
    g[10 + i] += -2.0f * c.C_rw * sn[10 + i] * dR;
  }
  g[3] += 2.0f * c.C_rq * sn[3] * dR;
  // the newest history slot's adjoint joins the action's
#pragma unroll
  for (int i = 0; i < NA; ++i) ga[i] = -2.0f * c.C_ra * (a[i] - c.C_rab) * dR + hn[i];

  // --- renormalisation ------------------------------------------------------
  if (renorm) {
    const float d = sn[3] * g[3] + sn[4] * g[4] + sn[5] * g[5] + sn[6] * g[6];
#pragma unroll
    for (int i = 0; i < 4; ++i) g[3 + i] = (g[3 + i] - sn[3 + i] * d) * rn;
  }

  // --- RK4 stages in reverse ----------------------------------------------
  float gk[NS], gs[NS], gu[NA] = {0.0f, 0.0f, 0.0f, 0.0f};
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
}

}  // namespace qs
