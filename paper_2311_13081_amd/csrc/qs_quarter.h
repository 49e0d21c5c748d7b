// Quarter-lane layout shared by the quarter-lane fused kernel and the
// split-actor kernel: lane L = j + 16 k holds quarter k of env j; register c
// of quarter k holds observation feature q_phi(c, k), the B operand of
// v_mfma_f32_16x16x4f32 for 16 envs with K-chunk c.
#pragma once
#include "qs_device.h"

namespace qs {

typedef float f4q __attribute__((ext_vector_type(4)));

constexpr int Q_C = 37;          // K-chunks of layer 1
constexpr int Q_CP = 40;         // padded to whole float4s
constexpr int Q_W1_P = 44;       // LDS pitch of one (quarter, neuron) row: 8 consecutive
                                 // lanes' 16-byte reads land on distinct banks
constexpr int Q_W1 = 0, Q_B1 = Q_W1 + NHID * 4 * Q_W1_P, Q_W2 = Q_B1 + NHID,
              Q_B2 = Q_W2 + NHID * 68, Q_W3 = Q_B2 + NHID, Q_B3 = Q_W3 + NA * 68,
              Q_TOTAL = Q_B3 + 4;

// Observation feature of chunk c, quarter k (or -1 for padding).
__host__ __device__ constexpr int q_phi(int c, int k) {
  return c < 5 ? (4 * c + k < 18 ? 4 * c + k : -1) : 18 + 4 * (c - 5) + k;
}

__device__ inline void stage_q(const float* __restrict__ W, float* lds) {
  // W1 in PHI order: [quarter][neuron][chunk], pitch Q_W1_P
  stage_lds(lds + Q_W1, NHID * 4 * Q_W1_P, W, [](int idx) {
    const int c = idx % Q_W1_P, rest = idx / Q_W1_P, nrn = rest % NHID, k = rest / NHID;
    const int f = c < Q_C ? q_phi(c, k) : -1;
    return f >= 0 ? OFF_W1 + nrn * NO + f : -1;
  });
  stage_lds(lds + Q_W2, NHID * 68, W, [](int i) {
    const int r = i / 68, k = i % 68;
    return k < NHID ? OFF_W2 + r * NHID + k : -1;
  });
  stage_lds(lds + Q_W3, NA * 68, W, [](int i) {
    const int r = i / 68, k = i % 68;
    return k < NHID ? OFF_W3 + r * NHID + k : -1;
  });
  stage_lds(lds + Q_B1, NHID, W, [](int i) { return OFF_B1 + i; });
  stage_lds(lds + Q_B2, NHID, W, [](int i) { return OFF_B2 + i; });
  stage_lds(lds + Q_B3, NA, W, [](int i) { return OFF_B3 + i; });
}


// The 18 observed state features of the lane's env (p, R row-major, v, w),
// with the actor's observation noise when enabled, in the quarter layout:
// F[c] = feature 4c + k (0 past the end).
template <bool EXTRAS>
__device__ inline void quarter_state_features(const DevCfg& c, uint32_t e, uint32_t ep, int t_ep,
                                              int k, const float x[NS], float F[5],
                                              const SetPoint& sp) {
  float Rm[9];
  rotmat(x + 3, Rm);
  float sf[20] = {x[0], x[1], x[2], Rm[0], Rm[1], Rm[2], Rm[3], Rm[4], Rm[5], Rm[6],
                  Rm[7], Rm[8], x[7], x[8], x[9], x[10], x[11], x[12], 0.0f, 0.0f};
  if (EXTRAS) {
    sp.apply(c, sf);
    add_obs_noise(c, e, ep, t_ep, sf);
  }
#pragma unroll
  for (int cc = 0; cc < 5; ++cc)
    F[cc] = k == 0 ? sf[4 * cc] : k == 1 ? sf[4 * cc + 1] : k == 2 ? sf[4 * cc + 2]
                                                                    : sf[4 * cc + 3];
}

// ReLU mask word of a quarter-lane record (row REC_M + k of the lane's env,
// k its quarter): bit 8 n + r is set when layer-1 neuron 16 n + 4 k + r of
// the env has a positive pre-activation, bit 8 n + 4 + r the same for layer
// 2.  z1, z2: the lane's result tiles, before or after the ReLU (z > 0 and
// relu(z) > 0 agree, NaN included).
__device__ inline uint32_t quarter_mask(const f4q z1[4], const f4q z2[4]) {
  uint32_t m = 0u;
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      m |= (z1[n][r] > 0.0f ? 1u : 0u) << (8 * n + r);
      m |= (z2[n][r] > 0.0f ? 1u : 0u) << (8 * n + 4 + r);
    }
  return m;
}

// Layer 3 from the four layer-2 result tiles acc2[n2] (ReLU applied): returns
// z3 (pre-tanh) of the lane's env in all 4 of its lanes.
__device__ inline void layer3_q(const float* lds, const f4q acc2[4], float z3[NA]) {
  const int lane = threadIdx.x & 63, lg = lane >> 4;
  // layer 3: block b (lanes 4b..4b+3) takes the neuron of lane group b/4 and
  // envs 4(b%4)..+3, A = that neuron's 4 output weights (row o = lane & 3);
  // the bias enters once, in lane group 0's partial sums
  f4q b3;
#pragma unroll
  for (int r = 0; r < 4; ++r) b3[r] = lg == 0 ? lds[Q_B3 + r] : 0.0f;
  f4q acc3;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    const f4q w = *reinterpret_cast<const f4q*>(&lds[Q_W3 + (lane & 3) * 68 + 16 * n2 + 4 * lg]);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc3 = __builtin_amdgcn_mfma_f32_4x4x1f32(w[v], acc2[n2][v],
                                                (n2 == 0 && v == 0) ? b3 : acc3, 0, 0, 0);
  }
  // Lane li + 16 g holds output o of env li summed over lane group g's
  // neurons.  A swap of the register with itself across 32 lanes and an add
  // sum groups {0,2} and {1,3}; the same across 16 lanes completes the sum,
  // the same value (same operands, same order) in all 4 lanes of env li.
#pragma unroll
  for (int o = 0; o < NA; ++o) {
    const uint32_t x = __float_as_uint(acc3[o]);
    const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    const float z = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(z), __float_as_uint(z),
                                                    false, false);
    z3[o] = __uint_as_float(q[0]) + __uint_as_float(q[1]);
  }
}

}  // namespace qs
