// Actor MLP building blocks shared by the forward and backward kernels: LDS
// layouts of the staged weights, staging, and the two forward evaluations
// (vector ALUs, fp32 matrix cores).
#pragma once
#include "qs_device.h"

namespace qs {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16 __attribute__((ext_vector_type(16)));

// LDS layouts (floats).
// MFMA: W1 row-major [64][148] with b1 in column 0 and feature k in column
// k + 1 (column 147 zero), b1, W2 [64][68], b2, W3 [4][68], b3.  Row pitches keep 16-byte alignment and spread the 16 rows one
// 16-lane group reads over distinct banks.
constexpr int M_W1_LD = 148, M_W2_LD = 68;
constexpr int M_W1 = 0, M_B1 = M_W1 + NHID * M_W1_LD, M_W2 = M_B1 + NHID,
              M_B2 = M_W2 + NHID * M_W2_LD, M_W3 = M_B2 + NHID, M_B3 = M_W3 + NA * M_W2_LD,
              M_TOTAL = M_B3 + 4;
// VALU: transposed weights so consecutive outputs are consecutive floats.
constexpr int V_W1T = 0, V_B1 = V_W1T + NO * NHID, V_W2T = V_B1 + NHID,
              V_B2 = V_W2T + NHID * NHID, V_W3T = V_B2 + NHID, V_B3 = V_W3T + NHID * NA,
              V_TOTAL = V_B3 + NA;
// bf16 actor option, one env per lane (bf16 elements first, then fp32):
//   MB_W1: W1 row-major [64][148] (features 146, 147 zero); a lane reads the
//          4 weights of one K-chunk as 8 bytes, and the pitch of 74 dwords
//          puts the 16 rows one lane group reads on distinct bank pairs;
//   MB_W2: [64][72], within a row instruction m (layer-1 tiles 2m, 2m+1) and
//          lane group g hold the 8 inputs mb_in(m, g, e), the order in which
//          the layer-1 result registers arrive.
// Biases stay fp32; W3 is kept as fp32 copies of its bf16-rounded values for
// the fp32 4x4x1 layer 3 (bf16 products are exact in fp32).
constexpr int MB_P1 = 148, MB_P2 = 72;
constexpr int MB_W1 = 0, MB_W2 = MB_W1 + NHID * MB_P1, MB_BF16_END = MB_W2 + NHID * MB_P2;
constexpr int MB_F = MB_BF16_END / 2;
constexpr int MB_B1 = MB_F, MB_B2 = MB_B1 + NHID, MB_W3 = MB_B2 + NHID,
              MB_B3 = MB_W3 + NA * M_W2_LD, MB_TOTAL = MB_B3 + 4;
static_assert(MB_BF16_END % 8 == 0, "fp32 part must stay 16-byte aligned");

// Layer-1 neuron that element e of lane group g feeds in layer-2 instruction m.
__host__ __device__ constexpr int mb_in(int m, int g, int e) {
  return 32 * m + 16 * (e >> 2) + 4 * g + (e & 3);
}

constexpr int LDS_FLOATS_F32 = M_TOTAL > V_TOTAL ? M_TOTAL : V_TOTAL;
constexpr int LDS_FLOATS = LDS_FLOATS_F32 > MB_TOTAL ? LDS_FLOATS_F32 : MB_TOTAL;

template <bool MFMA>
__device__ inline void stage_actor(const float* __restrict__ W, float* lds) {
  if (MFMA) {
    // W1 with the bias as column 0, rows padded to M_W1_LD
    stage_lds(lds + M_W1, NHID * M_W1_LD, W, [](int i) {
      const int r = i / M_W1_LD, k = i % M_W1_LD;
      return k == 0 ? OFF_B1 + r : k <= NO ? OFF_W1 + r * NO + k - 1 : -1;
    });
    stage_lds(lds + M_W2, NHID * M_W2_LD, W, [](int i) {
      const int r = i / M_W2_LD, k = i % M_W2_LD;
      return k < NHID ? OFF_W2 + r * NHID + k : -1;
    });
    stage_lds(lds + M_W3, NA * M_W2_LD, W, [](int i) {
      const int r = i / M_W2_LD, k = i % M_W2_LD;
      return k < NHID ? OFF_W3 + r * NHID + k : -1;
    });
    stage_lds(lds + M_B1, NHID, W, [](int i) { return OFF_B1 + i; });
    stage_lds(lds + M_B2, NHID, W, [](int i) { return OFF_B2 + i; });
    stage_lds(lds + M_B3, NA, W, [](int i) { return OFF_B3 + i; });
  } else {
    // transposed: [input][neuron]
    stage_lds(lds + V_W1T, NO * NHID, W,
              [](int i) { return OFF_W1 + (i % NHID) * NO + i / NHID; });
    stage_lds(lds + V_W2T, NHID * NHID, W,
              [](int i) { return OFF_W2 + (i % NHID) * NHID + i / NHID; });
    stage_lds(lds + V_W3T, NHID * NA, W,
              [](int i) { return OFF_W3 + (i % NA) * NHID + i / NA; });
    stage_lds(lds + V_B1, NHID, W, [](int i) { return OFF_B1 + i; });
    stage_lds(lds + V_B2, NHID, W, [](int i) { return OFF_B2 + i; });
    stage_lds(lds + V_B3, NA, W, [](int i) { return OFF_B3 + i; });
  }
}

__device__ inline void stage_actor_bf16(const float* __restrict__ W, float* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __bf16* h = reinterpret_cast<__bf16*>(lds);
  for (int i = tid; i < NHID * MB_P1; i += nt) {
    const int r = i / MB_P1, k = i % MB_P1;
    h[MB_W1 + i] = (__bf16)(k < NO ? W[OFF_W1 + r * NO + k] : 0.0f);
  }
  for (int i = tid; i < NHID * MB_P2; i += nt) {
    const int r = i / MB_P2, col = i % MB_P2;
    const float v = col < NHID ? W[OFF_W2 + r * NHID + mb_in(col >> 5, (col >> 3) & 3, col & 7)]
                               : 0.0f;
    h[MB_W2 + i] = (__bf16)v;
  }
  for (int i = tid; i < NA * M_W2_LD; i += nt) {
    const int r = i / M_W2_LD, k = i % M_W2_LD;
    lds[MB_W3 + i] = k < NHID ? (float)(__bf16)W[OFF_W3 + r * NHID + k] : 0.0f;
  }
  for (int i = tid; i < NHID; i += nt) {
    lds[MB_B1 + i] = W[OFF_B1 + i];
    lds[MB_B2 + i] = W[OFF_B2 + i];
  }
  for (int i = tid; i < NA; i += nt) lds[MB_B3 + i] = W[OFF_B3 + i];
}

// Observation feature k of this lane's env (compile-time k after unrolling).
#define QS_FEAT(k)                                                                  \
  ((k) < 3 ? s[(k)] : (k) < 12 ? Rm[(k)-3] : (k) < 15 ? s[(k)-12 + 7] : (k) < 18 ? \
   s[(k)-15 + 10] : H[(k)-18])

// Layer 3 of the one-env-per-lane actors from the layer-2 result registers
// acc2[n2][bb] (ReLU applied): one 16-block 4x4x1 fp32 MFMA per register, then
// two swap-and-add rounds.  W3 at w3 ([4][M_W2_LD] floats), b3 at b3.
__device__ inline void layer3_one_lane(const float* lds, int w3, int b3off, const f4 acc2[4][4],
                                       float z3out[NA]) {
  const int lane = threadIdx.x & 63, lg = lane >> 4;
  // the bias enters once, in lane group 0's partial sums
  f4 b3;
#pragma unroll
  for (int r = 0; r < 4; ++r) b3[r] = lg == 0 ? lds[b3off + r] : 0.0f;
  f4 acc3[4];  // [bb]: register o = output o, partial over lane group lg
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    const f4 w = *reinterpret_cast<const f4*>(&lds[w3 + (lane & 3) * M_W2_LD + 16 * n2 + 4 * lg]);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        acc3[bb] = __builtin_amdgcn_mfma_f32_4x4x1f32(
            w[v], acc2[n2][bb][v], (n2 == 0 && v == 0) ? b3 : acc3[bb], 0, 0, 0);
  }
  // Lane 16 g + i holds, for each bb, output o of env 16 bb + i summed over
  // the neurons of lane group g.  Swapping the upper 32 lanes of bb with the
  // lower 32 of bb + 2 and adding gives groups {0,2} and {1,3} of bb in the
  // lower half and of bb + 2 in the upper half; swapping the odd 16-lane rows
  // of (0,2) with the even rows of (1,3) and adding completes the sums with
  // row g holding bb = g, the env of the lane itself.
#pragma unroll
  for (int o = 0; o < NA; ++o) {
    const auto p02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc3[0][o]),
                                                      __float_as_uint(acc3[2][o]), false, false);
    const auto p13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc3[1][o]),
                                                      __float_as_uint(acc3[3][o]), false, false);
    const float z02 = __uint_as_float(p02[0]) + __uint_as_float(p02[1]);
    const float z13 = __uint_as_float(p13[0]) + __uint_as_float(p13[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(z02), __float_as_uint(z13),
                                                    false, false);
    z3out[o] = __uint_as_float(q[0]) + __uint_as_float(q[1]);
  }
}

// Actor on matrix cores.  Each wave evaluates its 64 envs together:
//  layer 1: 147 rank-1 updates per 16-neuron tile with the 4-block
//           16x16x1 fp32 MFMA, the first one the bias (a constant feature
//           1 on a zero accumulator, so the bias is added first as in the
//           plain evaluation); B = feature k of the 64 envs (one per lane,
//           4 blocks of 16 envs), A = weights of 16 neurons broadcast to
//           the 4 blocks.  The result registers hold (neuron, env) tiles.
//  layer 2:  16x16x4 fp32 MFMA.  A result register of layer 1 is directly a
//           B operand whose K-chunk is 4 neurons {4g+v}; the weights are
//           read in the matching order.  The bias tile is the accumulator
//           input of each chain's first product.
//  layer 3:  16-block 4x4x1 fp32 MFMA, one per layer-2 result register:
//           block b (lanes 4b..4b+3) takes that register's neuron for its
//           lane group g = b/4 and its 4 envs as B, the 4 output weights of
//           that neuron as A (row o = lane & 3), so no product is padding.
//           Each lane group ends with a partial sum over its quarter of the
//           neurons; two swap-and-add rounds across 32 and 16 lanes add the
//           quarters and leave output o of env (lane) in every lane.
//  REC: when rec_on (wave uniform), also store the layer pre-activations
//  and the ReLU masks into the backward's blocked record (zr: the record
//  span, the byte offsets of the z1, z2 and mask rows of the wave's 64-env
//  block in this step's record, the lane's offset 4 (4 lg 64 + li) in a tile
//  row and its own column's offset).  Register 4 bb + v (neuron 16 n + 4 lg
//  + v of env 16 bb + li) goes to row 16 n + 4 lg + v, column 16 bb + li.
//  Every column is written, those of envs past the batch with the values of
//  the lanes that shadow them.  The mask words, in the same layout (bit 16 n
//  + 4 bb + v of word n / 2: layer 1, words 0-1; layer 2, words 2-3), go to
//  the lane's own column of the mask rows.
struct ZRec {
  __amdgpu_buffer_rsrc_t r;
  uint32_t s1, s2, v, sm, vo;
};
// Sets bit 16 h + r of w (r = 15 .. 0 in turn, w shifted left each time) when
// z[r] > 0: the two halves of a mask word are filled high half first.
__device__ inline uint32_t push_mask_bit(uint32_t w, float z) {
  return (w << 1) | (z > 0.0f ? 1u : 0u);
}

template <bool REC = false>
__device__ inline void actor_mfma(const float* lds, const float s[NS], const float Rm[9],
                                  const float H[NH * NA], float z3out[NA],
                                  const ZRec* zr = nullptr, bool rec_on = false) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const f16 zero16 = {};
  f16 acc1[4];
#pragma unroll
  for (int kc = 0; kc < M_W1_LD / 4; ++kc) {
    f4 w[4];
#pragma unroll
    for (int n = 0; n < 4; ++n)
      w[n] = *reinterpret_cast<const f4*>(&lds[M_W1 + (16 * n + li) * M_W1_LD + 4 * kc]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int col = 4 * kc + kk;  // 0: bias, k + 1: feature k
      if (col == 0) {
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc1[n] = __builtin_amdgcn_mfma_f32_16x16x1f32(w[n][0], 1.0f, zero16, 0, 0, 0);
      } else if (col <= NO) {
        const float x = QS_FEAT(col - 1);
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc1[n] = __builtin_amdgcn_mfma_f32_16x16x1f32(w[n][kk], x, acc1[n], 0, 0, 0);
      }
    }
  }
  if (REC && rec_on) {
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          bst1(acc1[n][4 * bb + v], zr->r, zr->v, zr->s1 + 4u * ((16 * n + v) * 64 + 16 * bb));
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      uint32_t m = 0u;
#pragma unroll
      for (int h = 1; h >= 0; --h)
#pragma unroll
        for (int r = 15; r >= 0; --r) m = push_mask_bit(m, acc1[2 * w + h][r]);
      bst1(__uint_as_float(m), zr->r, zr->vo, zr->sm + 4u * w * 64);
    }
  }
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc1[n][r] = relu_bits(acc1[n][r]);

  f4 acc2[4][4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const f4 w =
          *reinterpret_cast<const f4*>(&lds[M_W2 + (16 * n2 + li) * M_W2_LD + 16 * n + 4 * lg]);
      const f4 b2 = *reinterpret_cast<const f4*>(&lds[M_B2 + 16 * n2 + 4 * lg]);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          acc2[n2][bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              w[v], acc1[n][4 * bb + v], (n == 0 && v == 0) ? b2 : acc2[n2][bb], 0, 0, 0);
    }
  if (REC && rec_on) {
    // register r of acc2[n2][bb]: neuron 16 n2 + 4 lg + r of env 16 bb + li
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          bst1(acc2[n2][bb][r], zr->r, zr->v, zr->s2 + 4u * ((16 * n2 + r) * 64 + 16 * bb));
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      uint32_t m = 0u;
#pragma unroll
      for (int h = 1; h >= 0; --h)
#pragma unroll
        for (int q = 15; q >= 0; --q) m = push_mask_bit(m, acc2[2 * w + h][q >> 2][q & 3]);
      bst1(__uint_as_float(m), zr->r, zr->vo, zr->sm + 4u * (2 + w) * 64);
    }
  }
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc2[n2][bb][r] = relu_bits(acc2[n2][bb][r]);

  layer3_one_lane(lds, M_W3, M_B3, acc2, z3out);
}

typedef short s4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// bf16 actor, one env per lane: weights and every layer input rounded to
// bf16 (round to nearest even), products accumulated in fp32, biases,
// activations and layer 3's accumulation in fp32.
//  layer 1: the 4-block v_mfma_f32_16x16x4bf16_1k: block b takes envs
//           16b..16b+15, B = 4 consecutive features of the lane's own env,
//           A = the 4 weights of 16 neurons (the same in every block); the
//           result registers have the fp32 kernel's (neuron, env) layout.
//  layer 2: v_mfma_f32_16x16x32_bf16 over two layer-1 tiles at a time, the
//           8 elements of a lane taken from its result registers in mb_in
//           order.
//  layer 3: as in the fp32 actor, on the bf16-rounded inputs and weights.
__device__ inline void actor_mfma_bf16(const float* lds, const float s[NS], const float Rm[9],
                                       const float H[NH * NA], float z3out[NA]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const __bf16* h = reinterpret_cast<const __bf16*>(lds);
  f16 acc1[4];
#pragma unroll
  for (int c = 0; c < MB_P1 / 4; ++c) {
    bf4v xb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * c + e;
      xb[e] = (__bf16)(k < NO ? QS_FEAT(k) : 0.0f);
    }
    const s4v x = __builtin_bit_cast(s4v, xb);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const s4v w = *reinterpret_cast<const s4v*>(&h[MB_W1 + (16 * n + li) * MB_P1 + 4 * c]);
      f16 b;
      if (c == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) b[r] = lds[MB_B1 + 16 * n + 4 * lg + (r & 3)];
      }
      acc1[n] = __builtin_amdgcn_mfma_f32_16x16x4bf16_1k(w, x, c == 0 ? b : acc1[n], 0, 0, 0);
    }
  }
  f4 acc2[4][4];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    bf8v x[4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        x[bb][e] = (__bf16)relu_bits(acc1[2 * m + (e >> 2)][4 * bb + (e & 3)]);
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const bf8v w =
          *reinterpret_cast<const bf8v*>(&h[MB_W2 + (16 * n2 + li) * MB_P2 + 32 * m + 8 * lg]);
      const f4 b2 = *reinterpret_cast<const f4*>(&lds[MB_B2 + 16 * n2 + 4 * lg]);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        acc2[n2][bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x[bb], m == 0 ? b2 : acc2[n2][bb],
                                                               0, 0, 0);
    }
  }
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc2[n2][bb][r] = (float)(__bf16)relu_bits(acc2[n2][bb][r]);
  layer3_one_lane(lds, MB_W3, MB_B3, acc2, z3out);
}

// Actor on the vector ALUs, one env per lane, weights broadcast from LDS.
__device__ inline void actor_valu(const float* lds, const float s[NS], const float Rm[9],
                                  const float H[NH * NA], float z3out[NA]) {
  float z1[NHID];
#pragma unroll
  for (int n = 0; n < NHID; ++n) z1[n] = lds[V_B1 + n];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const float x = QS_FEAT(k);
#pragma unroll
    for (int nc = 0; nc < NHID / 4; ++nc) {
      const f4 w = *reinterpret_cast<const f4*>(&lds[V_W1T + k * NHID + 4 * nc]);
#pragma unroll
      for (int j = 0; j < 4; ++j) z1[4 * nc + j] = fmaf(w[j], x, z1[4 * nc + j]);
    }
  }
  float z2[NHID];
#pragma unroll
  for (int n = 0; n < NHID; ++n) z2[n] = lds[V_B2 + n];
#pragma unroll
  for (int k = 0; k < NHID; ++k) {
    const float x = fmaxf(z1[k], 0.0f);
#pragma unroll
    for (int nc = 0; nc < NHID / 4; ++nc) {
      const f4 w = *reinterpret_cast<const f4*>(&lds[V_W2T + k * NHID + 4 * nc]);
#pragma unroll
      for (int j = 0; j < 4; ++j) z2[4 * nc + j] = fmaf(w[j], x, z2[4 * nc + j]);
    }
  }
#pragma unroll
  for (int n = 0; n < NA; ++n) z3out[n] = lds[V_B3 + n];
#pragma unroll
  for (int k = 0; k < NHID; ++k) {
    const float x = fmaxf(z2[k], 0.0f);
    const f4 w = *reinterpret_cast<const f4*>(&lds[V_W3T + k * NA]);
#pragma unroll
    for (int j = 0; j < 4; ++j) z3out[j] = fmaf(w[j], x, z3out[j]);
  }
}


}  // namespace qs
