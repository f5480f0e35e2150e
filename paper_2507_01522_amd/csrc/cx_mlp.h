// cx_mlp.h -- device helpers of the policy MLP shared by the standalone
// policy kernel and the fused policy rollout, so that both compute the same
// logits and draw the same levels bit for bit.
//
// Layout of the two products (both computed transposed, so that no operand is
// shuffled between lanes): with D = A * B on 16 x 16 tiles of
// v_mfma_f32_16x16x32_bf16, lane l holds column l % 16 and rows 4 (l / 16) + i
// (i < 4) of D, and the 8 K-values 8 (l / 16) .. 8 (l / 16) + 7 of A's row
// l % 16 and of B's column l % 16.
//   h^T [hidden x env] = W1^T [hidden x obs] * obs^T [obs x env]
//   z^T [logit x env]  = W2^T [logit x hidden] * h^T [hidden x env]
// A lane ends the first product holding 8 hidden units of one env, exactly the
// B operand of the second (the host stores W2 in that order), and ends the
// second holding every level of one port of one env.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cx_device.h"
#include "cx_internal.h"

namespace cx {
namespace {

constexpr int kPolK1 = 8;  // K-steps of 32 observation features (obs_dim <= 256)
constexpr int kPolHP = 8;  // K-steps of 32 hidden units (hidden <= 256)
constexpr int kPolR = 3;   // tiles of 4 levels per port (levels + 1 <= 12)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values -> two BF16 (lo in the low half), rounded to nearest even:
// one v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// tanh a = 1 - 2 / (e^{2a} + 1); saturates correctly at both ends.
__device__ __forceinline__ float tanh_f(float a) {
  const float e = __builtin_amdgcn_exp2f(a * 2.88539008177792681f);  // 2 / ln 2
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// The hidden units of one K-step of the second product from the two tiles of
// the first (c0: units 4 (l / 16) + i, c1: units 16 + 4 (l / 16) + i), bias
// added, tanh, rounded to BF16.
__device__ __forceinline__ u32x4 hidden_frag(f32x4 c0, f32x4 c1, f32x4 bA, f32x4 bB) {
  return u32x4{pack2(tanh_f(c0.x + bA.x), tanh_f(c0.y + bA.y)), pack2(tanh_f(c0.z + bA.z), tanh_f(c0.w + bA.w)),
               pack2(tanh_f(c1.x + bB.x), tanh_f(c1.y + bB.y)), pack2(tanh_f(c1.z + bB.z), tanh_f(c1.w + bB.w))};
}

// The uniform of a port's level draw from its Philox word: (top 24 bits + 1/2)
// 2^-24.  Port p takes word (p / 16) mod 4 of the call with counter index
// p mod 16 + 16 (p / 64): ports 16 apart share a call.
__device__ __forceinline__ float draw_uniform(uint32_t w) { return ((float)(w >> 8) + 0.5f) * 0x1p-24f; }
__device__ __forceinline__ uint32_t draw_index(int port) { return (uint32_t)(port % 16 + 16 * (port / 64)); }
__device__ __forceinline__ uint32_t draw_word(U4 w, int port) {
  const int k = (port / 16) % 4;
  return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// The level drawn from softmax of a port's logits (level 4 r + i in c[r][i],
// r < R, L1 levels): the first level whose cumulative softmax weight exceeds
// u times the total, i.e. the inverse of the distribution function at u.  The
// weights are 2^(z log2 e - zmax log2 e) (one fused multiply-add each); the
// running sums kept as they are formed are the cumulative weights.
__device__ __forceinline__ int sample_level(const f32x4 (&c)[kPolR], int R, int L1, float u) {
  constexpr float kLog2e = 1.44269504088896341f;
  float zmax = c[0][0];  // level 0 always exists
#pragma unroll
  for (int r = 0; r < kPolR; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (r < R && 4 * r + i < L1) zmax = c[r][i] > zmax ? c[r][i] : zmax;
  const float zs = zmax * kLog2e;
  float cum[kPolR][4], tot = 0.f;
#pragma unroll
  for (int r = 0; r < kPolR; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool in = r < R && 4 * r + i < L1;
      tot += in ? __builtin_amdgcn_exp2f(__builtin_fmaf(c[r][i], kLog2e, -zs)) : 0.f;
      cum[r][i] = tot;
    }
  const float target = u * tot;
  int lev = 0;
#pragma unroll
  for (int r = 0; r < kPolR; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) lev += (r < R && 4 * r + i < L1 - 1 && cum[r][i] <= target) ? 1 : 0;
  return lev;
}

}  // namespace
}  // namespace cx
