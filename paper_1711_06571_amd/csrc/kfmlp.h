// Search-window network (an addition to the paper's method): 27 inputs (the
// predicted state and the 21 covariance entries) -> 64 -> GELU -> 64 -> GELU
// -> 2, softplus head times a per-output scale, giving the half-width of the
// hit window as an arc at the layer radius (cm) and in z (cm).  Weights and
// the activations that feed products are BF16; products accumulate in FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// FP32 header of the device block (offsets in floats)
#define KFMLP_OFF_MU 0
#define KFMLP_OFF_ISD 27
#define KFMLP_OFF_B1 54
#define KFMLP_OFF_B2 118
#define KFMLP_OFF_B3 182
#define KFMLP_OFF_SCALE 184
#define KFMLP_OFF_KAPPA 186
#define KFMLP_OFF_FLOOR 187
#define KFMLP_HEADER_FLOATS 192
// BF16 weights after the header (offsets in bf16 elements from the weights
// start): W1 [64][32] (input padded 27 -> 32 with zeros), W2 [64][64],
// W3 [16][64] (rows 2..15 zero)
#define KFMLP_W1 0
#define KFMLP_W2 (64 * 32)
#define KFMLP_W3 (64 * 32 + 64 * 64)
#define KFMLP_WEIGHTS (64 * 32 + 64 * 64 + 16 * 64)
#define KFMLP_BLOCK_BYTES (KFMLP_HEADER_FLOATS * 4 + KFMLP_WEIGHTS * 2)
// one row of the training-data dump: 27 features, 2 labels, seed, layer, slot
#define KFMLP_DUMP_ROW 32

namespace kfmlp {

__host__ __device__ inline float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// round to nearest bfloat16, ties to even
__host__ __device__ inline uint16_t f_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_round(float f) { return bf16_to_f(f_to_bf16(f)); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float softplus(float o) { return o > 30.f ? o : log1pf(__expf(o)); }

// One lane evaluates the network for its own candidate (FP32 accumulation in
// index order).  Returns kappa * widths.
template <typename T>
__device__ __noinline__ void mlp_window_lane(const float* __restrict__ blk, const T Xp[6], const T Pp[21], float w[2]) {
  const uint16_t* W = (const uint16_t*)(blk + KFMLP_HEADER_FLOATS);
  float xh[27];
  for (int k = 0; k < 6; ++k) xh[k] = bf16_round(((float)Xp[k] - blk[KFMLP_OFF_MU + k]) * blk[KFMLP_OFF_ISD + k]);
  for (int k = 0; k < 21; ++k)
    xh[6 + k] = bf16_round(((float)Pp[k] - blk[KFMLP_OFF_MU + 6 + k]) * blk[KFMLP_OFF_ISD + 6 + k]);
  float h1[64];
  for (int j = 0; j < 64; ++j) {
    float s = 0.f;
    for (int k = 0; k < 27; ++k) s += bf16_to_f(W[KFMLP_W1 + j * 32 + k]) * xh[k];
    h1[j] = bf16_round(gelu(s + blk[KFMLP_OFF_B1 + j]));
  }
  float o0 = 0.f, o1 = 0.f;
  for (int j = 0; j < 64; ++j) {
    float s = 0.f;
    for (int k = 0; k < 64; ++k) s += bf16_to_f(W[KFMLP_W2 + j * 64 + k]) * h1[k];
    const float h2 = bf16_round(gelu(s + blk[KFMLP_OFF_B2 + j]));
    o0 += bf16_to_f(W[KFMLP_W3 + 0 * 64 + j]) * h2;
    o1 += bf16_to_f(W[KFMLP_W3 + 1 * 64 + j]) * h2;
  }
  const float kap = blk[KFMLP_OFF_KAPPA];
  w[0] = kap * blk[KFMLP_OFF_SCALE] * softplus(o0 + blk[KFMLP_OFF_B3]);
  w[1] = kap * blk[KFMLP_OFF_SCALE + 1] * softplus(o1 + blk[KFMLP_OFF_B3 + 1]);
}

}  // namespace kfmlp
