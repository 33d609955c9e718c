// Search-window network (an addition to the paper's method, which sizes its
// hit search from the covariance): 27 inputs (the predicted state and its 21
// covariance entries) -> 64 -> GELU -> 64 -> GELU -> 2, softplus head times
// a per-output scale, giving the half-width of the hit window as an arc at
// the layer radius (cm) and in z (cm).  Weights and the activations that feed
// products are BF16; every product runs on the matrix cores
// (v_mfma_f32_16x16x32_bf16) and accumulates in FP32.
//
// A wave evaluates 64 rows at once (one per lane): the rows of the wave are
// four 16-row tiles; layer 1 (K = 32, the 27 inputs padded), layer 2
// (K = 64) and the head (N padded 2 -> 16) each run over the four tiles with
// their weights held in registers, through one 64 x 72 BF16 LDS buffer.
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
// BF16 weights after the header (offsets in bf16 elements): W1 [64][32]
// (inputs padded 27 -> 32 with zeros), W2 [64][64], W3 [16][64] (rows 2..15
// zero), W2T [64][64] (W2 transposed, for the backward pass)
#define KFMLP_W1 0
#define KFMLP_W2 (64 * 32)
#define KFMLP_W3 (64 * 32 + 64 * 64)
#define KFMLP_W2T (64 * 32 + 64 * 64 + 16 * 64)
#define KFMLP_WEIGHTS (64 * 32 + 64 * 64 + 16 * 64 + 64 * 64)
#define KFMLP_BLOCK_BYTES (KFMLP_HEADER_FLOATS * 4 + KFMLP_WEIGHTS * 2)
// trainable parameters (FP32 master vector): W1 [64][27], b1 [64], W2 [64][64],
// b2 [64], W3 [2][64], b3 [2]
#define KFMLP_P_W1 0
#define KFMLP_P_B1 (64 * 27)
#define KFMLP_P_W2 (KFMLP_P_B1 + 64)
#define KFMLP_P_B2 (KFMLP_P_W2 + 64 * 64)
#define KFMLP_P_W3 (KFMLP_P_B2 + 64)
#define KFMLP_P_B3 (KFMLP_P_W3 + 2 * 64)
#define KFMLP_NPARAM (KFMLP_P_B3 + 2)
// one row of training data: 27 features, 2 labels, then seed, layer, slot
#define KFMLP_DUMP_ROW 32
// LDS row pitch of the activation buffer (bf16 elements; 64 + 8 padding)
#define KFMLP_PITCH 72
#define KFMLP_LDS_BYTES (64 * KFMLP_PITCH * 2)

namespace kfmlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// round to nearest bfloat16, ties to even (on gfx950 one v_cvt_pk_bf16_f32;
// the host sequence gives the same result for every finite value)
__host__ __device__ inline uint16_t f_to_bf16(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(uint16_t, (__bf16)f);
#else
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
#endif
}

__host__ __device__ inline float bf16_round(float f) { return bf16_to_f(f_to_bf16(f)); }

// erf(x) by Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26
// (after Hastings): 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p|x|),
// absolute error below 1.5e-7 (the activations are then rounded to BF16,
// whose resolution is 2^-8).  Branch-free; the caller passes exp(-x^2).
__device__ inline float erf_as(float x, float e) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.f + 0.3275911f * ax);
  float poly = 1.061405429f;
  poly = fmaf(poly, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  const float v = 1.f - poly * t * e;
  return copysignf(v, x);
}
// GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, and its derivative
// Phi(z) + z phi(z); exp(-z^2 / 2) serves both erf and phi.
__device__ inline float gelu(float z) {
  const float x = z * 0.70710678118654752f;
  return 0.5f * z * (1.f + erf_as(x, __expf(-x * x)));
}
__device__ inline float gelu_grad(float z) {
  const float x = z * 0.70710678118654752f;
  const float e = __expf(-x * x);
  return 0.5f * (1.f + erf_as(x, e)) + z * 0.39894228040143268f * e;
}
__device__ inline float softplus(float o) { return o > 30.f ? o : log1pf(__expf(o)); }
__device__ inline float sigmoid(float o) { return 1.f / (1.f + __expf(-o)); }

// 8 consecutive bf16 (16 bytes, 16-byte aligned) as an MFMA operand
__device__ inline bf16x8 load8(const uint16_t* p) {
  uint4 v = *(const uint4*)p;
  return __builtin_bit_cast(bf16x8, v);
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Operand layout of v_mfma_f32_16x16x32_bf16 (wave64), lane l:
//   A (16 x 32): row l % 16, k = 8 (l / 16) .. + 7
//   B (32 x 16): k = 8 (l / 16) .. + 7, column l % 16
//   C (16 x 16): rows 4 (l / 16) .. + 3, column l % 16
//
// Forward of the 64 rows of a wave, layer by layer over the wave's four
// 16-row tiles (each layer's weights are fetched once per forward).
// feature(k): this lane's raw feature k of 27 (its row is the lane index);
// buf: the wave's LDS buffer [64][KFMLP_PITCH] bf16, which holds the inputs
// (columns 0..31, the 27 standardised features padded with zeros), then the
// first hidden layer, then the second, each overwriting its own tile's rows
// after they have been read.  Writes the two widths (without kappa) of this
// lane's row into w.  Must be called by all 64 lanes.
template <typename Feature>
__device__ inline void wave_forward(const float* __restrict__ blk, uint16_t* buf, Feature feature, float w[2],
                                    float* o_out = nullptr) {
  const int lane = threadIdx.x & 63;
  const uint16_t* W = (const uint16_t*)(blk + KFMLP_HEADER_FLOATS);
  const int r16 = lane & 15, kq = lane >> 4;
  {
    uint16_t* row = buf + lane * KFMLP_PITCH;
#pragma unroll
    for (int k = 0; k < 27; ++k) row[k] = f_to_bf16((feature(k) - blk[KFMLP_OFF_MU + k]) * blk[KFMLP_OFF_ISD + k]);
#pragma unroll
    for (int k = 27; k < 32; ++k) row[k] = 0;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  // layer 1: Z1 = Xh W1^T (K = 32), 4 column tiles
  {
    bf16x8 b1[4];
    float bias[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      b1[nt] = load8(W + KFMLP_W1 + (nt * 16 + r16) * 32 + 8 * kq);
      bias[nt] = blk[KFMLP_OFF_B1 + nt * 16 + r16];
    }
    for (int mt = 0; mt < 4; ++mt) {
      uint16_t* tile = buf + (mt * 16) * KFMLP_PITCH;
      const bf16x8 a = load8(tile + r16 * KFMLP_PITCH + 8 * kq);
      f32x4 acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, b1[nt], f32x4{0.f, 0.f, 0.f, 0.f});
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          tile[(4 * kq + i) * KFMLP_PITCH + nt * 16 + r16] = f_to_bf16(gelu(acc[nt][i] + bias[nt]));
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  // layer 2: Z2 = H1 W2^T (K = 64 in two steps)
  {
    bf16x8 b2[4][2];
    float bias[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* wr = W + KFMLP_W2 + (nt * 16 + r16) * 64;
      b2[nt][0] = load8(wr + 8 * kq);
      b2[nt][1] = load8(wr + 32 + 8 * kq);
      bias[nt] = blk[KFMLP_OFF_B2 + nt * 16 + r16];
    }
    for (int mt = 0; mt < 4; ++mt) {
      uint16_t* tile = buf + (mt * 16) * KFMLP_PITCH;
      const bf16x8 a0 = load8(tile + r16 * KFMLP_PITCH + 8 * kq);
      const bf16x8 a1 = load8(tile + r16 * KFMLP_PITCH + 32 + 8 * kq);
      f32x4 acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        acc[nt] = mfma(a0, b2[nt][0], f32x4{0.f, 0.f, 0.f, 0.f});
        acc[nt] = mfma(a1, b2[nt][1], acc[nt]);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          tile[(4 * kq + i) * KFMLP_PITCH + nt * 16 + r16] = f_to_bf16(gelu(acc[nt][i] + bias[nt]));
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  // head: O = H2 W3^T (columns 0, 1 of a 16-wide tile)
  {
    const uint16_t* w3 = W + KFMLP_W3 + r16 * 64;
    const bf16x8 b30 = load8(w3 + 8 * kq), b31 = load8(w3 + 32 + 8 * kq);
    for (int mt = 0; mt < 4; ++mt) {
      uint16_t* tile = buf + (mt * 16) * KFMLP_PITCH;
      const bf16x8 a0 = load8(tile + r16 * KFMLP_PITCH + 8 * kq);
      const bf16x8 a1 = load8(tile + r16 * KFMLP_PITCH + 32 + 8 * kq);
      f32x4 acc = mfma(a0, b30, f32x4{0.f, 0.f, 0.f, 0.f});
      acc = mfma(a1, b31, acc);
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      // lanes holding columns 0 and 1 of rows 4kq..4kq+3 park the head in
      // the first two floats of those rows (as raw bits, 4 halves)
      if (r16 < 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t bits = __float_as_uint(acc[i]);
          uint16_t* dst = tile + (4 * kq + i) * KFMLP_PITCH + 2 * r16;
          dst[0] = (uint16_t)bits;
          dst[1] = (uint16_t)(bits >> 16);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  const uint16_t* src = buf + lane * KFMLP_PITCH;
  float head[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) head[j] = __uint_as_float((uint32_t)src[2 * j] | ((uint32_t)src[2 * j + 1] << 16));
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float o = head[j] + blk[KFMLP_OFF_B3 + j];
    if (o_out) o_out[j] = o;
    w[j] = blk[KFMLP_OFF_SCALE + j] * softplus(o);
  }
}

}  // namespace kfmlp
