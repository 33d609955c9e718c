// Search-window network (an addition to the paper's method, which sizes its
// hit search from the covariance): 27 inputs (the predicted state and its 21
// covariance entries) -> 64 -> GELU -> 64 -> GELU -> 2, softplus head times
// a per-output scale, giving the half-width of the hit window as an arc at
// the layer radius (cm) and in z (cm).  Weights and the activations that feed
// products are BF16; every product runs on the matrix cores
// (v_mfma_f32_16x16x32_bf16) and accumulates in FP32.
//
// A wave evaluates up to 64 rows at once (one per lane) in 16-row tiles, in
// transposed form: every product is W x X^T (weights as the A operand, the
// tile's samples as the 16 columns).  Then the outputs a lane holds for a
// sample (4 units of each 16-unit block) are exactly the K values it must
// supply for that sample to the next layer, once the next layer's weights
// are stored with their K index permuted to match (W2P, W3P): the hidden
// activations never leave registers; only the inputs pass through LDS.
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
#define KFMLP_OFF_GATE 189
#define KFMLP_HEADER_FLOATS 192
// BF16 weights after the header (offsets in bf16 elements): W1 [64][32]
// (inputs padded 27 -> 32 with zeros), W2 [64][64], W3 [16][64] (rows 2..15
// zero), W2T [64][64] (W2 transposed, for the backward pass), then W2 and W3
// in the operand order of the inference (kfmlp_perm): W2P [4][2][16][32],
// W3P [2][16][32]
#define KFMLP_W1 0
#define KFMLP_W2 (64 * 32)
#define KFMLP_W3 (64 * 32 + 64 * 64)
#define KFMLP_W2T (64 * 32 + 64 * 64 + 16 * 64)
#define KFMLP_W2P (KFMLP_W2T + 64 * 64)
#define KFMLP_W3P (KFMLP_W2P + 64 * 64)
#define KFMLP_WEIGHTS (KFMLP_W3P + 16 * 64)
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
// one row of training data: 27 features, 2 labels, the plain arc and z
// half-widths of the candidate's window, then (seed << 8) | (layer << 3) | slot
#define KFMLP_DUMP_ROW 32
// LDS row pitch of the activation buffer (bf16 elements; 64 + 8 padding)
#define KFMLP_PITCH 72
#define KFMLP_LDS_BYTES (64 * KFMLP_PITCH * 2)

namespace kfmlp {

// Hidden unit supplied as K slot j (0..7) of lane group kq (0..3) in K step
// ks (0..1) of a 64-wide hidden input: the lane's layer outputs for units
// 16 ot + 4 kq + i (ot = 2 ks + j / 4, i = j % 4).
__host__ __device__ constexpr int kfmlp_perm(int ks, int kq, int j) {
  return (2 * ks + (j >> 2)) * 16 + 4 * kq + (j & 3);
}
// Position in W2P of W2[out][unit] (and in W3P of W3[out][unit], ot = 0).
__host__ __device__ constexpr int kfmlp_packed_index(int out, int unit) {
  return ((((out >> 4) * 2 + (unit >> 5)) * 16 + (out & 15)) * 32) + ((unit & 15) >> 2) * 8 +
         ((unit >> 4) & 1) * 4 + (unit & 3);
}

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

// A wave-uniform pointer made opaque to the optimiser (the block pointer is
// the same in every lane; taken as a scalar, reads through it can be
// neither hoisted out of a loop nor moved across the call site)
__device__ inline const float* opaque_uniform(const float* p) {
  const uint64_t u = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  const float* q = (const float*)(((uint64_t)hi << 32) | lo);
  asm volatile("" : "+s"(q));
  return q;
}

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
// Forward of the active rows of a wave, in two steps.  wave_stage numbers
// the active lanes in lane order (rank) and writes their standardised rows
// into the first ceil(n/16) tiles of buf, the wave's LDS buffer [64]
// [KFMLP_PITCH] bf16 (columns 0..31, inputs padded with zeros); feature(k)
// is this lane's raw feature k of 27.  It returns the mask of active lanes.
// wave_tiles runs the network over those tiles only (none when no lane is
// active) and gives each active lane the head outputs of its row.  Both must
// be called by all 64 lanes together.
template <typename Feature>
__device__ inline uint64_t wave_stage(const float* __restrict__ blk, uint16_t* buf, Feature feature, bool active) {
  const uint64_t act = __ballot(active);
  if (active) {
    const int rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    // standardisation read through an opaque copy of the pointer: hoisted out
    // of a caller's loop, its 54 constants would occupy registers throughout
    const float* hk = opaque_uniform(blk);
    uint16_t* row = buf + rank * KFMLP_PITCH;
#pragma unroll
    for (int k = 0; k < 27; ++k) row[k] = f_to_bf16((feature(k) - hk[KFMLP_OFF_MU + k]) * hk[KFMLP_OFF_ISD + k]);
#pragma unroll
    for (int k = 27; k < 32; ++k) row[k] = 0;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  return act;
}

__device__ inline void wave_tiles(const float* __restrict__ blk, const uint16_t* buf, uint64_t act, float out[2]) {
  const int lane = threadIdx.x & 63;
  const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
  const int ntile = (__popcll(act) + 15) >> 4;
  const int r16 = lane & 15, kq = lane >> 4;
  float head[2] = {0.f, 0.f};
  for (int mt = 0; mt < ntile; ++mt) {
    // the weights and biases are read afresh in every tile (from cache): the
    // opaque copy of the block pointer keeps the compiler from hoisting them
    // out of the loop, where they would hold about 90 registers for the whole
    // loop inside kernels that are already short of them
    const float* bk = opaque_uniform(blk);
    const uint16_t* W = (const uint16_t*)(bk + KFMLP_HEADER_FLOATS);
    // samples 16 mt .. 16 mt + 15 (rows past the active count hold stale
    // values; each sample is its own column, so they touch only their own
    // outputs, which nobody reads): this lane supplies features
    // 8 kq .. 8 kq + 7 of sample 16 mt + r16
    const bf16x8 x = load8(buf + (16 * mt + r16) * KFMLP_PITCH + 8 * kq);
    // Each stage produces one 8-unit K slice of the next layer's input from
    // two 16-unit output blocks, so few accumulators are live at a time.
    // layer 1 (K = 32): units 16 ot + 4 kq + i of sample 16 mt + r16, for
    // ot = 2 ks, 2 ks + 1, give slice ks of the layer-2 input
    bf16x8 a1[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const f32x4 hA = mfma(load8(W + KFMLP_W1 + ((2 * ks) * 16 + r16) * 32 + 8 * kq), x, f32x4{0.f, 0.f, 0.f, 0.f});
      const f32x4 hB =
          mfma(load8(W + KFMLP_W1 + ((2 * ks + 1) * 16 + r16) * 32 + 8 * kq), x, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a1[ks][i] = (__bf16)gelu(hA[i] + bk[KFMLP_OFF_B1 + (2 * ks) * 16 + 4 * kq + i]);
        a1[ks][4 + i] = (__bf16)gelu(hB[i] + bk[KFMLP_OFF_B1 + (2 * ks + 1) * 16 + 4 * kq + i]);
      }
    }
    // layer 2 (K = 64 in two steps, W2 in permuted order), each slice of its
    // output feeding the head (outputs padded 2 -> 16) at once
    f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int oa = 2 * ks, ob = 2 * ks + 1;
      f32x4 hA = mfma(load8(W + KFMLP_W2P + ((oa * 2 + 0) * 16 + r16) * 32 + 8 * kq), a1[0], f32x4{0.f, 0.f, 0.f, 0.f});
      hA = mfma(load8(W + KFMLP_W2P + ((oa * 2 + 1) * 16 + r16) * 32 + 8 * kq), a1[1], hA);
      f32x4 hB = mfma(load8(W + KFMLP_W2P + ((ob * 2 + 0) * 16 + r16) * 32 + 8 * kq), a1[0], f32x4{0.f, 0.f, 0.f, 0.f});
      hB = mfma(load8(W + KFMLP_W2P + ((ob * 2 + 1) * 16 + r16) * 32 + 8 * kq), a1[1], hB);
      bf16x8 a2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a2[i] = (__bf16)gelu(hA[i] + bk[KFMLP_OFF_B2 + oa * 16 + 4 * kq + i]);
        a2[4 + i] = (__bf16)gelu(hB[i] + bk[KFMLP_OFF_B2 + ob * 16 + 4 * kq + i]);
      }
      o = mfma(load8(W + KFMLP_W3P + (ks * 16 + r16) * 32 + 8 * kq), a2, o);
    }
    // outputs 0 and 1 of sample 16 mt + c land in lane c (kq = 0), elements
    // 0 and 1; the lane of rank r takes sample r from lane r % 16 in tile r / 16
    const float s0 = __shfl(o[0], rank & 15, 64), s1 = __shfl(o[1], rank & 15, 64);
    if ((rank >> 4) == mt) {
      head[0] = s0;
      head[1] = s1;
    }
  }
  __builtin_amdgcn_wave_barrier();
  out[0] = head[0] + blk[KFMLP_OFF_B3 + 0];
  out[1] = head[1] + blk[KFMLP_OFF_B3 + 1];
}

// Both steps, and the widths (without kappa) of an active lane's row in w
// (head outputs in o_out); an inactive lane's are left untouched.
template <typename Feature>
__device__ inline void wave_forward(const float* __restrict__ blk, uint16_t* buf, Feature feature, bool active,
                                    float w[2], float* o_out = nullptr) {
  const uint64_t act = wave_stage(blk, buf, feature, active);
  if (act == 0) return;
  float o[2];
  wave_tiles(blk, buf, act, o);
  if (active) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (o_out) o_out[j] = o[j];
      w[j] = blk[KFMLP_OFF_SCALE + j] * softplus(o[j]);
    }
  }
}

}  // namespace kfmlp
