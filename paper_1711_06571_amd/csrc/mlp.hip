// Training and inference kernels of the search-window network (kfmlp.h):
// forward, hand-written backward of the asymmetric quantile loss, and Adam on
// FP32 master weights with BF16 working copies.  The 64-wide products run on
// the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation); the
// two-column head, its weight gradient and the bias gradients use the VALU.
//
// Loss per row and output: 20 * max(0, d - w) + max(0, w - d), d = |offset
// of the true hit|, w = scale * softplus(o); mean over rows and outputs.
// Gradients are reduced deterministically: each 64-row block writes its own
// partial gradient, a second kernel sums the partials in block order.
#include <stdint.h>

#include "kfhost.h"
#include "kfmlp.h"

using namespace kfmlp;

namespace {

constexpr float kMissWeight = 20.f;
constexpr int P = KFMLP_PITCH;

__device__ inline void store_bf16_tile_rows(uint16_t* buf, int row0, int col, const f32x4& v) {
  const int kq = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) buf[(row0 + 4 * kq + i) * P + col] = f_to_bf16(v[i]);
}

// transposed store: buf[col][row0 + 4kq .. + 3]
__device__ inline void store_bf16_tile_cols(uint16_t* buf, int row0, int col, const f32x4& v) {
  const int kq = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) buf[col * P + row0 + 4 * kq + i] = f_to_bf16(v[i]);
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One block = one wave = 64 rows.  Writes the block's partial gradient of
// the summed loss (not yet divided by 2N) and the summed loss.
__global__ void __launch_bounds__(64) grad_kernel(const float* __restrict__ blk, const float* __restrict__ rows,
                                                  int n, float* __restrict__ partial) {
  __shared__ __align__(16) uint16_t XT[32 * P];    // inputs, [k][row]
  __shared__ __align__(16) uint16_t XR[64 * P];    // inputs, [row][k]; later dZ1 [unit][row]
  __shared__ __align__(16) uint16_t H1R[64 * P];   // [row][unit]
  __shared__ __align__(16) uint16_t H1T[64 * P];   // [unit][row]
  __shared__ __align__(16) uint16_t H2R[64 * P];   // [row][unit]
  __shared__ __align__(16) uint16_t DZR[64 * P];   // dZ2 [row][unit]
  __shared__ __align__(16) uint16_t DZT[64 * P];   // dZ2 [unit][row]
  __shared__ float G[64 * 2];                      // dL/do per row
  const int lane = threadIdx.x;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row = blockIdx.x * 64 + lane;
  const bool valid = row < n;
  const uint16_t* W = (const uint16_t*)(blk + KFMLP_HEADER_FLOATS);
  float* out = partial + (size_t)blockIdx.x * (KFMLP_NPARAM + 1);

  // inputs
  float d[2] = {0.f, 0.f};
  {
    const float* src = rows + (size_t)(valid ? row : 0) * KFMLP_DUMP_ROW;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const float v = valid ? (src[k] - blk[KFMLP_OFF_MU + k]) * blk[KFMLP_OFF_ISD + k] : 0.f;
      const uint16_t b = f_to_bf16(v);
      XR[lane * P + k] = b;
      XT[k * P + lane] = b;
    }
#pragma unroll
    for (int k = 27; k < 32; ++k) { XR[lane * P + k] = 0; XT[k * P + lane] = 0; }
    d[0] = valid ? src[27] : 0.f;
    d[1] = valid ? src[28] : 0.f;
  }
  __syncthreads();
  // forward, keeping the pre-activations in registers (tile layout)
  f32x4 z1[4][4], z2[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const bf16x8 a = load8(XR + (mt * 16 + r16) * P + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      z1[mt][nt] = mfma(a, load8(W + KFMLP_W1 + (nt * 16 + r16) * 32 + 8 * kq), f32x4{0.f, 0.f, 0.f, 0.f});
      const float b1 = blk[KFMLP_OFF_B1 + nt * 16 + r16];
#pragma unroll
      for (int i = 0; i < 4; ++i) z1[mt][nt][i] += b1;
      f32x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = gelu(z1[mt][nt][i]);
      store_bf16_tile_rows(H1R, mt * 16, nt * 16 + r16, h);
      store_bf16_tile_cols(H1T, mt * 16, nt * 16 + r16, h);
    }
  }
  __syncthreads();
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const bf16x8 a0 = load8(H1R + (mt * 16 + r16) * P + 8 * kq);
    const bf16x8 a1 = load8(H1R + (mt * 16 + r16) * P + 32 + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* wr = W + KFMLP_W2 + (nt * 16 + r16) * 64;
      f32x4 acc = mfma(a0, load8(wr + 8 * kq), f32x4{0.f, 0.f, 0.f, 0.f});
      acc = mfma(a1, load8(wr + 32 + 8 * kq), acc);
      const float b2 = blk[KFMLP_OFF_B2 + nt * 16 + r16];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += b2;
      z2[mt][nt] = acc;
      f32x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = gelu(acc[i]);
      store_bf16_tile_rows(H2R, mt * 16, nt * 16 + r16, h);
    }
  }
  __syncthreads();
  // head, in FP32 from the BF16 activations of this lane's row
  float o[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float s = 0.f;
    for (int k = 0; k < 64; ++k) s += bf16_to_f(W[KFMLP_W3 + j * 64 + k]) * bf16_to_f(H2R[lane * P + k]);
    o[j] = s + blk[KFMLP_OFF_B3 + j];
  }
  float loss = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float w = blk[KFMLP_OFF_SCALE + j] * softplus(o[j]);
    const float gw = w > d[j] ? 1.f : (w < d[j] ? -kMissWeight : 0.f);
    loss += valid ? kMissWeight * fmaxf(0.f, d[j] - w) + fmaxf(0.f, w - d[j]) : 0.f;
    G[lane * 2 + j] = valid ? gw * blk[KFMLP_OFF_SCALE + j] * sigmoid(o[j]) : 0.f;
  }
  __syncthreads();
  // head gradients: dW3[j][k] = sum_r G[r][j] H2[r][k] (lane = k), db3
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float s = 0.f;
    for (int r = 0; r < 64; ++r) s += G[r * 2 + j] * bf16_to_f(H2R[r * P + lane]);
    out[KFMLP_P_W3 + j * 64 + lane] = s;
    const float gb = wave_sum(G[lane * 2 + j]);
    if (lane == 0) out[KFMLP_P_B3 + j] = gb;
  }
  // dZ2 = (G W3) * gelu'(Z2), tile layout; bias gradient db2
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int col = nt * 16 + r16;
    const float w3a = bf16_to_f(W[KFMLP_W3 + col]), w3b = bf16_to_f(W[KFMLP_W3 + 64 + col]);
    float bsum = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 dz;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = mt * 16 + 4 * kq + i;
        dz[i] = (G[r * 2] * w3a + G[r * 2 + 1] * w3b) * gelu_grad(z2[mt][nt][i]);
        bsum += dz[i];
      }
      store_bf16_tile_rows(DZR, mt * 16, col, dz);
      store_bf16_tile_cols(DZT, mt * 16, col, dz);
    }
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (kq == 0) out[KFMLP_P_B2 + col] = bsum;
  }
  __syncthreads();
  // dW2[j][k] = sum_r dZ2[r][j] H1[r][k]
  for (int mt = 0; mt < 4; ++mt) {
    const bf16x8 a0 = load8(DZT + (mt * 16 + r16) * P + 8 * kq);
    const bf16x8 a1 = load8(DZT + (mt * 16 + r16) * P + 32 + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* b = H1T + (nt * 16 + r16) * P;
      f32x4 acc = mfma(a0, load8(b + 8 * kq), f32x4{0.f, 0.f, 0.f, 0.f});
      acc = mfma(a1, load8(b + 32 + 8 * kq), acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[KFMLP_P_W2 + (mt * 16 + 4 * kq + i) * 64 + nt * 16 + r16] = acc[i];
    }
  }
  // dH1 = dZ2 W2, dZ1 = dH1 * gelu'(Z1) -> XR reused as dZ1 [unit][row]
  uint16_t* DZ1T = XR;
  __syncthreads();
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const bf16x8 a0 = load8(DZR + (mt * 16 + r16) * P + 8 * kq);
    const bf16x8 a1 = load8(DZR + (mt * 16 + r16) * P + 32 + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* b = W + KFMLP_W2T + (nt * 16 + r16) * 64;
      f32x4 acc = mfma(a0, load8(b + 8 * kq), f32x4{0.f, 0.f, 0.f, 0.f});
      acc = mfma(a1, load8(b + 32 + 8 * kq), acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] *= gelu_grad(z1[mt][nt][i]);
      z1[mt][nt] = acc;  // now dZ1
      store_bf16_tile_cols(DZ1T, mt * 16, nt * 16 + r16, acc);
    }
  }
  // db1
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    float bsum = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) bsum += z1[mt][nt][i];
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (kq == 0) out[KFMLP_P_B1 + nt * 16 + r16] = bsum;
  }
  __syncthreads();
  // dW1[j][k] = sum_r dZ1[r][j] Xh[r][k], k < 27
  for (int mt = 0; mt < 4; ++mt) {
    const bf16x8 a0 = load8(DZ1T + (mt * 16 + r16) * P + 8 * kq);
    const bf16x8 a1 = load8(DZ1T + (mt * 16 + r16) * P + 32 + 8 * kq);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const uint16_t* b = XT + (nt * 16 + r16) * P;
      f32x4 acc = mfma(a0, load8(b + 8 * kq), f32x4{0.f, 0.f, 0.f, 0.f});
      acc = mfma(a1, load8(b + 32 + 8 * kq), acc);
      const int k = nt * 16 + r16;
      if (k < 27) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[KFMLP_P_W1 + (mt * 16 + 4 * kq + i) * 27 + k] = acc[i];
      }
    }
  }
  const float ls = wave_sum(loss);
  if (lane == 0) out[KFMLP_NPARAM] = ls;
}

// grad[p] = scale * sum over blocks (fixed order); the last entry is the loss
__global__ void reduce_kernel(const float* __restrict__ partial, int nblk, float scale, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > KFMLP_NPARAM) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * (KFMLP_NPARAM + 1) + p];
  grad[p] = s * scale;
}

// Adam (Kingma and Ba) on the FP32 master vector; refreshes the block's BF16
// weights (W2 also transposed and permuted, W3 permuted) and FP32 biases.
__global__ void adam_kernel(float* __restrict__ blk, float* __restrict__ master, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ grad, float bc1, float bc2, float lr,
                            float beta1, float beta2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= KFMLP_NPARAM) return;
  const float gr = grad[p];
  const float mm = beta1 * m[p] + (1.f - beta1) * gr;
  const float vv = beta2 * v[p] + (1.f - beta2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / bc1, vh = vv / bc2;
  const float val = master[p] - lr * mh / (sqrtf(vh) + eps);
  master[p] = val;
  uint16_t* W = (uint16_t*)(blk + KFMLP_HEADER_FLOATS);
  if (p < KFMLP_P_B1) {
    const int j = p / 27, k = p % 27;
    W[KFMLP_W1 + j * 32 + k] = f_to_bf16(val);
  } else if (p < KFMLP_P_W2) {
    blk[KFMLP_OFF_B1 + (p - KFMLP_P_B1)] = val;
  } else if (p < KFMLP_P_B2) {
    const int q = p - KFMLP_P_W2, j = q / 64, k = q % 64;
    const uint16_t b = f_to_bf16(val);
    W[KFMLP_W2 + j * 64 + k] = b;
    W[KFMLP_W2T + k * 64 + j] = b;
    W[KFMLP_W2P + kfmlp_packed_index(j, k)] = b;
  } else if (p < KFMLP_P_W3) {
    blk[KFMLP_OFF_B2 + (p - KFMLP_P_B2)] = val;
  } else if (p < KFMLP_P_B3) {
    const int q = p - KFMLP_P_W3, j = q / 64, k = q % 64;
    const uint16_t b = f_to_bf16(val);
    W[KFMLP_W3 + j * 64 + k] = b;
    W[KFMLP_W3P + kfmlp_packed_index(j, k)] = b;
  } else {
    blk[KFMLP_OFF_B3 + (p - KFMLP_P_B3)] = val;
  }
}

__global__ void __launch_bounds__(64) infer_kernel(const float* __restrict__ blk, const float* __restrict__ rows,
                                                   int n, float* __restrict__ out, float* __restrict__ out_o) {
  __shared__ __align__(16) uint16_t buf[KFMLP_LDS_BYTES / 2];
  const int lane = threadIdx.x;
  const int row = blockIdx.x * 64 + lane;
  float x[27];
  const float* src = rows + (size_t)(row < n ? row : 0) * KFMLP_DUMP_ROW;
#pragma unroll
  for (int k = 0; k < 27; ++k) x[k] = row < n ? src[k] : 0.f;
  float w[2], o[2];
  wave_forward(blk, buf, [&](int k) { return x[k]; }, row < n, w, o);
  if (row < n) {
    const float kap = blk[KFMLP_OFF_KAPPA];
    out[(size_t)row * 2] = kap * w[0];
    out[(size_t)row * 2 + 1] = kap * w[1];
    if (out_o) {
      out_o[(size_t)row * 2] = o[0];
      out_o[(size_t)row * 2 + 1] = o[1];
    }
  }
}

}  // namespace

extern "C" size_t kf_mlp_block_bytes(void) { return KFMLP_BLOCK_BYTES; }

extern "C" size_t kf_mlp_grad_workspace_bytes(int32_t n_rows) {
  if (n_rows < 0) return 0;
  const size_t nblk = ((size_t)n_rows + 63) / 64;
  return (nblk > 0 ? nblk : 1) * (KFMLP_NPARAM + 1) * sizeof(float);
}

extern "C" int kf_mlp_forward(const void* block, int32_t n_rows, const float* rows, float* out, float* out_logits,
                              void* stream) {
  if (!block || n_rows < 0) return KF_E_INVALID_ARG;
  if (n_rows == 0) return KF_OK;
  if (!rows || !out) return KF_E_INVALID_ARG;
  const int nblk = (n_rows + 63) / 64;
  hipLaunchKernelGGL(infer_kernel, dim3(nblk), dim3(64), 0, (hipStream_t)stream, (const float*)block, rows, n_rows,
                     out, out_logits);
  return kf_check_launch();
}

extern "C" int kf_mlp_grad(const void* block, int32_t n_rows, const float* rows, float* grad, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!block || n_rows < 1 || !rows || !grad) return KF_E_INVALID_ARG;
  const size_t need = kf_mlp_grad_workspace_bytes(n_rows);
  if (!ws || ws_bytes < need) return KF_E_WORKSPACE;
  const int nblk = (n_rows + 63) / 64;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(grad_kernel, dim3(nblk), dim3(64), 0, s, (const float*)block, rows, n_rows, (float*)ws);
  if (int rc = kf_check_launch()) return rc;
  const float scale = 1.f / (2.f * (float)n_rows);
  hipLaunchKernelGGL(reduce_kernel, dim3((KFMLP_NPARAM + 1 + 255) / 256), dim3(256), 0, s, (const float*)ws, nblk,
                     scale, grad);
  return kf_check_launch();
}

extern "C" int kf_mlp_adam(void* block, float* master, float* m, float* v, const float* grad, int32_t step,
                           float lr, float beta1, float beta2, float eps, void* stream) {
  if (!block || !master || !m || !v || !grad || step < 1) return KF_E_INVALID_ARG;
  const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((KFMLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     (float*)block, master, m, v, grad, bc1, bc2, lr, beta1, beta2, eps);
  return kf_check_launch();
}
