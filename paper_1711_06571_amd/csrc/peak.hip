// Practical vector peak of the device: long chains of fused multiply-adds,
// eight independent ones per lane so the pipeline never waits on a result.
// Measurement support for the roofline fractions the library reports; not
// part of the method.
#include "kfhost.h"

namespace {

template <typename T>
__global__ void __launch_bounds__(256) fma_kernel(int iters, T* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (T)(i + k) * (T)1e-7;
  const T m = (T)0.9999999, c = (T)1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if constexpr (sizeof(T) == 4)
        a[k] = __builtin_fmaf(a[k], m, c);
      else
        a[k] = __builtin_fma(a[k], m, c);
    }
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[i] = s;
}

}  // namespace

extern "C" int kf_peak_fma(int32_t arith, int32_t blocks, int32_t iters, void* out, void* stream) {
  if (blocks < 1 || iters < 1 || !out) return KF_E_INVALID_ARG;
  if (arith == KF_ARITH_F64)
    hipLaunchKernelGGL(fma_kernel<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, (double*)out);
  else if (arith == KF_ARITH_F32)
    hipLaunchKernelGGL(fma_kernel<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, (float*)out);
  else
    return KF_E_INVALID_ARG;
  return kf_check_launch();
}
