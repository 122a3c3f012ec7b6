// Measurement utility: an FP64 fused multiply-add loop that runs at the
// VALU issue rate, so the achievable FP64 throughput of the device can be
// measured beside the kernels of the path (it computes nothing of the method).
//
// Each thread runs 8 independent multiply-add chains of `iters` steps on
// values that stay bounded (x <- x * a + b with |a| < 1) and stores their sum,
// so the compiler cannot drop the loop: 16 * iters flops per thread.
#include <hip/hip_runtime.h>

#include "fdl.h"

namespace {

__global__ __launch_bounds__(256) void k_fma64_probe(double* __restrict__ out, int iters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = 1e-3 * (double)(t + i);
  const double a = 0.999999, b = 1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = fma(x[i], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  out[t] = s;
}

}  // namespace

extern "C" int fdl_fma64_probe(double* out_dev, int blocks, int iters, void* stream) {
  if (!out_dev || blocks < 1 || iters < 1) return FDL_EINVAL;
  hipLaunchKernelGGL(k_fma64_probe, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), out_dev,
                     iters);
  return hipGetLastError() == hipSuccess ? FDL_OK : FDL_EHIP;
}
