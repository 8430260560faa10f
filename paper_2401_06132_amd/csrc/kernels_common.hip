// Element-wise kernels shared by every element type.
#include "fr_kernels.h"

namespace fr {

// RK4 stage update (double precision for both library precisions).
//   mode 1 (first stage): acc = u0 + a k;  ust = u0 + b k
//   mode 0 (middle)     : acc += a k;      ust = u0 + b k
//   mode 2 (last)       : ust = acc + a k   (ust may alias u0)
__global__ void rk_stage_kernel(int64_t n, const double* __restrict__ u0, const double* __restrict__ k,
                                double* __restrict__ acc, double* ust, double a, double b, int mode) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = k[i];
    if (mode == 2) {
      ust[i] = acc[i] + a * ki;
    } else {
      const double u = u0[i];
      acc[i] = (mode == 1 ? u : acc[i]) + a * ki;
      ust[i] = u + b * ki;
    }
  }
}

hipError_t rk_stage(int64_t n, const double* u0, const double* k, double* acc, double* ust, double a, double b,
                    int mode, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(rk_stage_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, u0, k, acc, ust, a, b, mode);
  return hipGetLastError();
}

}  // namespace fr
