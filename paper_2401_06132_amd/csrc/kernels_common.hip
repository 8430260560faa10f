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

// Taylor-Green vortex (the paper's test case, section 6) at the solution
// points: v = (sin x cos y cos z, -cos x sin y cos z, 0),
// p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16, rho = p/p0 (rho0 = U0 = 1),
// E = p/(gamma-1) + rho |v|^2/2.  One thread per solution point.
__global__ void tgv_init_kernel(int64_t E, int nu, const double* __restrict__ geo, const double* __restrict__ ref,
                                double gamma, double p0, double* __restrict__ U) {
  const int64_t n = E * nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / nu;
    const int u = int(i - e * nu);
    const double* G = geo + 12 * e;
    const double* xi = ref + 3 * u;
    double x[3];
    for (int d = 0; d < 3; ++d) x[d] = G[d] + G[3 + 3 * d] * xi[0] + G[4 + 3 * d] * xi[1] + G[5 + 3 * d] * xi[2];
    const double sx = sin(x[0]), cx = cos(x[0]), sy = sin(x[1]), cy = cos(x[1]), cz = cos(x[2]);
    const double vx = sx * cy * cz, vy = -cx * sy * cz;
    const double p = p0 + (cos(2 * x[0]) + cos(2 * x[1])) * (cos(2 * x[2]) + 2.0) / 16.0;
    const double rho = p / p0;
    double* ue = U + e * 5 * nu + u;
    ue[0] = rho;
    ue[nu] = rho * vx;
    ue[2 * nu] = rho * vy;
    ue[3 * nu] = 0.0;
    ue[4 * nu] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
  }
}

hipError_t tgv_init(int64_t E, int nu, const double* geo, const double* ref, double gamma, double p0, double* U,
                    hipStream_t st) {
  int64_t blocks = (E * nu + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(tgv_init_kernel, dim3((unsigned)blocks), dim3(256), 0, st, E, nu, geo, ref, gamma, p0, U);
  return hipGetLastError();
}

// Fills the device's LDS with one value: workgroups of 32 KB each (five
// share a CU's 160 KB), twenty per CU, written through a volatile pointer so
// that the stores stay.  Kernels launched afterwards then find that value
// wherever they read LDS that they have not written: tests use it to show
// that no kernel depends on what earlier kernels left in LDS.
__global__ void __launch_bounds__(256) lds_fill_kernel(float v) {
  constexpr int N = 8192;
  __shared__ float buf[N];
  volatile float* b = buf;
  for (int i = threadIdx.x; i < N; i += 256) b[i] = v;
}

hipError_t lds_fill(float v, hipStream_t st) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (cus < 1) cus = 1;
  hipLaunchKernelGGL(lds_fill_kernel, dim3(20 * cus), dim3(256), 0, st, v);
  return hipGetLastError();
}

}  // namespace fr
