// Plain (unfused) FP64 path: the paper's kernel sequence of PyFR v1.11.0
// (section 3, figure NSkernelorder) with dense operator matrices
// (section 2.2) and every intermediate array in HBM.  It is the comparison
// point for the fused kernels.  The matrix-multiplication kernels are plain
// library GEMMs (rocBLAS dgemm over all (element, variable) columns); the
// point-wise kernels are hand-written.
//
//   1 disu          U^f  = M0 U
//   2 con_u         C    = (1/2 - beta) uL + (1/2 + beta) uR at every flux point
//   3 tgradpcoru    Q~   = (M4 - M6 M0) U
//   4 tgradcoru     Q~  += M6 C
//   5 gradcoru      Q    = J^-T Q~
//   6 gradcoru_fpts Q^f  = (I3 x M0) Q
//   7 gradcoru_qpts Q^q  = (I3 x M7) Q
//   8 qptsu         U^q  = M7 U
//   9 tdisf         F~^q = det J J^-1 f(U^q, Q^q)     (in place over Q^q)
//  10 tdivpcorf     R~   = (M1 - M3 M2) M9 F~^q
//  11 comm_flux     D~   = +-mag F(uL, uR, qL, qR, nL)
//  12 tdivtconf     R~  += M3 D~
//  13 negdivconf    R    = -R~ / det J
//
// With a reference density the energy flux is split exactly as in the fused
// kernels: v (E + p) = v (E' + p' - kap rho') + kap rho v.  Steps 9-12 carry
// the first part; the linear part adds kap L(rho v) to the volume residual
// (L = sum_d Lv_d (S m)_d, a GEMM on the transformed momentum at the
// solution points) and kap mag 1/2 (m_nbr - m_own) . n_own to the common
// energy flux.  The O(gamma pref/(gamma-1)) energy flux then never enters the
// dense (M1 - M3 M2) M9 product, whose long sums would round it at ~1e-12.
//
// Layouts: per element type, element-major: U [E][5][N_u] is the
// column-major matrix N_u x 5E; Q [E][5][3][N_u] is 3N_u x 5E (rows (d,s)) and
// also N_u x 15E; the same holds at flux and quadrature points.
#include <rocblas/rocblas.h>

#include <vector>

#include "fr_kernels.h"
#include "fr_plain.h"

namespace fr {

namespace {

__global__ void con_u_kernel(int64_t nftot, const double* __restrict__ Uf, double* __restrict__ Cf,
                             const PlainFace* __restrict__ fc, PlainTypes ty, double beta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nftot; i += (int64_t)gridDim.x * blockDim.x) {
    const int t = plain_type_of(ty, i);
    const int64_t li = i - ty.f0[t];
    const int64_t e = li / ty.nf[t], f = li - e * ty.nf[t];
    const PlainFace F = fc[i];
    const int tn = F.nbr_type;
    const int64_t ob = ty.off_f[t] + e * 5 * ty.nf[t] + f;
    const int64_t nb = ty.off_f[tn] + (int64_t)F.nbr_elem * 5 * ty.nf[tn] + F.nbr_fpt;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double uo = Uf[ob + v * ty.nf[t]], un = Uf[nb + v * ty.nf[tn]];
      Cf[ob + v * ty.nf[t]] =
          F.is_left ? (0.5 - beta) * uo + (0.5 + beta) * un : (0.5 - beta) * un + (0.5 + beta) * uo;
    }
  }
}

__global__ void gradcoru_kernel(int64_t E, int nu, double* __restrict__ Q, const double* __restrict__ jinv) {
  const int64_t n = E * 5 * nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ev = i / nu, s = i - ev * nu, e = ev / 5;
    double* q = Q + ev * 3 * nu + s;
    const double g0 = q[0], g1 = q[nu], g2 = q[2 * nu];
    const double* B = jinv + 9 * e;
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c * nu] = B[c] * g0 + B[3 + c] * g1 + B[6 + c] * g2;
  }
}

__global__ void tdisf_kernel(int64_t E, int nq, const double* __restrict__ Uq, double* __restrict__ Qq,
                             const double* __restrict__ jinv, const double* __restrict__ detj, Gas<double> g) {
  const int64_t n = E * nq;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / nq, q = i - e * nq;
    double u[5], qq[3][5], f[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = Uq[(e * 5 + v) * nq + q];
#pragma unroll
      for (int d = 0; d < 3; ++d) qq[d][v] = Qq[((e * 5 + v) * 3 + d) * nq + q];
    }
    point_flux(u, qq, g, f);
    const double* B = jinv + 9 * e;
    const double dj = detj[e];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        Qq[((e * 5 + v) * 3 + d) * nq + q] = dj * (B[3 * d] * f[0][v] + B[3 * d + 1] * f[1][v] + B[3 * d + 2] * f[2][v]);
  }
}

__global__ void comm_flux_kernel(int64_t nftot, const double* __restrict__ Uf,
                                 const double* __restrict__ Qf, double* __restrict__ Df,
                                 const PlainFace* __restrict__ fc, const double* __restrict__ fgeo, PlainTypes ty,
                                 Gas<double> g) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nftot; i += (int64_t)gridDim.x * blockDim.x) {
    const int t = plain_type_of(ty, i);
    const int64_t li = i - ty.f0[t];
    const int64_t e = li / ty.nf[t], f = li - e * ty.nf[t];
    const PlainFace F = fc[i];
    const int tn = F.nbr_type;
    const int64_t en = F.nbr_elem, fn = F.nbr_fpt;
    double uo[5], un[5], qo[3][5], qn[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      uo[v] = Uf[ty.off_f[t] + (e * 5 + v) * ty.nf[t] + f];
      un[v] = Uf[ty.off_f[tn] + (en * 5 + v) * ty.nf[tn] + fn];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        qo[d][v] = Qf[3 * ty.off_f[t] + ((e * 5 + v) * 3 + d) * ty.nf[t] + f];
        qn[d][v] = Qf[3 * ty.off_f[tn] + ((en * 5 + v) * 3 + d) * ty.nf[tn] + fn];
      }
    }
    const double nL[3] = {fgeo[4 * i], fgeo[4 * i + 1], fgeo[4 * i + 2]};
    const double nR[3] = {-nL[0], -nL[1], -nL[2]};
    const double mag = fgeo[4 * i + 3];
    double Vo[4], Vn[4], Fc[5];
    normal_viscous(uo, qo, F.is_left ? nL : nR, g, Vo);
    normal_viscous(un, qn, F.is_left ? nR : nL, g, Vn);
    if (F.is_left)
      common_flux(uo, un, Vo, Vn, nL, g, Fc);
    else
      common_flux(un, uo, Vn, Vo, nL, g, Fc);
    const double sc = F.is_left ? mag : -mag;
    double D[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) D[v] = sc * Fc[v];
    // the linear energy-flux part: its strong-form interface term
    const double* no = F.is_left ? nL : nR;
    D[4] += g.kap * mag * 0.5 * ((un[1] - uo[1]) * no[0] + (un[2] - uo[2]) * no[1] + (un[3] - uo[3]) * no[2]);
#pragma unroll
    for (int v = 0; v < 5; ++v) Df[ty.off_f[t] + (e * 5 + v) * ty.nf[t] + f] = D[v];
  }
}

__global__ void negdivconf_kernel(int64_t E, int nu, double* __restrict__ R, const double* __restrict__ detj) {
  const int64_t n = E * 5 * nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    R[i] = -R[i] / detj[i / (5 * nu)];
}

// rho' = rho - rho0, E' = E - pref/(gamma-1) (reference-state form) into a
// scratch copy of U
__global__ void refstate_kernel(int64_t E, int nu, const double* __restrict__ U, double* __restrict__ W, double eref,
                                double rho0) {
  const int64_t n = E * 5 * nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int v = int((i / nu) % 5);
    W[i] = v == 4 ? U[i] - eref : (v == 0 ? U[i] - rho0 : U[i]);
  }
}

// the transformed momentum (S m)_d = det J sum_c (J^-1)_dc m_c at the solution
// points: SM [E][3][N_u], the columns of the L(rho v) product
__global__ void sm_kernel(int64_t E, int nu, const double* __restrict__ W, double* __restrict__ SM,
                          const double* __restrict__ jinv, const double* __restrict__ detj) {
  const int64_t n = E * nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / nu, s = i - e * nu;
    const double* m = W + (e * 5 + 1) * nu + s;
    const double m0 = m[0], m1 = m[nu], m2 = m[2 * nu];
    const double* B = jinv + 9 * e;
    const double dj = detj[e];
#pragma unroll
    for (int d = 0; d < 3; ++d) SM[(e * 3 + d) * nu + s] = dj * (B[3 * d] * m0 + B[3 * d + 1] * m1 + B[3 * d + 2] * m2);
  }
}

dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 1 << 20) b = 1 << 20;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// host matrix product with extended-precision accumulation (composite
// operators are rounded to double once)
void mat_mul(const double* A, int M, int K, const double* B, int64_t N, double* C, double beta, double* out) {
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0;
      for (int k = 0; k < K; ++k) s += (long double)A[i * K + k] * (long double)B[k * N + j];
      out[i * N + j] = (double)((beta != 0 ? (long double)beta * C[i * N + j] : 0.0L) + s);
    }
}

void mat_mul_ld(const long double* A, int M, int K, const double* B, int64_t N, long double* out) {
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0;
      for (int k = 0; k < K; ++k) s += A[i * K + k] * (long double)B[k * N + j];
      out[i * N + j] = s;
    }
}

}  // namespace

// dense composite operators of one element type (row-major)
void build_plain_ops(const RefElem& r, PlainOps& o) {
  const int nu = r.nu, nf = r.nf, nq = r.nq;
  o.nu = nu;
  o.nf = nf;
  o.nq = nq;
  o.M0 = r.M0;
  o.M7 = r.M7;
  o.M3 = r.M3;
  // M6 = n_d M3 (rows (d, s)); G1 = M4 - M6 M0 (rows (d, s))
  o.M6.assign(3 * nu * nf, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < nu; ++s)
      for (int f = 0; f < nf; ++f) {
        int face = 0;
        while (face + 1 < r.nfaces && f >= r.face_start[face + 1]) ++face;
        o.M6[(d * nu + s) * nf + f] = r.face_normal[3 * face + d] * r.M3[s * nf + f];
      }
  std::vector<long double> M6ld(o.M6.begin(), o.M6.end()), M6M0(3 * nu * nu);
  mat_mul_ld(M6ld.data(), 3 * nu, nf, r.M0.data(), nu, M6M0.data());
  o.G1.assign(3 * nu * nu, 0.0);
  for (int k = 0; k < 3 * nu * nu; ++k) o.G1[k] = (double)((long double)r.Dg[k] - M6M0[k]);
  // LV = [Lv_0 | Lv_1 | Lv_2] (rows s, columns (d, u)): Lv_d = D_d (the strong
  // form plus the lift of the own trace); pyramids Ku_d + M3 n_d M0 (their
  // weak form plus the lift of the own trace)
  o.LV.assign((size_t)nu * 3 * nu, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < nu; ++s)
      for (int u = 0; u < nu; ++u) {
        long double acc;
        if (r.etype == 3) {
          acc = r.Ku[((size_t)d * nu + s) * nu + u];
          for (int f = 0; f < nf; ++f) {
            int face = 0;
            while (face + 1 < r.nfaces && f >= r.face_start[face + 1]) ++face;
            acc += (long double)r.M3[s * nf + f] * r.face_normal[3 * face + d] * r.M0[f * nu + u];
          }
        } else {
          acc = r.Dg[((size_t)d * nu + s) * nu + u];
        }
        o.LV[(size_t)s * 3 * nu + d * nu + u] = (double)acc;
      }
  // K = (M1 - M3 M2) M9: for component d, (Dg_d - M3 N_d M0) M8, columns (d, q).
  // Pyramids (space not closed under differentiation): the weak form AP_d.
  o.K.assign((size_t)nu * 3 * nq, 0.0);
  if (r.etype == 3) {
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < nu; ++s)
        for (int q = 0; q < nq; ++q) o.K[(size_t)s * 3 * nq + d * nq + q] = r.APd[((size_t)d * nu + s) * nq + q];
    return;
  }
  std::vector<long double> Ad(nu * nu), M3NM0(nu * nu), Kd(nu * nq), M3ld(r.M3.begin(), r.M3.end());
  std::vector<double> NM0(nf * nu);
  for (int d = 0; d < 3; ++d) {
    for (int f = 0; f < nf; ++f) {
      int face = 0;
      while (face + 1 < r.nfaces && f >= r.face_start[face + 1]) ++face;
      for (int u = 0; u < nu; ++u) NM0[f * nu + u] = r.face_normal[3 * face + d] * r.M0[f * nu + u];
    }
    mat_mul_ld(M3ld.data(), nu, nf, NM0.data(), nu, M3NM0.data());
    for (int k = 0; k < nu * nu; ++k) Ad[k] = (long double)r.Dg[(size_t)d * nu * nu + k] - M3NM0[k];
    mat_mul_ld(Ad.data(), nu, nu, r.M8.data(), nq, Kd.data());
    for (int s = 0; s < nu; ++s)
      for (int q = 0; q < nq; ++q) o.K[(size_t)s * 3 * nq + d * nq + q] = (double)Kd[s * nq + q];
  }
}

// C (M x N, col-major, leading dimension ldc) = alpha A B + beta C, A row-major
// (M x K), B col-major (K x N)
static rocblas_status gemm_ld(rocblas_handle h, const double* A, int M, int K, const double* B, int64_t N, double* C,
                              int64_t ldc, double alpha, double beta) {
  return rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, M, (rocblas_int)N, K, &alpha, A, K, B,
                       K, &beta, C, (rocblas_int)ldc);
}

static rocblas_status gemm(rocblas_handle h, const double* A, int M, int K, const double* B, int64_t N, double* C,
                           double beta) {
  // C (M x N, col-major) = A (M x K, row-major = col-major K x M, transposed) B (K x N col-major)
  const double one = 1.0;
  rocblas_status s = rocblas_status_success;
  const int64_t chunk = 1 << 30;  // rocblas_int columns per call
  for (int64_t c0 = 0; c0 < N && s == rocblas_status_success; c0 += chunk) {
    const int64_t nc = N - c0 < chunk ? N - c0 : chunk;
    s = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, M, (rocblas_int)nc, K, &one, A, K,
                      B + c0 * K, K, &beta, C + c0 * M, M);
  }
  return s;
}

hipError_t plain_rhs(PlainCtx& P, const double* U, double* du, hipStream_t st) {
  rocblas_handle h = (rocblas_handle)P.blas;
  if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorUnknown;
  const PlainTypes& ty = P.ty;
  const Gas<double>& g = P.gas;
  // reference-state copy of the state, then disu per type
  for (int t = 0; t < NTYPES; ++t) {
    if (!ty.E[t]) continue;
    const PlainOps& o = P.ops[t];
    const double* Ut = U + P.state_off[t];
    double* W = P.W + P.state_off[t];
    hipLaunchKernelGGL(refstate_kernel, grid_for(ty.E[t] * 5 * o.nu), dim3(256), 0, st, ty.E[t], o.nu, Ut, W, P.eref,
                       P.rho0);
    if (gemm(h, P.dM0[t], o.nf, o.nu, W, 5 * ty.E[t], P.Uf + ty.off_f[t], 0.0) != rocblas_status_success)
      return hipErrorUnknown;  // 1 disu
  }
  int64_t nftot = 0;
  for (int t = 0; t < NTYPES; ++t) nftot += ty.E[t] * ty.nf[t];
  hipLaunchKernelGGL(con_u_kernel, grid_for(nftot), dim3(256), 0, st, nftot, P.Uf, P.Cf, P.faces, ty,
                     P.beta);  // 2 con_u
  for (int t = 0; t < NTYPES; ++t) {
    if (!ty.E[t]) continue;
    const PlainOps& o = P.ops[t];
    const int64_t E = ty.E[t];
    const double* W = P.W + P.state_off[t];
    double* Q = P.Q + 3 * P.state_off[t];
    if (gemm(h, P.dG1[t], 3 * o.nu, o.nu, W, 5 * E, Q, 0.0) != rocblas_status_success) return hipErrorUnknown;  // 3
    if (gemm(h, P.dM6[t], 3 * o.nu, o.nf, P.Cf + ty.off_f[t], 5 * E, Q, 1.0) != rocblas_status_success)
      return hipErrorUnknown;  // 4 tgradcoru
    hipLaunchKernelGGL(gradcoru_kernel, grid_for(E * 5 * o.nu), dim3(256), 0, st, E, o.nu, Q, P.jinv[t]);  // 5
    if (gemm(h, P.dM0[t], o.nf, o.nu, Q, 15 * E, P.Qf + 3 * ty.off_f[t], 0.0) != rocblas_status_success)
      return hipErrorUnknown;  // 6 gradcoru_fpts
    if (gemm(h, P.dM7[t], o.nq, o.nu, Q, 15 * E, P.Qq, 0.0) != rocblas_status_success) return hipErrorUnknown;  // 7
    if (gemm(h, P.dM7[t], o.nq, o.nu, W, 5 * E, P.Uq, 0.0) != rocblas_status_success) return hipErrorUnknown;  // 8
    hipLaunchKernelGGL(tdisf_kernel, grid_for(E * o.nq), dim3(256), 0, st, E, o.nq, P.Uq, P.Qq, P.jinv[t], P.detj[t],
                       g);  // 9 tdisf
    if (gemm(h, P.dK[t], o.nu, 3 * o.nq, P.Qq, 5 * E, du + P.state_off[t], 0.0) != rocblas_status_success)
      return hipErrorUnknown;  // 10 tdivpcorf
    if (g.kap != 0.0) {
      // kap L(rho v) onto the energy rows (columns 5 e + 4 of N_u x 5E): the
      // transformed momentum into the (free) quadrature-point scratch first
      hipLaunchKernelGGL(sm_kernel, grid_for(E * o.nu), dim3(256), 0, st, E, o.nu, W, P.Uq, P.jinv[t], P.detj[t]);
      if (gemm_ld(h, P.dLV[t], o.nu, 3 * o.nu, P.Uq, E, du + P.state_off[t] + 4 * o.nu, 5 * o.nu, g.kap, 1.0) !=
          rocblas_status_success)
        return hipErrorUnknown;
    }
  }
  hipLaunchKernelGGL(comm_flux_kernel, grid_for(nftot), dim3(256), 0, st, nftot, P.Uf, P.Qf, P.Df, P.faces,
                     P.fgeo, ty, g);  // 11 comm_flux
  for (int t = 0; t < NTYPES; ++t) {
    if (!ty.E[t]) continue;
    const PlainOps& o = P.ops[t];
    double* R = du + P.state_off[t];
    if (gemm(h, P.dM3[t], o.nu, o.nf, P.Df + ty.off_f[t], 5 * ty.E[t], R, 1.0) != rocblas_status_success)
      return hipErrorUnknown;  // 12 tdivtconf
    hipLaunchKernelGGL(negdivconf_kernel, grid_for(ty.E[t] * 5 * o.nu), dim3(256), 0, st, ty.E[t], o.nu, R,
                       P.detj[t]);  // 13 negdivconf
  }
  return hipGetLastError();
}

bool plain_create_handle(void** h) {
  rocblas_handle hh;
  if (rocblas_create_handle(&hh) != rocblas_status_success) return false;
  *h = hh;
  return true;
}

void plain_destroy_handle(void* h) {
  if (h) rocblas_destroy_handle((rocblas_handle)h);
}

}  // namespace fr
