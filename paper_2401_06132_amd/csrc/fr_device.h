// Device-side physics shared by the fused and plain kernels: point-wise
// inviscid and viscous fluxes (eqs. fluxe, fluxv), the LDG common solution
// (eq. FR-conu) and the common normal interface flux (eq. FR-comm_flux,
// Rusanov + LDG), in the reference-state form: the energy slot holds
// E' = E - pref/(gamma-1), the momentum flux carries p' = p - pref and the
// energy flux v (E' + p' + gamma pref/(gamma-1)) = v (E + p).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fr {

template <typename R>
struct Gas {
  R gamma, gm1, mu, muh;  // muh = mu gamma / Pr  (c_p grad T = gamma grad e)
  R pref, eref, href;     // reference pressure, pref/(gamma-1), gamma pref/(gamma-1)
  R beta, tau;            // LDG parameters
};

template <typename R>
__device__ __forceinline__ R rcp(R x) {
  return R(1) / x;
}
// single precision: the hardware reciprocal (1 ulp), well inside the FP32
// path's rounding budget; double precision keeps the correctly rounded division
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// orders global memory, which makes every barrier wait for all outstanding
// global loads and stores of the wave; kernels whose global data is never
// exchanged between the waves of a workgroup use this one so that prefetched
// loads stay in flight across barriers.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Physical flux f = f^e - f^v at one point.  u: 5 conserved (reference
// form), q[d][v]: physical gradients d/dx_d of the conserved variables.
// f[d][v]: component d of the flux of variable v.
template <typename R>
__device__ __forceinline__ void point_flux(const R u[5], const R q[3][5], const Gas<R>& g, R f[3][5]) {
  const R rho = u[0], ir = rcp(rho);
  const R v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const R pp = g.gm1 * (u[4] - R(0.5) * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
  const R H = u[4] + pp + g.href;
  // velocity gradient gv[d][i] = d v_i / d x_d
  R gv[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < 3; ++i) gv[d][i] = (q[d][1 + i] - v[i] * q[d][0]) * ir;
  const R div = gv[0][0] + gv[1][1] + gv[2][2];
  const R et = (u[4] + g.eref) * ir;  // total energy per unit mass
  R ge[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    ge[d] = (q[d][4] - et * q[d][0]) * ir - (v[0] * gv[d][0] + v[1] * gv[d][1] + v[2] * gv[d][2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = g.mu * (gv[d][i] + gv[i][d]);
    t[d] -= (R(2) / R(3)) * g.mu * div;
    f[d][0] = u[1 + d];
#pragma unroll
    for (int i = 0; i < 3; ++i) f[d][1 + i] = u[1 + d] * v[i] - t[i];
    f[d][1 + d] += pp;
    f[d][4] = v[d] * H - (v[0] * t[0] + v[1] * t[1] + v[2] * t[2] + g.muh * ge[d]);
  }
}

// Normal viscous flux n . f^v (momentum x,y,z and energy; the mass
// component is zero) at one point.
template <typename R>
__device__ __forceinline__ void normal_viscous(const R u[5], const R q[3][5], const R n[3], const Gas<R>& g,
                                               R V[4]) {
  const R rho = u[0], ir = rcp(rho);
  const R v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  R gv[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < 3; ++i) gv[d][i] = (q[d][1 + i] - v[i] * q[d][0]) * ir;
  const R div = gv[0][0] + gv[1][1] + gv[2][2];
  const R et = (u[4] + g.eref) * ir;
  R tn[3] = {0, 0, 0}, hn = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R ge = (q[d][4] - et * q[d][0]) * ir - (v[0] * gv[d][0] + v[1] * gv[d][1] + v[2] * gv[d][2]);
    hn += n[d] * g.muh * ge;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R t = g.mu * (gv[d][i] + gv[i][d]);
      if (i == d) t -= (R(2) / R(3)) * g.mu * div;
      tn[i] += n[d] * t;
    }
  }
  V[0] = tn[0];
  V[1] = tn[1];
  V[2] = tn[2];
  V[3] = v[0] * tn[0] + v[1] * tn[1] + v[2] * tn[2] + hn;
}

// Common normal flux w.r.t. the unit normal n of the L side (per unit area):
//   F = 1/2 (f^e_L + f^e_R).n + 1/2 s (uL - uR)          (Rusanov)
//       - [(1/2 + beta) VL - (1/2 - beta) VR]            (LDG, VR = n_R . f^v_R)
//       + tau (uL - uR)                                   (penalty)
// with s = max(|vL.n| + cL, |vR.n| + cR).  Both sides of a pair evaluate the
// same expression on the same inputs, so the two results are bitwise equal.
template <typename R>
__device__ __forceinline__ void common_flux(const R uL[5], const R uR[5], const R VL[4], const R VR[4],
                                            const R n[3], const Gas<R>& g, R F[5]) {
  R fl[5], fr[5], sl, sr;
  {
    const R ir = rcp(uL[0]);
    const R vn = (uL[1] * n[0] + uL[2] * n[1] + uL[3] * n[2]) * ir;
    const R pp = g.gm1 * (uL[4] - R(0.5) * (uL[1] * uL[1] + uL[2] * uL[2] + uL[3] * uL[3]) * ir);
    fl[0] = uL[0] * vn;
    fl[1] = uL[1] * vn + pp * n[0];
    fl[2] = uL[2] * vn + pp * n[1];
    fl[3] = uL[3] * vn + pp * n[2];
    fl[4] = vn * (uL[4] + pp + g.href);
    sl = fabs(vn) + sqrt(g.gamma * (pp + g.pref) * ir);
  }
  {
    const R ir = rcp(uR[0]);
    const R vn = (uR[1] * n[0] + uR[2] * n[1] + uR[3] * n[2]) * ir;
    const R pp = g.gm1 * (uR[4] - R(0.5) * (uR[1] * uR[1] + uR[2] * uR[2] + uR[3] * uR[3]) * ir);
    fr[0] = uR[0] * vn;
    fr[1] = uR[1] * vn + pp * n[0];
    fr[2] = uR[2] * vn + pp * n[1];
    fr[3] = uR[3] * vn + pp * n[2];
    fr[4] = vn * (uR[4] + pp + g.href);
    sr = fabs(vn) + sqrt(g.gamma * (pp + g.pref) * ir);
  }
  const R s = sl > sr ? sl : sr;
  const R a = R(0.5) * s + g.tau;
  const R bl = R(0.5) + g.beta, br = R(0.5) - g.beta;
  F[0] = R(0.5) * (fl[0] + fr[0]) + a * (uL[0] - uR[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    F[1 + k] = R(0.5) * (fl[1 + k] + fr[1 + k]) + a * (uL[1 + k] - uR[1 + k]) - (bl * VL[k] - br * VR[k]);
}

// The two parts of common_flux, for surface-flux anti-aliasing, where the
// nonlinear Rusanov part is evaluated at the face quadrature points and the
// part that is linear in the two sides' values at the flux points:
//   rusanov_flux : 1/2 (f^e_L + f^e_R).n + 1/2 s (uL - uR)
//   linear_flux  : tau (uL - uR) - [(1/2 + beta) VL - (1/2 - beta) VR]
template <typename R>
__device__ __forceinline__ void euler_normal(const R u[5], const R n[3], const Gas<R>& g, R f[5], R& s) {
  const R ir = rcp(u[0]);
  const R vn = (u[1] * n[0] + u[2] * n[1] + u[3] * n[2]) * ir;
  const R pp = g.gm1 * (u[4] - R(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * ir);
  f[0] = u[0] * vn;
  f[1] = u[1] * vn + pp * n[0];
  f[2] = u[2] * vn + pp * n[1];
  f[3] = u[3] * vn + pp * n[2];
  f[4] = vn * (u[4] + pp + g.href);
  s = fabs(vn) + sqrt(g.gamma * (pp + g.pref) * ir);
}

template <typename R>
__device__ __forceinline__ void rusanov_flux(const R uL[5], const R uR[5], const R n[3], const Gas<R>& g, R F[5]) {
  R fl[5], fr[5], sl, sr;
  euler_normal(uL, n, g, fl, sl);
  euler_normal(uR, n, g, fr, sr);
  const R a = R(0.5) * (sl > sr ? sl : sr);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = R(0.5) * (fl[v] + fr[v]) + a * (uL[v] - uR[v]);
}

template <typename R>
__device__ __forceinline__ void linear_flux(const R uL[5], const R uR[5], const R VL[4], const R VR[4],
                                            const Gas<R>& g, R F[5]) {
  const R bl = R(0.5) + g.beta, br = R(0.5) - g.beta;
  F[0] = g.tau * (uL[0] - uR[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k) F[1 + k] = g.tau * (uL[1 + k] - uR[1 + k]) - (bl * VL[k] - br * VR[k]);
}

// Per-slot face record shared by the fused kernels.
struct FaceRec {
  int32_t nbr;   // paired slot
  int32_t info;  // (permutation id << 1) | is_left
};

}  // namespace fr
