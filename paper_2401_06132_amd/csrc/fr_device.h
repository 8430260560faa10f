// Device-side physics shared by the fused and plain kernels: point-wise
// inviscid and viscous fluxes (eqs. fluxe, fluxv), the LDG common solution
// (eq. FR-conu) and the common normal interface flux (eq. FR-comm_flux,
// Rusanov + LDG), in the reference-state form: the density slot holds
// rho' = rho - rho0, the energy slot E' = E - pref/(gamma-1), the momentum
// flux carries p' = p - pref and the energy flux v (E + p).
//
// Energy-flux split (fused kernels, rho0 > 0 on affine meshes).  With
// kap = gamma pref / ((gamma - 1) rho0) the energy flux is written exactly as
//   v (E + p) = v (E' + p' - kap rho') + kap (rho v),
// so the part evaluated point-wise is O(1) instead of O(gamma pref/(gamma-1))
// (~250 at Mach 0.1).  The remainder kap (rho v) is linear in the state: its
// DG divergence kap L(rho v) is formed in double precision from the state
// itself (the disu kernels), L being the central DG divergence of the mass
// flux.  The mass equation then needs no point-wise flux at all: its
// residual is L(rho v) plus the lifted dissipation of the common flux.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fr {

template <typename R>
struct Gas {
  R gamma, gm1, mu, muh;  // muh = mu gamma / Pr  (c_p grad T = gamma grad e)
  R pref, eref, href;     // reference pressure, pref/(gamma-1), gamma pref/(gamma-1)
  R beta, tau;            // LDG parameters
  R rho0;                 // reference density (rho = u[0] + rho0)
  R kap, hc0;             // split energy flux: H = E' + p' + hc0 - kap rho'
                          // (kap = href/rho0, hc0 = 0; unsplit: kap = 0, hc0 = href)
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
// f[d][v]: component d of the flux of variable v; the energy component is
// the split form (v H with H = E' + p' + hc0 - kap rho').
template <typename R>
__device__ __forceinline__ void point_flux(const R u[5], const R q[3][5], const Gas<R>& g, R f[3][5]) {
  const R rho = u[0] + g.rho0, ir = rcp(rho);
  const R v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const R pp = g.gm1 * (u[4] - R(0.5) * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
  const R H = u[4] + pp + g.hc0 - g.kap * u[0];
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
  const R rho = u[0] + g.rho0, ir = rcp(rho);
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

// Normal inviscid flux f^e . n and the wave-speed bound |v.n| + c at one
// point (reference-state form; the energy component in the split form).
template <typename R>
__device__ __forceinline__ void euler_normal(const R u[5], const R n[3], const Gas<R>& g, R f[5], R& s) {
  const R ir = rcp(u[0] + g.rho0);
  const R mn = u[1] * n[0] + u[2] * n[1] + u[3] * n[2];
  const R vn = mn * ir;
  const R pp = g.gm1 * (u[4] - R(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * ir);
  f[0] = mn;
  f[1] = u[1] * vn + pp * n[0];
  f[2] = u[2] * vn + pp * n[1];
  f[3] = u[3] * vn + pp * n[2];
  f[4] = vn * (u[4] + pp + g.hc0 - g.kap * u[0]);
  s = fabs(vn) + sqrt(g.gamma * (pp + g.pref) * ir);
}

// Common normal flux w.r.t. the unit normal n of the L side (per unit area):
//   F = 1/2 (f^e_L + f^e_R).n + 1/2 s (uL - uR)          (Rusanov)
//       - [(1/2 + beta) VL - (1/2 - beta) VR]            (LDG, VR = n_R . f^v_R)
//       + tau (uL - uR)                                   (penalty)
// with s = max(|vL.n| + cL, |vR.n| + cR).  Used by the unsplit plain path
// (kap = 0).
template <typename R>
__device__ __forceinline__ void common_flux(const R uL[5], const R uR[5], const R VL[4], const R VR[4],
                                            const R n[3], const Gas<R>& g, R F[5]) {
  R fl[5], fr[5], sl, sr;
  euler_normal(uL, n, g, fl, sl);
  euler_normal(uR, n, g, fr, sr);
  const R s = sl > sr ? sl : sr;
  const R a = R(0.5) * s + g.tau;
  const R bl = R(0.5) + g.beta, br = R(0.5) - g.beta;
  F[0] = R(0.5) * (fl[0] + fr[0]) + a * (uL[0] - uR[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    F[1 + k] = R(0.5) * (fl[1 + k] + fr[1 + k]) + a * (uL[1 + k] - uR[1 + k]) - (bl * VL[k] - br * VR[k]);
}

// The fused kernels' interface flux at one own flux point, for the own side:
// D such that mag * D is the own element's transformed common normal flux
// (eq. FR-comm_flux; mag = own area factor).
//   uo, un : own and neighbour states; j = un - uo, formed from the stored
//            face base and deviations, so it keeps the digits that uo and un
//            lose to their O(1) magnitude;
//   nL     : the L side's unit normal; left: this side is L.
// Momentum and energy: sg F with sg = +-1 and F as in common_flux (with
// uL - uR taken from j), so the two sides' values are bitwise opposite.
// LIN: the central part of the mass flux and the linear part kap (rho v) of
// the energy flux are handed to the double-precision L(rho v) of the volume
// term; here remains only their strong-form interface term
// 1/2 (m_nbr - m_own) . n_own (the own-trace part is inside L), and the mass
// flux keeps its dissipation.
template <typename R, bool LIN>
__device__ __forceinline__ void face_flux(const R uo[5], const R un[5], const R j[5], const R Vo[4], const R Vn[4],
                                          const R nL[3], bool left, const Gas<R>& g, R D[5]) {
  R fo[5], fn[5], so, sn;
  euler_normal(uo, nL, g, fo, so);
  euler_normal(un, nL, g, fn, sn);
  const R a = R(0.5) * (so > sn ? so : sn) + g.tau;
  const R sg = left ? R(1) : R(-1);
  const R bo = left ? R(0.5) + g.beta : R(0.5) - g.beta;  // weight of the own viscous flux
  const R bn = left ? R(0.5) - g.beta : R(0.5) + g.beta;
#pragma unroll
  for (int k = 1; k < 5; ++k) {
    // uL - uR = -sg j; the L side's viscous flux enters with (1/2 + beta)
    const R jl = left ? -j[k] : j[k];
    const R vv = left ? bo * Vo[k - 1] - bn * Vn[k - 1] : bn * Vn[k - 1] - bo * Vo[k - 1];
    D[k] = sg * (R(0.5) * (left ? fo[k] + fn[k] : fn[k] + fo[k]) + a * jl - vv);
  }
  if constexpr (LIN) {
    const R jn = R(0.5) * sg * (j[1] * nL[0] + j[2] * nL[1] + j[3] * nL[2]);
    D[0] = jn - a * j[0];
    D[4] += g.kap * jn;
  } else {
    const R jl = left ? -j[0] : j[0];
    D[0] = sg * (R(0.5) * (left ? fo[0] + fn[0] : fn[0] + fo[0]) + a * jl);
  }
}

// Surface-flux anti-aliasing splits face_flux in two: the part linear in
// the two sides' values (penalty, LDG viscous flux, and with LIN the
// interface terms of L(rho v)), evaluated at the flux points, and the
// Rusanov part, evaluated at the face quadrature points from the L state
// and the jump jl = uL - uR interpolated there.
template <typename R, bool LIN>
__device__ __forceinline__ void face_flux_linear(const R j[5], const R Vo[4], const R Vn[4], const R nL[3],
                                                 bool left, const Gas<R>& g, R D[5]) {
  const R sg = left ? R(1) : R(-1);
  const R bo = left ? R(0.5) + g.beta : R(0.5) - g.beta;
  const R bn = left ? R(0.5) - g.beta : R(0.5) + g.beta;
#pragma unroll
  for (int k = 1; k < 5; ++k) {
    const R jl = left ? -j[k] : j[k];
    const R vv = left ? bo * Vo[k - 1] - bn * Vn[k - 1] : bn * Vn[k - 1] - bo * Vo[k - 1];
    D[k] = sg * (g.tau * jl - vv);
  }
  D[0] = -g.tau * j[0];
  if constexpr (LIN) {
    const R jn = R(0.5) * sg * (j[1] * nL[0] + j[2] * nL[1] + j[3] * nL[2]);
    D[0] += jn;
    D[4] += g.kap * jn;
  }
}

// Rusanov flux w.r.t. nL from the L state and jl = uL - uR: the mass
// component is the dissipation only when LIN (its central part is in L).
template <typename R, bool LIN>
__device__ __forceinline__ void rusanov_jump(const R uL[5], const R jl[5], const R n[3], const Gas<R>& g, R F[5]) {
  R uR[5], fl[5], fr[5], sl, sr;
#pragma unroll
  for (int v = 0; v < 5; ++v) uR[v] = uL[v] - jl[v];
  euler_normal(uL, n, g, fl, sl);
  euler_normal(uR, n, g, fr, sr);
  const R a = R(0.5) * (sl > sr ? sl : sr);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = (LIN && v == 0 ? R(0) : R(0.5) * (fl[v] + fr[v])) + a * jl[v];
}

// Per-slot face record shared by the fused kernels.
struct FaceRec {
  int32_t nbr;   // paired slot
  int32_t info;  // (permutation id << 1) | is_left
  int32_t npo;   // the paired slot's first point in the face arrays
  int32_t pad;
};

}  // namespace fr
