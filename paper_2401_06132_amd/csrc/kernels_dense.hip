// Fused flux-reconstruction kernels for tetrahedra and pyramids (gfx950).
//
// Tetrahedra and pyramids have no tensor-product structure: the paper's sum
// factorisation does not apply to them (sections 1 and 4.1), so every
// operator is a dense per-element matrix: M0 (N_f x N_u), the corrected-
// gradient operator [D_d | n_d M3] (N_u x (N_u + N_f)), M7 (N_q x N_u), the
// projection-divergence AP_d = -Mass^-1 Dq_d^T W_q (N_u x N_q; the weak form
// of (M1 - M3 M2) M9 for tetrahedra, as for the other types; for pyramids,
// whose rational space is not closed under differentiation, the divergence
// by definition) and the lifting M3 (N_u x N_f).  Without anti-aliasing
// tetrahedra take the strong form sum_d D_d F~_d - M3 (M2 F~) at the solution
// points, pyramids the weak form Ku_d = AP_d M7 (N_u x N_u).  The kernel
// groups are those of the hexahedral and prism kernels: disu | volume group
// | interface group.
//
// Dense products C = A B on the vector units run one operator row per
// thread: the row is read from the device table into registers (in chunks
// of KC entries, so long rows at p = 4 stay within the register budget) and
// applied to the columns of one element held in LDS.  In the volume and
// interface kernels the lanes of a wave work on rows of the same element,
// so every LDS read is a broadcast; the disu kernel runs the element index
// fastest instead, so that the lanes of a wave share an operator row.  At
// p >= 3 the volume group runs its products on the matrix cores
// (dense_volume_mf).
//
// Reference tetrahedron {xi, eta, zeta >= -1, xi + eta + zeta <= -1};
// faces 0..3 = zeta = -1, eta = -1, xi = -1, the slanted face.  Reference
// pyramid: base [-1,1]^2 at zeta = -1 (face 0, GL(n)^2 points), apex (0,0,1),
// triangles 1..4.  A face slot holds the face's values (the N_t triangle
// nodes, or the n^2 base points; slot stride (p+1)^2).
#include <type_traits>

#include "fr_device.h"
#include "fr_kernels.h"

namespace fr {

// ET: 2 tetrahedron, 3 pyramid
template <int ET, int P>
struct DenseCfg {
  static constexpr bool PYR = ET == 3;
  static constexpr int n = P + 1;
  static constexpr int NU = PYR ? n * (n + 1) * (2 * n + 1) / 6 : n * (n + 1) * (n + 2) / 6;  // solution points
  static constexpr int NFACE = PYR ? 5 : 4;
  static constexpr int NTN = n * (n + 1) / 2;            // points per triangle
  static constexpr int NB = PYR ? n * n : 0;              // points on the pyramid base
  static constexpr int NF = NB + 4 * NTN;                 // flux points
  static constexpr int NQ = n * n * n;                    // quadrature points
  static constexpr int NFPS = n * n;                      // permutation table stride
  // face arrays: an element's faces are stored in flux-point order with
  // their own point counts; face f has fsz(f) points
  __host__ __device__ static constexpr int fsz(int f) { return (PYR && f == 0) ? NB : NTN; }
  static constexpr int KG = NU + NF;                      // gradient operator row
  // device table (working precision), row-major blocks
  static constexpr int O_M0 = 0;                 // [NF][NU]
  static constexpr int O_G = O_M0 + NF * NU;     // [3][NU][KG]
  static constexpr int O_M7 = O_G + 3 * NU * KG; // [NQ][NU]
  static constexpr int O_AP = O_M7 + NQ * NU;    // [3][NU][NQ]
  static constexpr int O_M3 = O_AP + 3 * NU * NQ;  // [NU][NF]
  static constexpr int O_N = O_M3 + NU * NF;       // [NFACE][3] reference unit normals
  static constexpr int O_KU = O_N + 3 * NFACE;      // pyramids: [3][NU][NU] AP_d M7
  // matrix-core (FP32) copies of the volume operators: 16-row tiles, k in
  // steps of 4, each (tile, step) a block of 64 values in lane order (lane l:
  // row 16 mt + l % 16, column 4 ks + l / 16), zero padded
  static constexpr int KSU = (NU + 3) / 4, KSF = (NF + 3) / 4, KSQ = (NQ + 3) / 4;
  static constexpr int MTF = (NF + 15) / 16, MTG = (3 * NU + 15) / 16, MTQ = (NQ + 15) / 16, MTU = (NU + 15) / 16;
  static constexpr int O_PM0 = O_KU + (PYR ? 3 * NU * NU : 0);  // M0: MTF x KSU
  static constexpr int O_PG = O_PM0 + MTF * KSU * 64;            // [D_d | n_d M3]: MTG x (KSU + KSF)
  static constexpr int O_PM7 = O_PG + MTG * (KSU + KSF) * 64;    // M7: MTQ x KSU
  static constexpr int O_PAP = O_PM7 + MTQ * KSU * 64;           // [AP_0 | AP_1 | AP_2]: MTU x 3 KSQ
  // without anti-aliasing the divergence of the flux at the solution points,
  // [K0_0 | K0_1 | K0_2]: MTU x 3 KSU, K0_d = D_d - M3 n_d M0 for tetrahedra
  // (the strong form (M1 - M3 M2) in one operator), Ku_d for pyramids
  static constexpr int O_PK0 = O_PAP + MTU * 3 * KSQ * 64;
  static constexpr int SIZE = O_PK0 + MTU * 3 * KSU * 64;
  // LDS per element of the volume kernel: state + gradients [20][NU]
  // (later the partial divergences [3][5][NU]), neighbour values then jumps
  // [5][NF], the transformed flux at the quadrature points [3][5][FQS]
  static constexpr int FQS = NQ + 1;  // odd stride: the three components' rows hit different banks
  static constexpr int SZ_X = 20 * NU, SZ_J = 5 * NF, SZ_F = 15 * FQS;
  static constexpr int PER_ELEM = SZ_X + SZ_J + SZ_F;
  // LDS per element of the matrix-core volume kernel: state + gradients
  // [20][NU], then one region holding in turn the jumps [5][NF], the face
  // values [NF][LDW] and the quadrature values, later the transformed flux,
  // [NQ][LDW].  Rows of 20 values, 16-byte aligned: a thread reads its row as
  // 16-byte words (five per row, consecutive rows 80 bytes apart, so a
  // wave's reads spread over the banks), and the matrix-core outputs, four
  // rows apart per lane group, land 320 bytes apart (disjoint banks).  The
  // transformed flux F~_d of variable v (1..4) overwrites the row's columns
  // 4 d + v - 1.
  // (each region padded so that reads of the zero-weighted k-step padding stay
  // inside it: the matrix-core products read B without bounds checks)
  static constexpr int LDW = 20;
  // the row layouts hold NF face rows, and the products read 4 KSQ
  // quadrature rows and 4 KSU solution-point rows (the rows past NQ and NU
  // are zero padding)
  static constexpr int U2A = 5 * NF + 4, U2B = LDW * NF, U2C = LDW * 4 * (KSQ > KSU ? KSQ : KSU);
  static constexpr int SZ_U2 = U2A > U2B ? (U2A > U2C ? U2A : U2C) : (U2B > U2C ? U2B : U2C);
  // the padding after the state and gradients that the last column's
  // k range reads (a multiple of 4 values, so that U2 stays 16-byte aligned)
  static constexpr int XPAD = (4 * KSU - NU + 3) / 4 * 4;
  static constexpr int PE_MF = SZ_X + XPAD + SZ_U2;
  // without anti-aliasing there are no quadrature rows: U2 holds the jumps,
  // the NF face rows and the 4 KSU solution-point rows of the flux
  static constexpr int U2D = LDW * 4 * KSU;
  static constexpr int SZ_U2_NOAA = U2A > U2B ? (U2A > U2D ? U2A : U2D) : (U2B > U2D ? U2B : U2D);
  static constexpr int PE_MF_NOAA = SZ_X + XPAD + SZ_U2_NOAA;
  // face f and point t within the face of flux point fp
  // (branch-free: with a select here the compiler kept the operator loops of
  // both cases live in the callers, tripling their registers)
  __host__ __device__ static constexpr int face_of(int fp) {
    const int g = fp - NB, base = g >> 31;  // -1 on the base, 0 on a triangle
    return (int(PYR) + g / NTN) & ~base;
  }
  __host__ __device__ static constexpr int point_of(int fp) {
    const int g = fp - NB, base = g >> 31;
    return (fp & base) | ((g % NTN) & ~base);
  }
};

// acc[c] += sum_k A[k] B[c * ldb + k] (k < K, c < NC): a row A of a dense
// operator (device memory, read KC entries at a time) against NC columns of
// one element in LDS.  The scheduling barrier after each column stops the
// compiler from hoisting the LDS reads of all columns ahead of their use,
// which spilled registers for the longer rows.
template <int K, int NC, typename R>
__device__ __forceinline__ void row_cols(const R* __restrict__ A, const R* B, int ldb, R (&acc)[NC]) {
  constexpr int KC = 32;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += KC) {
    R a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k)
      if (k0 + k < K) a[k] = A[k0 + k];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k0 + k < K) acc[c] += a[k] * B[c * ldb + k0 + k];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Single precision works relative to a per-element base state u_b (the
// base of the element's first face): the volume kernels hold the state as
// u - u_b, so the linear operators (face values, gradients, quadrature
// values) round the variation within the element instead of the O(1)
// values, and add u_b back where the point-wise physics needs u.  Likewise
// the constant transformed flux Fc[d][v] = det J sum_c (J^-1)_dc f^e_c(u_b)
// (v = 1..4) is subtracted from the transformed flux before the divergence
// product.  The constant's own
// divergence is minus the lift of its reference normal component (a
// constant flux has zero DG divergence; the free-stream pins fix this
// identity for both element types), so the interface kernel subtracts
// n^ . Fc from the transformed common flux: the sum is unchanged.
template <typename R>
__device__ __forceinline__ void const_flux(const float* __restrict__ ub, const R* met, const Gas<R>& g, R* out) {
  R u[5], q[3][5] = {}, f[3][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = ub[v];
  point_flux(u, q, g, f);  // zero gradient: the inviscid flux
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int v = 1; v < 5; ++v)
      out[d * 4 + v - 1] = met[9] * (met[3 * d] * f[0][v] + met[3 * d + 1] * f[1][v] + met[3 * d + 2] * f[2][v]);
}

// ----------------------------------------------------------------- disu
// Double-precision operators of the disu kernel, stored after the working-
// precision table: M0 and the operator of the mass-flux divergence,
//   L(rho v) = sum_d Lv_d (S m)_d,  Lv_d = D_d (tetrahedra: the strong form
//   (M1 - M3 M2) plus the lift of the own trace), Lv_d = Ku_d + M3 n_d M0
//   (pyramids: their weak form plus the lift of the own trace).
template <int ET, int P>
struct DenseDisu {
  using C = DenseCfg<ET, P>;
  static constexpr int O_M0 = 0, O_LV = C::NF * C::NU, SIZE = O_LV + 3 * C::NU * C::NU;
};

// byte offset of the double-precision block behind the table
template <int ET, int P>
constexpr size_t dense_disu_offset(size_t rs) {
  return (rs * DenseCfg<ET, P>::SIZE + 255) / 256 * 256;
}

// Group 1 (eq. FR-disu) in double precision, as for hexahedra and prisms:
// single precision stores a float base per face (its value at the face's
// first flux point) and the deviations.  LIN: L(rho v) to row 0 of the
// volume residual.
template <int ET, int P, typename R, int EB, int NT>
__global__ void __launch_bounds__(NT) dense_disu(const Seg sg, const bool from_ust, const double* __restrict__ ops,
                                               const double eref, const double rho0, const bool lin) {
  using C = DenseCfg<ET, P>;
  using DD = DenseDisu<ET, P>;
  constexpr int NU = C::NU, NF = C::NF, NFACE = C::NFACE;
  constexpr bool FB = sizeof(R) == 4;
  __shared__ double sU[EB * 5 * NU];
  __shared__ double sF[EB * 5 * NF];
  __shared__ double sS[EB][9];
  const int e0 = blockIdx.x * EB, E = sg.E, tid = threadIdx.x;
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  R* __restrict__ Uf = (R*)sg.Uf;
  if (lin && tid < EB * 9) {
    const int le = tid / 9, k = tid - le * 9;
    const R* __restrict__ met = (const R*)sg.met;
    const size_t e = e0 + le < E ? (size_t)(e0 + le) : 0;
    sS[le][k] = double(met[e * 10 + 9]) * double(met[e * 10 + k]);
  }
  // the state: every thread issues its loads before the first use
  constexpr int NSL = (EB * 5 * NU + NT - 1) / NT;
  const int nvs = (E - e0 < EB ? E - e0 : EB) * 5 * NU;
  double xs[NSL];
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int it = tid + k * NT;
    xs[k] = U[(size_t)e0 * 5 * NU + (it < nvs ? it : 0)];
  }
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int it = tid + k * NT;
    if (it < EB * 5 * NU) {
      const int r = it % (5 * NU);
      double x = xs[k];
      if (r >= 4 * NU) x -= eref;
      if (r < NU) x -= rho0;
      sU[it] = x;
    }
  }
  lds_barrier();
  for (int it = tid; it < EB * NF; it += NT) {
    // element fastest: the lanes of a wave share operator rows (EB lanes a row)
    const int fp = it / EB, le = it - fp * EB;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    row_cols<NU, 5>(ops + DD::O_M0 + fp * NU, sU + le * 5 * NU, NU, acc);
#pragma unroll
    for (int v = 0; v < 5; ++v) sF[(le * 5 + v) * NF + fp] = acc[v];
  }
  lds_barrier();
  for (int it = tid; it < EB * 5 * NF; it += NT) {
    const int le = it / (5 * NF), r0 = it - le * (5 * NF), v = r0 / NF, fp = r0 - v * NF, e = e0 + le;
    if (e >= E) continue;
    const int f = C::face_of(fp), t = C::point_of(fp);
    const size_t slot = (size_t)(sg.slot_base + e * NFACE + f);
    const double x = sF[(le * 5 + v) * NF + fp];
    if constexpr (FB) {
      // the face's first flux point: the base square's first point, or a
      // triangle's first node
      const int fp0 = (C::PYR && f == 0) ? 0 : C::NB + (f - int(C::PYR)) * C::NTN;
      const float b = float(sF[(le * 5 + v) * NF + fp0]);
      Uf[(size_t)(sg.po_base + e * NF + fp - t) * 5 + v * C::fsz(f) + t] = R(x - double(b));
      if (t == 0) sg.Ub[slot * 5 + v] = b;
    } else {
      Uf[(size_t)(sg.po_base + e * NF + fp - t) * 5 + v * C::fsz(f) + t] = R(x);
    }
  }
  if (!lin) return;
  // (S m)_d in place over the momentum (each point by one thread)
  for (int it = tid; it < EB * NU; it += NT) {
    const int le = it / NU, s = it - le * NU;
    double* M = sU + le * 5 * NU + NU;
    const double m0 = M[s], m1 = M[NU + s], m2 = M[2 * NU + s];
#pragma unroll
    for (int d = 0; d < 3; ++d) M[d * NU + s] = sS[le][3 * d] * m0 + sS[le][3 * d + 1] * m1 + sS[le][3 * d + 2] * m2;
  }
  lds_barrier();
  R* __restrict__ Rp = (R*)sg.Rp;
  for (int it = tid; it < EB * NU; it += NT) {
    const int s = it / EB, le = it - s * EB, e = e0 + le;
    if (e >= E) continue;
    double acc[1] = {0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      row_cols<NU, 1>(ops + DD::O_LV + (d * NU + s) * NU, sU + le * 5 * NU + (1 + d) * NU, NU, acc);
    Rp[(size_t)e * 5 * NU + s] = R(acc[0]);
  }
}

// --------------------------------------------------------------- volume
// AA: flux anti-aliasing; without it the flux is evaluated at the solution
// points and the divergence takes the strong form (M1 - M3 M2) F~:
// sum_d D_d F~_d - M3 (nhat . M0 F~)
template <int ET, int P, typename R, int EB, int NT, bool AA>
__global__ void __launch_bounds__(NT) dense_volume(const Seg sg, const bool from_ust, const R* __restrict__ ops,
                                                 const Gas<R> g, const double eref, const double rho0) {
  using C = DenseCfg<ET, P>;
  constexpr int NU = C::NU, NF = C::NF, NQ = C::NQ, NFPS = C::NFPS, FQS = C::FQS, NFACE = C::NFACE;
  // the mass flux's divergence and the linear energy-flux part come from the
  // disu kernel's L(rho v): the fluxes of the other four variables are
  // projected
  constexpr int NVF = 4, V0 = 1;
  constexpr bool FC = sizeof(R) == 4;  // constant-flux subtraction (single precision)
  constexpr int PE = C::PER_ELEM;
  __shared__ R smem[EB * PE];
  __shared__ R sMet[EB][10];
  __shared__ FaceRec sFR[EB * NFACE];
  __shared__ R sFG[EB * NFACE][4];
  __shared__ uint8_t sPerm[MAX_PERMS * NFPS];
  __shared__ R sFc[EB][12];
  __shared__ R sUb[EB][5];  // single precision: the element's base state
  const int e0 = blockIdx.x * EB, E = sg.E, tid = threadIdx.x;
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  const R* __restrict__ Uf = (const R*)sg.Uf;
  R* __restrict__ Vf = (R*)sg.Vf;
  R* __restrict__ Rp = (R*)sg.Rp;
  const R* __restrict__ met = (const R*)sg.met;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
#define XS(le) (smem + (le)*PE)                        /* [20][NU]    */
#define JS(le) (smem + (le)*PE + C::SZ_X)              /* [5][NF]     */
#define FQ(le) (smem + (le)*PE + C::SZ_X + C::SZ_J)    /* [3][5][FQS] */

  // phase 0: face records, geometry, permutations and metrics to LDS, the
  // state (reference form), then the neighbour face values
  for (int it = tid; it < EB * NFACE; it += NT) {
    const int slot = sg.slot_base + (e0 + it / NFACE < E ? e0 * NFACE + it : 0);
    sFR[it] = sg.faces[slot];
#pragma unroll
    for (int k = 0; k < 4; ++k) sFG[it][k] = fgeo[4 * slot + k];
  }
  for (int it = tid; it < sg.nperm * NFPS; it += NT) sPerm[it] = sg.perms[it];
  for (int it = tid; it < EB * 10; it += NT) {
    const int le = it / 10, k = it - le * 10;
    sMet[le][k] = met[e0 + le < E ? (size_t)(e0 + le) * 10 + k : 0];
  }
  for (int it = tid; it < EB * 5 * NU; it += NT) {
    const int le = it / (5 * NU), r = it - le * (5 * NU);
    double x = U[e0 + le < E ? (size_t)e0 * 5 * NU + it : 0];
    if (r >= 4 * NU) x -= eref;
    if (r < NU) x -= rho0;
    if constexpr (FC) {
      // the state as deviations from the element's base state u_b (the base
      // of its first face): the linear operators then round the variation
      // within the element instead of the O(1) values
      const int e = e0 + le < E ? e0 + le : 0;
      x -= double(sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + r / NU]);
    }
    XS(le)[r] = R(x);
  }
  lds_barrier();
  for (int it = tid; it < EB * 5 * NF; it += NT) {
    const int le = it / (5 * NF), r0 = it - le * (5 * NF), v = r0 / NF, fp = r0 - v * NF;
    const int f = C::face_of(fp), t = C::point_of(fp);
    const FaceRec fr = sFR[le * NFACE + f];
    R x = Uf[(size_t)fr.npo * 5 + v * C::fsz(f) + sPerm[(fr.info >> 1) * NFPS + t]];
    if constexpr (FC) {
      // neighbour value relative to this element's base state
      const int e = e0 + le < E ? e0 + le : 0;
      x += sg.Ub[(size_t)fr.nbr * 5 + v] - sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + v];
    }
    JS(le)[r0] = x;
  }
  if (FC && tid < EB) {
    const int e = e0 + tid < E ? e0 + tid : 0;
    const_flux(sg.Ub + (size_t)(sg.slot_base + e * NFACE) * 5, &sMet[tid][0], g, &sFc[tid][0]);
#pragma unroll
    for (int v = 0; v < 5; ++v) sUb[tid][v] = sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + v];
    if (e0 + tid < E)
#pragma unroll
      for (int k = 0; k < 12; ++k) sg.fbar[(size_t)e * 12 + k] = sFc[tid][k];
  }
  lds_barrier();

  // phase 1: own face values (disu, M0) and the jumps C - u^f (eq. FR-conu:
  // L side (1/2 + beta)(u_nbr - u_own), R side (1/2 - beta)(u_nbr - u_own)),
  // in place over the neighbour values
  for (int it = tid; it < EB * NF; it += NT) {
    const int le = it / NF, fp = it - le * NF;
    R uf[5] = {R(0), R(0), R(0), R(0), R(0)};
    row_cols<NU, 5>(ops + C::O_M0 + fp * NU, XS(le), NU, uf);
    const bool left = sFR[le * NFACE + C::face_of(fp)].info & 1;
    const R w = left ? R(0.5) + g.beta : R(0.5) - g.beta;
#pragma unroll
    for (int v = 0; v < 5; ++v) JS(le)[v * NF + fp] = w * (JS(le)[v * NF + fp] - uf[v]);
  }
  lds_barrier();

  // phase 2: corrected reference gradient (eq. FR-qfinal), one (point,
  // direction) row of [D_d | n_d M3] per thread
  for (int it = tid; it < EB * 3 * NU; it += NT) {
    const int le = it / (3 * NU), r0 = it - le * (3 * NU), d = r0 / NU, s = r0 - d * NU;
    const R* row = ops + C::O_G + (d * NU + s) * C::KG;
    R q[5] = {R(0), R(0), R(0), R(0), R(0)};
    row_cols<NU, 5>(row, XS(le), NU, q);
    row_cols<NF, 5>(row + NU, JS(le), NF, q);
#pragma unroll
    for (int v = 0; v < 5; ++v) XS(le)[(5 + d * 5 + v) * NU + s] = q[v];
  }
  lds_barrier();

  // phase 3: physical gradient q = J^-T q~ (eq. FR-gradcoru), in place
  for (int it = tid; it < EB * NU; it += NT) {
    const int le = it / NU, s = it - le * NU;
    R* X = XS(le);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R g0 = X[(5 + v) * NU + s], g1 = X[(10 + v) * NU + s], g2 = X[(15 + v) * NU + s];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        X[(5 + c * 5 + v) * NU + s] = sMet[le][c] * g0 + sMet[le][3 + c] * g1 + sMet[le][6 + c] * g2;
    }
  }
  lds_barrier();

  // phase 3a: gradcoru_fpts and the own normal viscous flux at every flux
  // point (exchanged instead of the gradient)
  for (int it = tid; it < EB * NF; it += NT) {
    const int le = it / NF, fp = it - le * NF, e = e0 + le;
    if (e >= E) continue;
    R w[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) w[k] = R(0);
    row_cols<NU, 20>(ops + C::O_M0 + fp * NU, XS(le), NU, w);
    const int f = C::face_of(fp), t = C::point_of(fp), lf = le * NFACE + f;
    const R sgn = (sFR[lf].info & 1) ? R(1) : R(-1);
    const R nn[3] = {sgn * sFG[lf][0], sgn * sFG[lf][1], sgn * sFG[lf][2]};
    R u[5], q[3][5], V[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = w[v] + (FC ? sUb[le][v] : R(0));
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][v] = w[5 + c * 5 + v];
    }
    normal_viscous(u, q, nn, g, V);
    const size_t po = (size_t)(sg.po_base + e * NF + fp - t);
#pragma unroll
    for (int k = 0; k < 4; ++k) Vf[po * 4 + k * C::fsz(f) + t] = V[k];
  }

  if constexpr (!AA) {
    // tdisf at the solution points, F~ into the flux region (NU <= FQS)
    for (int it = tid; it < EB * NU; it += NT) {
      const int le = it / NU, s = it - le * NU;
      const R* X = XS(le);
      R u[5], q[3][5], f[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        u[v] = X[v * NU + s] + (FC ? sUb[le][v] : R(0));
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c][v] = X[(5 + c * 5 + v) * NU + s];
      }
      point_flux(u, q, g, f);
      const R dj = sMet[le][9];
      R* F = FQ(le);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = V0; v < 5; ++v)
          F[(d * 5 + v) * FQS + s] =
              dj * (sMet[le][3 * d] * f[0][v] + sMet[le][3 * d + 1] * f[1][v] + sMet[le][3 * d + 2] * f[2][v]) -
              (FC ? sFc[le][d * 4 + v - 1] : R(0));
    }
    lds_barrier();
    if constexpr (C::PYR) {
      // weak form without anti-aliasing: sum_d Ku_d F~_d (the lifting of the
      // interior normal flux is part of the weak form)
      for (int it = tid; it < EB * NU; it += NT) {
        const int le = it / NU, s = it - le * NU, e = e0 + le;
        if (e >= E) continue;
        R acc[NVF] = {R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int d = 0; d < 3; ++d)
          row_cols<NU, NVF>(ops + C::O_KU + (d * NU + s) * NU, FQ(le) + (d * 5 + V0) * FQS, FQS, acc);
        acc[NVF - 1] += g.kap * Rp[(size_t)e * 5 * NU + s];  // kap L(rho v)
#pragma unroll
        for (int v = 0; v < NVF; ++v) Rp[(size_t)e * 5 * NU + (V0 + v) * NU + s] = acc[v];
      }
      return;
    }
    // M2 F~: reference normal flux at the own flux points, into the jump
    // region (free since the gradient phase)
    for (int it = tid; it < EB * NF; it += NT) {
      const int le = it / NF, fp = it - le * NF;
      const R* nh = ops + C::O_N + 3 * C::face_of(fp);
      R nf[NVF] = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R a[NVF] = {R(0), R(0), R(0), R(0)};
        row_cols<NU, NVF>(ops + C::O_M0 + fp * NU, FQ(le) + (d * 5 + V0) * FQS, FQS, a);
#pragma unroll
        for (int v = 0; v < NVF; ++v) nf[v] += nh[d] * a[v];
      }
#pragma unroll
      for (int v = 0; v < NVF; ++v) JS(le)[v * NF + fp] = nf[v];
    }
    lds_barrier();
    // (M1 - M3 M2) F~ = sum_d D_d F~_d - M3 (M2 F~)
    for (int it = tid; it < EB * NU; it += NT) {
      const int le = it / NU, s = it - le * NU, e = e0 + le;
      if (e >= E) continue;
      R acc[NVF] = {R(0), R(0), R(0), R(0)}, lift[NVF] = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        row_cols<NU, NVF>(ops + C::O_G + (d * NU + s) * C::KG, FQ(le) + (d * 5 + V0) * FQS, FQS, acc);
      row_cols<NF, NVF>(ops + C::O_M3 + s * NF, JS(le), NF, lift);
      acc[NVF - 1] += g.kap * Rp[(size_t)e * 5 * NU + s];  // kap L(rho v)
#pragma unroll
      for (int v = 0; v < NVF; ++v) Rp[(size_t)e * 5 * NU + (V0 + v) * NU + s] = acc[v] - lift[v];
    }
    return;
  }
  // phase 4: uqpts / gradcoru_qpts (M7) and tdisf at each quadrature point
  // (eq. FR-tdisfq): F~_d = det J sum_c (J^-1)_{dc} f_c
  for (int it = tid; it < EB * NQ; it += NT) {
    const int le = it / NQ, q0 = it - le * NQ;
    R w[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) w[k] = R(0);
    row_cols<NU, 20>(ops + C::O_M7 + q0 * NU, XS(le), NU, w);
    R u[5], q[3][5], f[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = w[v] + (FC ? sUb[le][v] : R(0));
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][v] = w[5 + c * 5 + v];
    }
    point_flux(u, q, g, f);
    const R dj = sMet[le][9];
    R* F = FQ(le);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = V0; v < 5; ++v)
        F[(d * 5 + v) * FQS + q0] =
            dj * (sMet[le][3 * d] * f[0][v] + sMet[le][3 * d + 1] * f[1][v] + sMet[le][3 * d + 2] * f[2][v]) -
            (FC ? sFc[le][d * 4 + v - 1] : R(0));
  }
  lds_barrier();  // every face and quadrature point has read the state and gradients

  // phase 5: projection-divergence (M1 - M3 M2) M9 in weak form, one (point,
  // direction) row of AP_d per thread; the three partial sums go over the
  // state slots
  for (int it = tid; it < EB * 3 * NU; it += NT) {
    const int le = it / (3 * NU), r0 = it - le * (3 * NU), d = r0 / NU, s = r0 - d * NU;
    R acc[NVF] = {R(0), R(0), R(0), R(0)};
    row_cols<NQ, NVF>(ops + C::O_AP + (d * NU + s) * NQ, FQ(le) + (d * 5 + V0) * FQS, FQS, acc);
#pragma unroll
    for (int v = 0; v < NVF; ++v) XS(le)[(d * 5 + V0 + v) * NU + s] = acc[v];
  }
  lds_barrier();
  for (int it = tid; it < EB * NVF * NU; it += NT) {
    const int le = it / (NVF * NU), r0 = V0 * NU + it - le * (NVF * NU), e = e0 + le;
    if (e >= E) continue;
    const R* X = XS(le);
    R s = X[r0] + X[5 * NU + r0] + X[10 * NU + r0];
    if (r0 >= 4 * NU) s += g.kap * Rp[(size_t)e * 5 * NU + r0 - 4 * NU];  // kap L(rho v)
    Rp[(size_t)e * 5 * NU + r0] = s;
  }
#undef XS
#undef JS
#undef FQ
}

// ------------------------------------------------- volume, matrix cores
// The volume group with every dense product on the matrix cores
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64: D(16x16) += A(16x4)
// B(4x16) per wave; lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds, for r < 4, D[4 (l / 16) + r][l % 16] in FP32 and
// D[l / 16 + 4 r][l % 16] in FP64).  A product C = A B runs over 16 x 16
// output tiles: rows are operator rows, columns the (element, field) pairs
// of the workgroup.  M0, the gradient operator and M7 give each wave a
// contiguous range of tiles (row tile major), so that a wave loads an
// operator tile once for its column tiles; the projection-divergence (two
// or three tiles at p = 3 and 4) gives the waves its tiles in turn.  A comes from the
// packed operator copy (one coalesced 64-value load per k-step), B from the
// element's columns in LDS.  Products that feed point-wise physics (face and
// quadrature values) go through LDS rows; the three directions of the
// projection-divergence are one product with K concatenated.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename R>
struct MfVec;
template <>
struct MfVec<float> {
  typedef mf4 T;
  // output row of value r of this lane within the 16-row tile
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  __device__ static mf4 mfma(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct MfVec<double> {
  typedef md4 T;
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  __device__ static md4 mfma(double a, double b, md4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// acc += A B over KS k-steps: A a packed tile (its KS values of this lane
// loaded up front), B the column of this lane at bcol with stride bs in k.
// The packed A is zero past the operator's K, and the B reads there stay in
// finite (zero-initialised or written) LDS, so no bounds checks are needed.
template <int KS, typename R>
__device__ __forceinline__ void mf_acc(typename MfVec<R>::T& acc, const R* __restrict__ Ap, const R* bcol, int bs,
                                       int lane) {
  R a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a[ks] = Ap[ks * 64 + lane];
  const R* b = bcol + (lane >> 4) * bs;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) acc = MfVec<R>::mfma(a[ks], b[4 * ks * bs], acc);
}

// The same product in two steps, for a wave that applies one operator tile
// to several column tiles: the tile's KS values of this lane into
// registers, then the k-steps against one column
template <int KS, typename R>
__device__ __forceinline__ void mf_load(R (&a)[KS], const R* __restrict__ Ap, int lane) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a[ks] = Ap[ks * 64 + lane];
}
template <int KS, typename R>
__device__ __forceinline__ void mf_run(typename MfVec<R>::T& acc, const R (&a)[KS], const R* bcol, int bs, int lane) {
  const R* b = bcol + (lane >> 4) * bs;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) acc = MfVec<R>::mfma(a[ks], b[4 * ks * bs], acc);
}
// LEAN: the matrix-core volume kernel keeps the element metrics, base
// states, constant fluxes and the permutation table out of its own LDS
// arrays (global reads, the permutations in element 0's region, the rest
// copied into the dead state region once the quadrature values are
// formed), so that its LDS is the element regions alone; and it asks for
// six waves per SIMD (at most 80 VGPRs).  At p = 3 with flux anti-aliasing;
// the CU's LDS is allocated in 128 blocks of 1280 bytes:
//  * tetrahedra, 4 elements x 1680 values = 26 880 bytes, exactly 21
//    blocks: six workgroups share a CU instead of five;
//  * pyramids, 3 elements per workgroup (dense_rhs_t) x 1884 values =
//    22 608 bytes (18 blocks) at 65 VGPRs: seven workgroups instead of five
//    of four elements;
//  * double-precision tetrahedra, 2 elements x 1680 values x 8 bytes =
//    26 880 bytes: six workgroups instead of five;
//  * double-precision pyramids, 2 elements x 1884 values x 8 bytes =
//    30 144 bytes (24 blocks) at most 96 VGPRs: five workgroups instead of
//    four.
template <int ET, int P, typename R, bool AA>
struct MfLean {
  static constexpr bool value = P == 3 && AA;
  // without anti-aliasing the element regions hold no quadrature rows and
  // the LDS allows more than six workgroups; six waves per SIMD all the
  // same.  Double-precision pyramids (2 elements, 30 144 bytes: five
  // workgroups) ask for five.
  static constexpr int min_waves = P != 3 ? 1 : (sizeof(R) == 8 && ET == 3 ? 5 : 6);
};

// The tiles t = mt NTL + nt (operator row tile mt, column tile nt) of a
// product, in one contiguous range per wave: a wave reloads its operator
// tile only where mt changes, so each tile is read from the device table
// about once per wave instead of once per (mt, nt)
__device__ __forceinline__ void wave_tiles(int T, int NW, int wave, int& t0, int& t1) {
  t0 = wave * T / NW;
  t1 = (wave + 1) * T / NW;
}

template <int ET, int P, typename R, int EB, int NT, bool AA>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MfLean<ET, P, R, AA>::min_waves)))
    dense_volume_mf(const Seg sg, const bool from_ust, const R* __restrict__ ops, const Gas<R> g,
                    const double eref, const double rho0) {
  using C = DenseCfg<ET, P>;
  using V4 = typename MfVec<R>::T;
  constexpr int NU = C::NU, NF = C::NF, NQ = C::NQ, NFPS = C::NFPS, NFACE = C::NFACE, LDW = C::LDW;
  // the mass flux's divergence and the linear energy-flux part come from the
  // disu kernel's L(rho v): the fluxes of the other four variables are
  // projected
  constexpr int NVF = 4, V0 = 1;
  constexpr bool FC = sizeof(R) == 4;  // constant-flux subtraction (single precision)
  constexpr int PE = AA ? C::PE_MF : C::PE_MF_NOAA, NW = NT / 64;
  static_assert(NU * LDW >= 5 * NF + 4 && (!AA || 4 * C::KSQ <= C::SZ_U2 / LDW) &&
                    4 * C::KSU * LDW <= PE - C::SZ_X - C::XPAD,
                "padding rows lie after the jumps and inside the element's region");
  static_assert((LDW * sizeof(R)) % 16 == 0 && ((C::SZ_X + C::XPAD) * sizeof(R)) % 16 == 0 &&
                    (PE * sizeof(R)) % 16 == 0,
                "rows start on 16-byte boundaries");
  constexpr bool LEAN = MfLean<ET, P, R, AA>::value;
  // RIN: the face records and face geometry of each element sit in its U2
  // region after the NF face rows (16-byte aligned), where nothing is
  // written before the quadrature values (phase 4), after their last reads
  // (phase 3a); the zero padding rows lie elsewhere (NU rows below NF, NQ
  // rows above)
  constexpr int AL = 16 / (int)sizeof(R), ROFF = (C::SZ_X + C::XPAD + NF * LDW + AL - 1) / AL * AL;
  constexpr int RSZ = NFACE * (16 + 4 * (int)sizeof(R)) / (int)sizeof(R);
  constexpr bool RIN = PE % AL == 0 && ROFF + RSZ <= PE && ROFF + RSZ <= C::SZ_X + C::XPAD + NQ * LDW &&
                       4 * C::KSU <= NF;
  // LEAN: the permutation table after element 0's face records (read by
  // the gather of phase 0 only); the metrics, base state and constant flux
  // of element le at XS(le) + [0, 27) once the quadrature values are formed
  constexpr int POFF = ROFF + RSZ;
  static_assert(!LEAN || (RIN && AA && POFF + MAX_PERMS * NFPS / (int)sizeof(R) <= C::SZ_X + C::XPAD + NQ * LDW),
                "the lean layout's permutation table fits before the quadrature rows are written");
  __shared__ __align__(16) R smem[EB * PE];
  __shared__ R sMetA[LEAN ? 1 : EB][10];
  __shared__ FaceRec sFRA[RIN ? 1 : EB * NFACE];
  __shared__ R sFGA[RIN ? 1 : EB * NFACE * 4];
  __shared__ uint8_t sPermA[LEAN ? 1 : MAX_PERMS * NFPS];
  __shared__ R sFcA[LEAN ? 1 : EB][12];
  __shared__ R sUbA[LEAN ? 1 : EB][5];  // single precision: the element's base state
  uint8_t* const sPerm = LEAN ? (uint8_t*)(smem + POFF) : sPermA;
#define FRQ(le, f) (RIN ? ((FaceRec*)(smem + (le)*PE + ROFF))[f] : sFRA[(le)*NFACE + (f)])
#define FGQ(le, f, k) (RIN ? (smem + (le)*PE + ROFF + NFACE * 16 / (int)sizeof(R))[4 * (f) + (k)] \
                           : sFGA[((le)*NFACE + (f)) * 4 + (k)])
  const int e0 = blockIdx.x * EB, E = sg.E, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  const R* __restrict__ Uf = (const R*)sg.Uf;
  R* __restrict__ Vf = (R*)sg.Vf;
  R* __restrict__ Rp = (R*)sg.Rp;
  const R* __restrict__ met = (const R*)sg.met;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
#define XS(le) (smem + (le)*PE)              /* [20][NU] */
#define U2(le) (smem + (le)*PE + C::SZ_X + C::XPAD) /* [5][NF] | [NF][LDW] | [NQ][LDW] */
  // metrics, base state and constant flux of element le: LDS arrays, or
  // (LEAN) global reads before the quadrature phase and XS(le) + [0, 27)
  // from it on (QP: the quadrature-phase copy)
  auto ec = [&](int le) { return (size_t)(e0 + le < E ? e0 + le : e0); };
  auto metg = [&](int le, int k) -> R { return LEAN ? met[ec(le) * 10 + k] : sMetA[LEAN ? 0 : le][k]; };
  auto ubg = [&](int le, int v) -> R {
    return LEAN ? R(sg.Ub[(size_t)(sg.slot_base + ec(le) * NFACE) * 5 + v]) : sUbA[LEAN ? 0 : le][v];
  };
#define METQ(le, k) (LEAN ? XS(le)[k] : sMetA[LEAN ? 0 : (le)][k])
#define UBQ(le, v) (LEAN ? XS(le)[10 + (v)] : sUbA[LEAN ? 0 : (le)][v])
#define FCQ(le, k) (LEAN ? XS(le)[15 + (k)] : sFcA[LEAN ? 0 : (le)][k])
  // The products read past a column's end into the next column or into the
  // padding when a k range is not a multiple of 4; the operator's zero
  // padding weights those reads, which therefore have to be finite.  LDS
  // holds whatever earlier kernels left there, so every location a product
  // reads is either written before that product or set to zero here:
  //  * the 4 KSU - NU entries after the state, which the state columns'
  //    products (phases 1 and 2) read before phase 2 writes the gradients
  //    there (a gradient written meanwhile is finite as well),
  //  * the padding after the state and gradients and after the jumps,
  //  * the rows from NU to 4 KSU and from NQ to 4 KSQ.
  // These writes touch no location that phase 0 writes, and the barriers
  // before the first product order them.
  {
    constexpr int XP = C::XPAD, ZX = 4 * C::KSU - NU, ZU = ZX * LDW, ZQ = AA ? (4 * C::KSQ - NQ) * LDW : 0;
    constexpr int NZ = XP + 4 + ZX + ZU + ZQ;
    for (int it = tid; it < EB * NZ; it += NT) {
      const int le = it / NZ, k = it - le * NZ;
      R* z;
      if (k < XP)
        z = XS(le) + C::SZ_X + k;
      else if (k < XP + 4)
        z = U2(le) + 5 * NF + (k - XP);
      else if (k < XP + 4 + ZX)
        z = XS(le) + 5 * NU + (k - XP - 4);
      else if (k < XP + 4 + ZX + ZU)
        z = U2(le) + NU * LDW + (k - XP - 4 - ZX);
      else
        z = U2(le) + NQ * LDW + (k - XP - 4 - ZX - ZU);
      *z = R(0);
    }
  }

  // phase 0: as in dense_volume (neighbour face values into U2 as [5][NF]).
  // Every thread issues its state loads before the first barrier and its
  // gather loads after it, each set before the first use, so that a
  // thread's loads are in flight together; out-of-range items read valid
  // addresses and are not stored.
  const int nv = E - e0 < EB ? E - e0 : EB;  // valid elements of the workgroup
  constexpr int NSL = (EB * 5 * NU + NT - 1) / NT, NGL = (EB * 5 * NF + NT - 1) / NT;
  double xs[NSL];
  float xb[FC ? NSL : 1];
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int it = tid + k * NT;
    const bool ok = it < nv * 5 * NU;
    const int itc = ok ? it : 0, le = itc / (5 * NU), r = itc - le * (5 * NU);
    xs[k] = U[(size_t)e0 * 5 * NU + itc];
    // single precision: the element's base state (the base of its first face)
    if constexpr (FC) xb[k] = sg.Ub[(size_t)(sg.slot_base + (e0 + le) * NFACE) * 5 + r / NU];
  }
  for (int it = tid; it < EB * NFACE; it += NT) {
    const int slot = sg.slot_base + (e0 + it / NFACE < E ? e0 * NFACE + it : 0);
    const int le = it / NFACE, f = it - le * NFACE;
    FRQ(le, f) = sg.faces[slot];
#pragma unroll
    for (int k = 0; k < 4; ++k) FGQ(le, f, k) = fgeo[4 * slot + k];
  }
  for (int it = tid; it < sg.nperm * NFPS; it += NT) sPerm[it] = sg.perms[it];
  if constexpr (!LEAN)
    for (int it = tid; it < EB * 10; it += NT) {
      const int le = it / 10, k = it - le * 10;
      sMetA[le][k] = met[e0 + le < E ? (size_t)(e0 + le) * 10 + k : 0];
    }
  lds_barrier();
  R gx[NGL];
  float gn[FC ? NGL : 1], go[FC ? NGL : 1];
#pragma unroll
  for (int k = 0; k < NGL; ++k) {
    const int it = tid + k * NT;
    const int itc = it < EB * 5 * NF ? it : 0;
    const int le = itc / (5 * NF), r0 = itc - le * (5 * NF), v = r0 / NF, fp = r0 - v * NF;
    const int f = C::face_of(fp), t = C::point_of(fp);
    const FaceRec fr = FRQ(le, f);
    gx[k] = Uf[(size_t)fr.npo * 5 + v * C::fsz(f) + sPerm[(fr.info >> 1) * NFPS + t]];
    if constexpr (FC) {
      // neighbour value relative to this element's base state
      const int e = le < nv ? e0 + le : e0;
      gn[k] = sg.Ub[(size_t)fr.nbr * 5 + v];
      go[k] = sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + v];
    }
  }
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int it = tid + k * NT;
    if (it < EB * 5 * NU) {
      const int le = it / (5 * NU), r = it - le * (5 * NU);
      double x = xs[k];
      if (r >= 4 * NU) x -= eref;
      if (r < NU) x -= rho0;
      // single precision: the state as deviations from the element's base
      // state u_b: the linear operators then round the variation within the
      // element instead of the O(1) values
      if constexpr (FC) x -= double(xb[k]);
      XS(le)[r] = R(x);
    }
  }
#pragma unroll
  for (int k = 0; k < NGL; ++k) {
    const int it = tid + k * NT;
    if (it < EB * 5 * NF) {
      const int le = it / (5 * NF), r0 = it - le * (5 * NF);
      U2(le)[r0] = FC ? gx[k] + (gn[k] - go[k]) : gx[k];
    }
  }
  if (FC && tid < EB) {
    const int e = e0 + tid < E ? e0 + tid : 0;
    if constexpr (LEAN) {
      R fc[12];
      const_flux(sg.Ub + (size_t)(sg.slot_base + e * NFACE) * 5, met + (size_t)e * 10, g, fc);
      if (e0 + tid < E)
#pragma unroll
        for (int k = 0; k < 12; ++k) sg.fbar[(size_t)e * 12 + k] = fc[k];
    } else {
      const_flux(sg.Ub + (size_t)(sg.slot_base + e * NFACE) * 5, &sMetA[tid][0], g, &sFcA[tid][0]);
#pragma unroll
      for (int v = 0; v < 5; ++v) sUbA[tid][v] = sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + v];
      if (e0 + tid < E)
#pragma unroll
        for (int k = 0; k < 12; ++k) sg.fbar[(size_t)e * 12 + k] = sFcA[tid][k];
    }
  }
  lds_barrier();

  // phase 1: jumps (eq. FR-conu), M0 on the matrix cores, in place over the
  // neighbour values: columns (element, variable)
  {
    constexpr int NTL = (5 * EB + 15) / 16;
    int t0, t1, amt = -1;
    wave_tiles(C::MTF * NTL, NW, wave, t0, t1);
    R a[C::KSU];
    for (int t = t0; t < t1; ++t) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < 5 * EB;
      const int le = ok ? j / 5 : EB - 1, v = ok ? j % 5 : 0;
      if (mt != amt) {
        mf_load<C::KSU>(a, ops + C::O_PM0 + mt * C::KSU * 64, lane);
        amt = mt;
      }
      V4 acc = {R(0), R(0), R(0), R(0)};
      mf_run<C::KSU>(acc, a, XS(le) + v * NU, 1, lane);
      if (ok)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int fp = mt * 16 + MfVec<R>::row(lane, r);
          if (fp < NF) {
            const bool left = FRQ(le, C::face_of(fp)).info & 1;
            const R w = left ? R(0.5) + g.beta : R(0.5) - g.beta;
            R* J = U2(le) + v * NF + fp;
            *J = w * (*J - acc[r]);
          }
        }
    }
  }
  lds_barrier();

  // phase 2: corrected reference gradient (eq. FR-qfinal): rows (direction,
  // point) of [D_d | n_d M3] against [u; jumps]
  {
    constexpr int NTL = (5 * EB + 15) / 16;
    int t0, t1, amt = -1;
    wave_tiles(C::MTG * NTL, NW, wave, t0, t1);
    R au[C::KSU], af[C::KSF];
    for (int t = t0; t < t1; ++t) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < 5 * EB;
      const int le = ok ? j / 5 : EB - 1, v = ok ? j % 5 : 0;
      if (mt != amt) {
        const R* Ap = ops + C::O_PG + mt * (C::KSU + C::KSF) * 64;
        mf_load<C::KSU>(au, Ap, lane);
        mf_load<C::KSF>(af, Ap + C::KSU * 64, lane);
        amt = mt;
      }
      V4 acc = {R(0), R(0), R(0), R(0)};
      mf_run<C::KSU>(acc, au, XS(le) + v * NU, 1, lane);
      mf_run<C::KSF>(acc, af, U2(le) + v * NF, 1, lane);
      if (ok)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mt * 16 + MfVec<R>::row(lane, r);
          if (row < 3 * NU) {
            const int d = row / NU, s = row - d * NU;
            XS(le)[(5 + d * 5 + v) * NU + s] = acc[r];
          }
        }
    }
  }
  lds_barrier();

  // phase 3: physical gradient q = J^-T q~ (eq. FR-gradcoru), in place
  for (int it = tid; it < EB * NU; it += NT) {
    const int le = it / NU, s = it - le * NU;
    R* X = XS(le);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R g0 = X[(5 + v) * NU + s], g1 = X[(10 + v) * NU + s], g2 = X[(15 + v) * NU + s];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        X[(5 + c * 5 + v) * NU + s] = metg(le, c) * g0 + metg(le, 3 + c) * g1 + metg(le, 6 + c) * g2;
    }
  }
  lds_barrier();

  // phase 3a: state and gradient at the flux points (M0, 20 columns per
  // element) into U2 rows, then the own normal viscous flux per flux point
  {
    constexpr int NTL = (20 * EB + 15) / 16;
    int t0, t1, amt = -1;
    wave_tiles(C::MTF * NTL, NW, wave, t0, t1);
    R a[C::KSU];
    for (int t = t0; t < t1; ++t) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < 20 * EB;
      const int le = ok ? j / 20 : EB - 1, c = ok ? j % 20 : 0;
      if (mt != amt) {
        mf_load<C::KSU>(a, ops + C::O_PM0 + mt * C::KSU * 64, lane);
        amt = mt;
      }
      V4 acc = {R(0), R(0), R(0), R(0)};
      mf_run<C::KSU>(acc, a, XS(le) + c * NU, 1, lane);
      if (ok)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int fp = mt * 16 + MfVec<R>::row(lane, r);
          if (fp < NF) U2(le)[fp * LDW + c] = acc[r];
        }
    }
  }
  lds_barrier();
  for (int it = tid; it < EB * NF; it += NT) {
    const int le = it / NF, fp = it - le * NF, e = e0 + le;
    if (e >= E) continue;
    const R* w = (const R*)__builtin_assume_aligned(U2(le) + fp * LDW, 16);
    const int f = C::face_of(fp), t = C::point_of(fp);
    const R sgn = (FRQ(le, f).info & 1) ? R(1) : R(-1);
    const R nn[3] = {sgn * FGQ(le, f, 0), sgn * FGQ(le, f, 1), sgn * FGQ(le, f, 2)};
    R u[5], q[3][5], V[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = w[v] + (FC ? ubg(le, v) : R(0));
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][v] = w[5 + c * 5 + v];
    }
    normal_viscous(u, q, nn, g, V);
    const size_t po = (size_t)(sg.po_base + e * NF + fp - t);
#pragma unroll
    for (int k = 0; k < 4; ++k) Vf[po * 4 + k * C::fsz(f) + t] = V[k];
  }
  lds_barrier();

  if constexpr (!AA) {
    // tdisf at the solution points, F~_d of variable v into column 5 d + v of
    // the point's U2 row, then the divergence [K0_0 | K0_1 | K0_2] F~ as one
    // product over K = (direction, solution point)
    for (int it = tid; it < EB * NU; it += NT) {
      const int le = it / NU, s0 = it - le * NU;
      const R* X = XS(le);
      R u[5], q[3][5], f[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        u[v] = X[v * NU + s0] + (FC ? UBQ(le, v) : R(0));
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c][v] = X[(5 + c * 5 + v) * NU + s0];
      }
      point_flux(u, q, g, f);
      const R dj = METQ(le, 9);
      R* w = (R*)__builtin_assume_aligned(U2(le) + s0 * LDW, 16);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = V0; v < 5; ++v)
          w[4 * d + v - 1] =
              dj * (METQ(le, 3 * d) * f[0][v] + METQ(le, 3 * d + 1) * f[1][v] + METQ(le, 3 * d + 2) * f[2][v]) -
              (FC ? FCQ(le, d * 4 + v - 1) : R(0));
    }
    lds_barrier();
    constexpr int NTL = (NVF * EB + 15) / 16;
    for (int t = wave; t < C::MTU * NTL; t += NW) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < NVF * EB;
      const int le = ok ? j / NVF : EB - 1, v = ok ? V0 + j % NVF : V0;
      const R* Ap = ops + C::O_PK0 + mt * 3 * C::KSU * 64;
      V4 acc = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) mf_acc<C::KSU>(acc, Ap + d * C::KSU * 64, U2(le) + 4 * d + v - 1, LDW, lane);
      const int e = e0 + le;
      if (ok && e < E)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int s0 = mt * 16 + MfVec<R>::row(lane, r);
          if (s0 < NU) {
            R x = acc[r];
            if (v == 4) x += g.kap * Rp[(size_t)e * 5 * NU + s0];  // kap L(rho v)
            Rp[(size_t)e * 5 * NU + v * NU + s0] = x;
          }
        }
    }
    return;
  }

  // phase 4: state and gradient at the quadrature points (M7) into U2 rows,
  // then tdisf per point (eq. FR-tdisfq), F~_d of variable v in place into
  // column 5 d + v of the point's row
  {
    constexpr int NTL = (20 * EB + 15) / 16;
    int t0, t1, amt = -1;
    wave_tiles(C::MTQ * NTL, NW, wave, t0, t1);
    R a[C::KSU];
    for (int t = t0; t < t1; ++t) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < 20 * EB;
      const int le = ok ? j / 20 : EB - 1, c = ok ? j % 20 : 0;
      if (mt != amt) {
        mf_load<C::KSU>(a, ops + C::O_PM7 + mt * C::KSU * 64, lane);
        amt = mt;
      }
      V4 acc = {R(0), R(0), R(0), R(0)};
      mf_run<C::KSU>(acc, a, XS(le) + c * NU, 1, lane);
      if (ok)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q0 = mt * 16 + MfVec<R>::row(lane, r);
          if (q0 < NQ) U2(le)[q0 * LDW + c] = acc[r];
        }
    }
  }
  lds_barrier();
  if constexpr (LEAN) {
    // the state region is dead now: element le's metrics, base state and
    // constant flux go to XS(le) + [0, 27) for the flux of every point
    if (tid < EB) {
      R* x = XS(tid);
      const size_t e = ec(tid);
#pragma unroll
      for (int k = 0; k < 10; ++k) x[k] = met[e * 10 + k];
      if constexpr (FC) {  // single precision: base state and constant flux
#pragma unroll
        for (int v = 0; v < 5; ++v) x[10 + v] = sg.Ub[(size_t)(sg.slot_base + e * NFACE) * 5 + v];
        const_flux(sg.Ub + (size_t)(sg.slot_base + e * NFACE) * 5, met + e * 10, g, x + 15);
      }
    }
    lds_barrier();
  }
  for (int it = tid; it < EB * NQ; it += NT) {
    const int le = it / NQ, q0 = it - le * NQ;
    R* w = (R*)__builtin_assume_aligned(U2(le) + q0 * LDW, 16);
    R u[5], q[3][5], f[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = w[v] + (FC ? UBQ(le, v) : R(0));
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c][v] = w[5 + c * 5 + v];
    }
    point_flux(u, q, g, f);
    const R dj = METQ(le, 9);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = V0; v < 5; ++v)
        w[4 * d + v - 1] = dj * (METQ(le, 3 * d) * f[0][v] + METQ(le, 3 * d + 1) * f[1][v] + METQ(le, 3 * d + 2) * f[2][v]) -
                           (FC ? FCQ(le, d * 4 + v - 1) : R(0));
  }
  lds_barrier();

  // phase 5: projection-divergence, sum_d AP_d F~_d as one product over the
  // concatenated K = (direction, quadrature point)
  {
    constexpr int NTL = (NVF * EB + 15) / 16;
    for (int t = wave; t < C::MTU * NTL; t += NW) {
      const int mt = t / NTL, nt = t - mt * NTL, j = nt * 16 + (lane & 15);
      const bool ok = j < NVF * EB;
      const int le = ok ? j / NVF : EB - 1, v = ok ? V0 + j % NVF : V0;
      const R* Ap = ops + C::O_PAP + mt * 3 * C::KSQ * 64;
      V4 acc = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        mf_acc<C::KSQ>(acc, Ap + d * C::KSQ * 64, U2(le) + 4 * d + v - 1, LDW, lane);
      const int e = e0 + le;
      if (ok && e < E)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int s = mt * 16 + MfVec<R>::row(lane, r);
          if (s < NU) {
            R x = acc[r];
            if (v == 4) x += g.kap * Rp[(size_t)e * 5 * NU + s];  // kap L(rho v)
            Rp[(size_t)e * 5 * NU + v * NU + s] = x;
          }
        }
    }
  }
#undef XS
#undef U2
#undef FRQ
#undef FGQ
#undef METQ
#undef UBQ
#undef FCQ
}

// -------------------------------------------------------------- surface
// comm_flux at every own flux point (both sides of a pair evaluate the same
// expression on the same inputs and normal; each side scales by its own area
// factor), then tdivtconf (M3) + negdivconf and the RK4 stage store
template <int ET, int P, typename R, int EB, int NT>
__global__ void __launch_bounds__(NT) dense_surface(const Seg sg, const int rk, const R* __restrict__ ops,
                                                  const Gas<R> g) {
  using C = DenseCfg<ET, P>;
  constexpr int NU = C::NU, NF = C::NF, NFPS = C::NFPS, NFACE = C::NFACE;
  __shared__ R sD[EB * 5 * NF];
  const int e0 = blockIdx.x * EB, E = sg.E, tid = threadIdx.x;
  const R* __restrict__ Uf = (const R*)sg.Uf;
  const R* __restrict__ Vf = (const R*)sg.Vf;
  const R* __restrict__ Rp = (const R*)sg.Rp;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
  for (int it = tid; it < EB * NF; it += NT) {
    const int le = it / NF, fp = it - le * NF, e = e0 + le;
    if (e >= E) continue;
    const int f = C::face_of(fp), t = C::point_of(fp);
    const int slot = sg.slot_base + e * NFACE + f;
    const FaceRec fr = sg.faces[slot];
    const int rr = sg.perms[(fr.info >> 1) * NFPS + t];
    const bool left = fr.info & 1;
    const size_t po = (size_t)(sg.po_base + e * NF + fp - t);
    const int fs = C::fsz(f);
    R uo[5], un[5], jn[5], Vo[4], Vn[4], F[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      uo[v] = Uf[po * 5 + v * fs + t];
      un[v] = Uf[(size_t)fr.npo * 5 + v * fs + rr];
    }
    // u_nbr - u_own from the face bases and deviations (single precision),
    // before the states themselves are formed
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if constexpr (sizeof(R) == 4) {
        const float bo = sg.Ub[(size_t)slot * 5 + v], bn = sg.Ub[(size_t)fr.nbr * 5 + v];
        jn[v] = (bn - bo) + (un[v] - uo[v]);
        uo[v] += bo;
        un[v] += bn;
      } else {
        jn[v] = un[v] - uo[v];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Vo[k] = Vf[po * 4 + k * fs + t];
      Vn[k] = Vf[(size_t)fr.npo * 4 + k * fs + rr];
    }
    const R nL[3] = {fgeo[4 * slot], fgeo[4 * slot + 1], fgeo[4 * slot + 2]};
    const R mag = fgeo[4 * slot + 3];
    face_flux<R, true>(uo, un, jn, Vo, Vn, nL, left, g, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] *= mag;
    if constexpr (sizeof(R) == 4) {
      // the element's constant transformed flux, taken out of the volume
      // product, leaves through its reference normal component here
      const R* nh = ops + C::O_N + 3 * f;
      const float* fc = sg.fbar + (size_t)e * 12;
#pragma unroll
      for (int v = 1; v < 5; ++v) F[v] -= nh[0] * fc[v - 1] + nh[1] * fc[4 + v - 1] + nh[2] * fc[8 + v - 1];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sD[(le * 5 + v) * NF + fp] = F[v];
  }
  lds_barrier();
  for (int it = tid; it < EB * NU; it += NT) {
    const int le = it / NU, s = it - le * NU, e = e0 + le;
    if (e >= E) continue;
    R acc[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] = Rp[(size_t)e * 5 * NU + v * NU + s];
    {
      // lifting row (a plain partly unrolled loop: the fully unrolled product
      // ahead of the RK store needed all registers)
      const R* Arow = ops + C::O_M3 + s * NF;
      const R* Bv = sD + le * 5 * NF;
#pragma unroll 4
      for (int k = 0; k < NF; ++k) {
        const R w = Arow[k];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += w * Bv[v * NF + k];
      }
    }
    const double dj = sg.detj[e];
#pragma unroll
    for (int v = 0; v < 5; ++v) rk_store(sg, rk, (size_t)e * 5 * NU + v * NU + s, -double(acc[v]) / dj);
  }
}

// ------------------------------------------------------------ host side
template <int ET, int P, typename R>
static void pack_dense(const RefElem& r, R* o) {
  using C = DenseCfg<ET, P>;
  constexpr int NU = C::NU, NF = C::NF, NQ = C::NQ, KG = C::KG;
  for (int f = 0; f < NF; ++f)
    for (int u = 0; u < NU; ++u) o[C::O_M0 + f * NU + u] = R(r.M0[f * NU + u]);
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < NU; ++s) {
      R* row = o + C::O_G + (d * NU + s) * KG;
      for (int u = 0; u < NU; ++u) row[u] = R(r.Dg[(d * NU + s) * NU + u]);
      for (int f = 0; f < NF; ++f) row[NU + f] = R(r.face_normal[3 * C::face_of(f) + d] * r.M3[s * NF + f]);
    }
  for (int q = 0; q < NQ; ++q)
    for (int u = 0; u < NU; ++u) o[C::O_M7 + q * NU + u] = R(r.M7[q * NU + u]);
  for (int i = 0; i < 3 * NU * NQ; ++i) o[C::O_AP + i] = R(r.APd[i]);
  for (int i = 0; i < NU * NF; ++i) o[C::O_M3 + i] = R(r.M3[i]);
  for (int i = 0; i < 3 * C::NFACE; ++i) o[C::O_N + i] = R(r.face_normal[i]);
  if constexpr (C::PYR)
    for (int i = 0; i < 3 * NU * NU; ++i) o[C::O_KU + i] = R(r.Ku[i]);
  // matrix-core copies (lane order, zero padded)
  auto tiles = [&](int off, int MT, int KS, auto val) {
    for (int mt = 0; mt < MT; ++mt)
      for (int ks = 0; ks < KS; ++ks)
        for (int l = 0; l < 64; ++l) o[off + (mt * KS + ks) * 64 + l] = R(val(mt * 16 + l % 16, ks * 4 + l / 16));
  };
  tiles(C::O_PM0, C::MTF, C::KSU, [&](int row, int k) { return row < NF && k < NU ? r.M0[row * NU + k] : 0.0; });
  tiles(C::O_PG, C::MTG, C::KSU + C::KSF, [&](int row, int k) {
    if (row >= 3 * NU) return 0.0;
    const int d = row / NU, s = row % NU;
    if (k < 4 * C::KSU) return k < NU ? r.Dg[(d * NU + s) * NU + k] : 0.0;
    const int f = k - 4 * C::KSU;
    return f < NF ? r.face_normal[3 * C::face_of(f) + d] * r.M3[s * NF + f] : 0.0;
  });
  tiles(C::O_PM7, C::MTQ, C::KSU, [&](int row, int k) { return row < NQ && k < NU ? r.M7[row * NU + k] : 0.0; });
  tiles(C::O_PAP, C::MTU, 3 * C::KSQ, [&](int row, int k) {
    const int d = k / (4 * C::KSQ), q = k % (4 * C::KSQ);
    return row < NU && q < NQ ? r.APd[(d * NU + row) * NQ + q] : 0.0;
  });
  tiles(C::O_PK0, C::MTU, 3 * C::KSU, [&](int row, int k) {
    const int d = k / (4 * C::KSU), u = k % (4 * C::KSU);
    if (row >= NU || u >= NU) return 0.0;
    if (C::PYR) return r.Ku[(d * NU + row) * NU + u];
    long double acc = r.Dg[(d * NU + row) * NU + u];
    for (int f = 0; f < NF; ++f)
      acc -= (long double)r.M3[row * NF + f] * r.face_normal[3 * C::face_of(f) + d] * r.M0[f * NU + u];
    return (double)acc;
  });
}

template <int ET>
static size_t dense_size(int p) {
  switch (p) {
    case 1: return DenseCfg<ET, 1>::SIZE;
    case 2: return DenseCfg<ET, 2>::SIZE;
    case 3: return DenseCfg<ET, 3>::SIZE;
    case 4: return DenseCfg<ET, 4>::SIZE;
  }
  return 0;
}

// the double-precision disu block: M0 and Lv_d (long double on the host)
template <int ET, int P>
static void pack_disu(const RefElem& r, double* o) {
  using C = DenseCfg<ET, P>;
  using DD = DenseDisu<ET, P>;
  constexpr int NU = C::NU, NF = C::NF;
  for (int i = 0; i < NF * NU; ++i) o[DD::O_M0 + i] = r.M0[i];
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < NU; ++s)
      for (int u = 0; u < NU; ++u) {
        long double acc;
        if (C::PYR) {
          acc = r.Ku[(d * NU + s) * NU + u];
          for (int f = 0; f < NF; ++f)
            acc += (long double)r.M3[s * NF + f] * r.face_normal[3 * C::face_of(f) + d] * r.M0[f * NU + u];
        } else {
          acc = r.Dg[(d * NU + s) * NU + u];
        }
        o[DD::O_LV + (d * NU + s) * NU + u] = (double)acc;
      }
}

template <int ET, int P>
static size_t dense_bytes_t(size_t rs) {
  return dense_disu_offset<ET, P>(rs) + sizeof(double) * DenseDisu<ET, P>::SIZE;
}

template <int ET>
static size_t dense_bytes_e(int p, size_t rs) {
  switch (p) {
    case 1: return dense_bytes_t<ET, 1>(rs);
    case 2: return dense_bytes_t<ET, 2>(rs);
    case 3: return dense_bytes_t<ET, 3>(rs);
    case 4: return dense_bytes_t<ET, 4>(rs);
  }
  return 0;
}

// the device table: the operators in the working precision, then the
// double-precision disu block
size_t dense_ops_bytes(int etype, int p, int prec) {
  const size_t rs = prec == 0 ? 8 : 4;
  return etype == 3 ? dense_bytes_e<3>(p, rs) : etype == 2 ? dense_bytes_e<2>(p, rs) : 0;
}

template <int ET, int P, typename R>
static void pack_dense_t(const RefElem& r, R* dst) {
  pack_dense<ET, P>(r, dst);
  pack_disu<ET, P>(r, (double*)((char*)dst + dense_disu_offset<ET, P>(sizeof(R))));
}

template <int ET, typename R>
static void pack_dense_p(const RefElem& r, R* dst) {
  switch (r.p) {
    case 1: pack_dense_t<ET, 1>(r, dst); break;
    case 2: pack_dense_t<ET, 2>(r, dst); break;
    case 3: pack_dense_t<ET, 3>(r, dst); break;
    case 4: pack_dense_t<ET, 4>(r, dst); break;
  }
}

void dense_ops_pack(const RefElem& r, int prec, void* dst) {
  const bool d = prec == 0;
  if (r.etype == 2)
    d ? pack_dense_p<2>(r, (double*)dst) : pack_dense_p<2>(r, (float*)dst);
  else if (r.etype == 3)
    d ? pack_dense_p<3>(r, (double*)dst) : pack_dense_p<3>(r, (float*)dst);
}


// elements per workgroup of the volume kernel: about one quadrature point
// per thread at 256 threads; the workgroup then takes enough threads for one
// item per thread in every phase ((point, direction) rows, quadrature points,
// flux points), since a second pass made the compiler keep the operands of
// both passes live
template <int ET, int P>
struct DenseLaunch {
  using C = DenseCfg<ET, P>;
  static constexpr int NQ = C::NQ;
  static constexpr int EB = NQ >= 256 ? 1 : (256 / NQ > 16 ? 16 : 256 / NQ);
  static constexpr int MX0 = EB * 3 * C::NU > EB * NQ ? EB * 3 * C::NU : EB * NQ;
  static constexpr int MX = MX0 > EB * C::NF ? MX0 : EB * C::NF;
  static constexpr int NT = (MX + 63) / 64 * 64;
};
constexpr int DENSE_DISU_EB = 8, DENSE_DISU_NT = 256, DENSE_SURF_EB = 8;

template <int ET, int P, typename R>
static hipError_t dense_rhs_t(const TypeArgs& a, hipStream_t st) {
  const R* ops = (const R*)a.dops;
  const double* dops = (const double*)((const char*)a.dops + dense_disu_offset<ET, P>(sizeof(R)));
  // tetrahedra and pyramids are affine: the mass flux and the linear
  // energy-flux part come from the double-precision L(rho v)
  const Gas<R> g = make_gas<R>(*a.gas, true);
  const double eref = a.gas->pref / (a.gas->gamma - 1.0), rho0 = a.gas->rho_ref;
  const int E = a.one.E;
  constexpr int EB = DenseLaunch<ET, P>::EB, NTV = DenseLaunch<ET, P>::NT;
  if ((a.stage & 1) && E > 0)
    hipLaunchKernelGGL((dense_disu<ET, P, R, DENSE_DISU_EB, DENSE_DISU_NT>),
                       dim3((E + DENSE_DISU_EB - 1) / DENSE_DISU_EB), dim3(DENSE_DISU_NT), 0, st, a.one, a.from_ust,
                       dops, eref, rho0, true);
  if ((a.stage & 2) && E > 0) {
    // p >= 3 on the matrix cores.  With anti-aliasing at 48^3 cells the
    // volume group runs 14-42% faster than the VALU kernel in FP32 and
    // 1.3-2.4x faster in FP64, except FP64 tetrahedra at p = 4 (21.7 ms
    // against 16.7 on the VALU).  At p <= 2 the tiles are too small and the
    // VALU kernel is faster.
    constexpr bool MF = P >= 3 && !(sizeof(R) == 8 && !DenseCfg<ET, P>::PYR && P >= 4);
    // FP64 doubles the LDS per element: half the elements per workgroup;
    // FP32 pyramids at p = 3: three (seven workgroups per CU, MfLean)
    constexpr int EBM = sizeof(R) == 8 ? (EB > 1 ? EB / 2 : 1) : (DenseCfg<ET, P>::PYR && P == 3 ? 3 : EB);
    if constexpr (MF) {
      if (a.aa)
        hipLaunchKernelGGL((dense_volume_mf<ET, P, R, EBM, 256, true>), dim3((E + EBM - 1) / EBM), dim3(256), 0, st,
                           a.one, a.from_ust, ops, g, eref, rho0);
      else
        hipLaunchKernelGGL((dense_volume_mf<ET, P, R, EBM, 256, false>), dim3((E + EBM - 1) / EBM), dim3(256), 0, st,
                           a.one, a.from_ust, ops, g, eref, rho0);
    } else {
      if (a.aa)
        hipLaunchKernelGGL((dense_volume<ET, P, R, EB, NTV, true>), dim3((E + EB - 1) / EB), dim3(NTV), 0, st,
                           a.one, a.from_ust, ops, g, eref, rho0);
      else
        hipLaunchKernelGGL((dense_volume<ET, P, R, EB, NTV, false>), dim3((E + EB - 1) / EB), dim3(NTV), 0, st,
                           a.one, a.from_ust, ops, g, eref, rho0);
    }
  }
  if ((a.stage & 4) && E > 0)
    hipLaunchKernelGGL((dense_surface<ET, P, R, DENSE_SURF_EB, 256>), dim3((E + DENSE_SURF_EB - 1) / DENSE_SURF_EB),
                       dim3(256), 0, st, a.one, a.rk, ops, g);
  return hipGetLastError();
}

template <int ET>
static hipError_t dense_rhs_e(const TypeArgs& a, int prec, hipStream_t st) {
  const bool d = prec == 0;
  switch (a.p) {
    case 1: return d ? dense_rhs_t<ET, 1, double>(a, st) : dense_rhs_t<ET, 1, float>(a, st);
    case 2: return d ? dense_rhs_t<ET, 2, double>(a, st) : dense_rhs_t<ET, 2, float>(a, st);
    case 3: return d ? dense_rhs_t<ET, 3, double>(a, st) : dense_rhs_t<ET, 3, float>(a, st);
    case 4: return d ? dense_rhs_t<ET, 4, double>(a, st) : dense_rhs_t<ET, 4, float>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t dense_rhs(int etype, const TypeArgs& a, int prec, hipStream_t st) {
  if (!a.dops) return hipErrorInvalidValue;
  if (etype == 2) return dense_rhs_e<2>(a, prec, st);
  if (etype == 3) return dense_rhs_e<3>(a, prec, st);
  return hipErrorInvalidValue;
}

}  // namespace fr
