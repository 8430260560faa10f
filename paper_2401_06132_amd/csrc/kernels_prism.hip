// Fused flux-reconstruction kernels for prisms (gfx950).
//
// Same kernel groups as the hexahedral kernels (section 6.1): disu | volume
// group | interface group.  The prism operators factor into a dense
// triangle-plane block times a sparse line operator (section 4.1, figure
// priplanarint):  M7 = I_line (x) T_q,  and the projection-divergence
//   (M1 - M3 M2) M9 F = (AP_xi (x) P_line) F_xi + (AP_eta (x) P_line) F_eta
//                     + (P_T (x) AP_line) F_zeta
// with P_T = M_T^-1 T_q^T W, AP_xi/eta = -M_T^-1 (d_xi/eta T_q)^T W (M_T the
// triangle mass matrix), i.e. the weak form of the DG divergence with the
// L2-projected flux.  Triangle blocks are applied by one thread per (field,
// plane) with all rows unrolled, so the operator entries are wave-uniform
// scalar loads; the line direction uses the same on-the-fly quadrature
// columns as the hexahedral kernel.
//
// Reference prism: triangle {xi, eta >= -1, xi + eta <= 0} x zeta in [-1,1];
// solution point t + NT k; faces 0/1 = zeta -1/+1 (triangle nodes), faces
// 2/3/4 = edges eta=-1, xi+eta=0, xi=-1 (GL points along the edge x GL in zeta,
// index i + n k).
#include <type_traits>

#include "fr_device.h"
#include "fr_kernels.h"

namespace fr {

template <int P, typename R>
struct PrismOps {
  static constexpr int n = P + 1, m = P + 3, NT = (P + 1) * (P + 2) / 2, NTQ = (P + 1) * (P + 1);
  // line factors (kernel argument)
  R I[m][n], D[n][n], Pj[n][m], AP[n][m];
  R lb[n], rb[n], liftL[n], liftR[n];
  R x[n], xq[m];  // GL(n) solution and GL(m) quadrature nodes
};

template <int P, typename R>
struct PrismTriOps {
  static constexpr int n = P + 1, NT = (P + 1) * (P + 2) / 2, NTQ = (P + 1) * (P + 1);
  R Tq[NTQ][NT];              // triangle nodal basis at the conical quadrature points
  R Dxi[NT][NT], Deta[NT][NT];  // triangle derivatives at the nodes
  R PT[NT][NTQ], APxi[NT][NTQ], APeta[NT][NTQ];
  R Tedge[3][n][NT];          // nodal basis at the GL points of each edge
  R LiftEdge[3][NT][n];       // DG lifting of an edge point into the plane
};
// the device table: the operators, then the triangle nodes and conical
// quadrature points (needed by curved prisms only; the volume kernel stages
// them in LDS only then, so the affine kernels keep their LDS size)
template <int P, typename R>
struct PrismTri : PrismTriOps<P, R> {
  static constexpr int NT = PrismTriOps<P, R>::NT, NTQ = PrismTriOps<P, R>::NTQ;
  R nodes[NT][2], qp[NTQ][2];
};

// Curved prisms: the map of the six vertices X (vertex t + 3c at triangle
// vertex t of (-1,-1), (1,-1), (-1,1) and zeta = 2c - 1) by
// lambda_t(xi, eta) (1 -+ zeta)/2.  At reference point (xi, eta, zeta): the
// columns J_c = dx/dxi_c, the cofactor rows S_d = J_{d+1} x J_{d+2}
// (S = det J J^-1) and det J = J_0 . S_0.
template <typename R>
__device__ __forceinline__ void wedge_metric(const R* X, R xi, R eta, R zeta, R S[3][3], R& det) {
  const R zm = R(0.5) * (R(1) - zeta), zp = R(0.5) * (R(1) + zeta);
  const R l0 = -R(0.5) * (xi + eta), l1 = R(0.5) * (R(1) + xi), l2 = R(0.5) * (R(1) + eta);
  R J[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    J[0][i] = R(0.5) * (zm * (X[3 + i] - X[i]) + zp * (X[12 + i] - X[9 + i]));
    J[1][i] = R(0.5) * (zm * (X[6 + i] - X[i]) + zp * (X[15 + i] - X[9 + i]));
    J[2][i] = R(0.5) * (l0 * (X[9 + i] - X[i]) + l1 * (X[12 + i] - X[3 + i]) + l2 * (X[15 + i] - X[6 + i]));
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R* a = J[(d + 1) % 3];
    const R* b = J[(d + 2) % 3];
    S[d][0] = a[1] * b[2] - a[2] * b[1];
    S[d][1] = a[2] * b[0] - a[0] * b[2];
    S[d][2] = a[0] * b[1] - a[1] * b[0];
  }
  det = J[0][0] * S[0][0] + J[0][1] * S[0][1] + J[0][2] * S[0][2];
}

// reference coordinates (xi, eta) of GL point s along edge e (counter-clockwise)
template <typename R>
__device__ __forceinline__ void edge_point(int e, R s, R& xi, R& eta) {
  xi = e == 0 ? s : (e == 1 ? -s : R(-1));
  eta = e == 0 ? R(-1) : (e == 1 ? s : -s);
}

template <int P>
struct PrismCfg {
  static constexpr int n = P + 1, m = P + 3, NT = (P + 1) * (P + 2) / 2, NTQ = (P + 1) * (P + 1);
  static constexpr int NU = NT * n, NFP = n * n;
  // face arrays: an element's faces are stored with their own point counts,
  // the two triangles (NT points) then the three quadrilaterals (n^2)
  static constexpr int PPE = 2 * NT + 3 * NFP;
  __host__ __device__ static constexpr int fsz(int f) { return f < 2 ? NT : NFP; }
  __host__ __device__ static constexpr int foff(int f) { return f < 2 ? f * NT : 2 * NT + (f - 2) * NFP; }
  static constexpr int SZ_X = 20 * NU;
  static constexpr int SZ_J = 25 * NFP;  // 5 faces x 5 variables
  static constexpr int SZ_Z = 15 * NTQ * n;
  static constexpr int SZ_A = (SZ_X + SZ_J > SZ_Z) ? SZ_X + SZ_J : SZ_Z;
  static constexpr int SZ_T1 = 20 * n * NTQ;
  static constexpr int PER_ELEM = SZ_A + SZ_T1;
};

// reference unit normals of the three quadrilateral faces (xi, eta components)
template <typename R>
__device__ __forceinline__ void edge_normal(int e, R& nx, R& ny) {
  const R h = R(0.70710678118654752440);
  nx = e == 0 ? R(0) : (e == 1 ? h : R(-1));
  ny = e == 0 ? R(-1) : (e == 1 ? h : R(0));
}

template <int N, typename R>
__device__ __forceinline__ R psel(const R (&v)[N], int idx) {
  R r = v[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = idx == k ? v[k] : r;
  return r;
}

// ----------------------------------------------------------------- disu
// Double-precision operators of the disu kernel, stored after the prism
// table in the same device allocation.
template <int P>
struct PrismDisuTab {
  static constexpr int n = P + 1, NT = (P + 1) * (P + 2) / 2;
  double lb[n], rb[n], D[n][n];   // line: l_k(-1), l_k(+1), l_j' at the GL points
  double Tedge[3][n][NT];         // nodal basis at the GL points of each edge
  double Dxi[NT][NT], Deta[NT][NT];
};

// byte offset of the disu table behind the prism table
template <int P, typename R>
constexpr size_t prism_disu_offset() {
  return (sizeof(PrismTri<P, R>) + 255) / 256 * 256;
}

// Group 1 (eq. FR-disu) in double precision, as for hexahedra: triangle
// faces by the zeta lines, quadrilateral faces by the edge interpolation of
// each triangle plane; single precision stores a float base per face (the
// value at its first flux point) and the deviations.  LIN: the mass-flux
// divergence L(rho v) = D_xi (S m)_xi + D_eta (S m)_eta + D_zeta (S m)_zeta
// to row 0 of the volume residual.
template <int P, typename R, int EB, int NT_, bool BT>
__global__ void __launch_bounds__(NT_) prism_disu(const Seg one, const BlkRef* __restrict__ bt,
                                                  const Seg* __restrict__ segs, const bool from_ust,
                                                  const PrismDisuTab<P>* __restrict__ tab, const double eref,
                                                  const double rho0, const bool lin) {
  using C = PrismCfg<P>;
  constexpr int n = C::n, NT = C::NT, NU = C::NU, NFP = C::NFP;
  constexpr bool FB = sizeof(R) == 4;
  __shared__ double sU[EB * 5 * NU];
  __shared__ double sS[EB][9];
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  R* __restrict__ Uf = (R*)sg.Uf;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
  constexpr int NS = (EB * 5 * NU + NT_ - 1) / NT_;
  double xs[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int it = tid + k * NT_;
    const bool ok = it < EB * 5 * NU && e0 + it / (5 * NU) < E;
    xs[k] = U[ok ? (size_t)e0 * 5 * NU + it : 0];
  }
  if (lin && tid < EB * 9) {
    const int le = tid / 9, k = tid - le * 9;
    const R* __restrict__ met = (const R*)sg.met;
    const size_t e = e0 + le < E ? (size_t)(e0 + le) : 0;
    sS[le][k] = double(met[e * 10 + 9]) * double(met[e * 10 + k]);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int it = tid + k * NT_;
    if (it < EB * 5 * NU) {
      const int r = it % (5 * NU);
      double x = xs[k];
      if (r >= 4 * NU) x -= eref;
      if (r < NU) x -= rho0;
      sU[it] = x;
    }
  }
  lds_barrier();
  // triangle faces: line interpolation in zeta at every node
  for (int it = tid; it < EB * 5 * NT; it += NT_) {
    const int le = it / (5 * NT), r = it - le * (5 * NT), v = r / NT, t = r - v * NT, e = e0 + le;
    if (e >= E) continue;
    const double* X = sU + le * 5 * NU + v * NU;
    double xm = 0.0, xp = 0.0, bm = 0.0, bp = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      xm += tab->lb[k] * X[t + NT * k];
      xp += tab->rb[k] * X[t + NT * k];
      bm += tab->lb[k] * X[NT * k];
      bp += tab->rb[k] * X[NT * k];
    }
    const size_t s0 = (size_t)(slot_base + e * 5);
    R* __restrict__ um = Uf + (size_t)(sg.po_base + e * C::PPE) * 5 + v * NT + t;  // face 0
    R* __restrict__ up = um + 5 * NT;                                               // face 1
    if constexpr (FB) {
      const float fm = float(bm), fp = float(bp);
      *um = R(xm - double(fm));
      *up = R(xp - double(fp));
      if (t == 0) {
        sg.Ub[s0 * 5 + v] = fm;
        sg.Ub[(s0 + 1) * 5 + v] = fp;
      }
    } else {
      *um = R(xm);
      *up = R(xp);
    }
  }
  // quadrilateral faces: triangle-plane interpolation to the edge points;
  // the base of edge face ed is its value at (i, k) = (0, 0)
  for (int it = tid; it < EB * 5 * n; it += NT_) {
    const int le = it / (5 * n), r = it - le * (5 * n), v = r / n, k = r - v * n, e = e0 + le;
    if (e >= E) continue;
    const double* X = sU + le * 5 * NU + v * NU;
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      const size_t slot = (size_t)(slot_base + e * 5 + 2 + ed);
      float fb = 0.0f;
      if constexpr (FB) {
        double b0 = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) b0 += tab->Tedge[ed][0][t] * X[t];
        fb = float(b0);
        if (k == 0) sg.Ub[slot * 5 + v] = fb;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) s += tab->Tedge[ed][i][t] * X[t + NT * k];
        Uf[(size_t)(sg.po_base + e * C::PPE + C::foff(2 + ed)) * 5 + v * NFP + i + n * k] = R(FB ? s - double(fb) : s);
      }
    }
  }
  if (!lin) return;
  lds_barrier();
  // the transformed mass flux (S m)_d at every point, in place over the
  // momentum (each point is read and written by one thread)
  for (int it = tid; it < EB * NU; it += NT_) {
    const int le = it / NU, s = it - le * NU;
    double* M = sU + le * 5 * NU + NU;
    const double m0 = M[s], m1 = M[NU + s], m2 = M[2 * NU + s];
#pragma unroll
    for (int d = 0; d < 3; ++d) M[d * NU + s] = sS[le][3 * d] * m0 + sS[le][3 * d + 1] * m1 + sS[le][3 * d + 2] * m2;
  }
  lds_barrier();
  R* __restrict__ Rp = (R*)sg.Rp;
  for (int it = tid; it < EB * NU; it += NT_) {
    const int le = it / NU, s = it - le * NU, e = e0 + le;
    if (e >= E) continue;
    const int k = s / NT, t = s - k * NT;
    const double* M = sU + le * 5 * NU + NU;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NT; ++c) acc += tab->Dxi[t][c] * M[c + NT * k] + tab->Deta[t][c] * M[NU + c + NT * k];
#pragma unroll
    for (int q = 0; q < n; ++q) acc += tab->D[k][q] * M[2 * NU + t + NT * q];
    Rp[(size_t)e * 5 * NU + s] = R(acc);
  }
}

// --------------------------------------------------------------- volume
// LDS per element: region A = state + gradients at the solution points;
// region B = neighbour face states / jumps and face fields.  The
// triangle-interpolated fields T1 are written from offset 0 over both once
// every thread holds its plane values in registers (the state and gradients
// are dead after the plane sweep), then the line-projected flux Z (after a
// barrier).  The footprint is the largest of A + B, T1 and Z (p = 3: 1780
// values instead of 2160).  Measured at 48^3 (volume group): FP32 p = 4
// 4.92 -> 4.62 ms (7 one-wave workgroups per CU instead of 6), FP64 p = 3
// 4.36 -> 3.43 ms (4 instead of 3); FP32 p = 3 is bound by registers and
// unchanged.  FP64 at p = 4 keeps T1 and Z after region A.  The triangle
// operator tables are staged in LDS once per workgroup so that every
// triangle-plane product can run one output point per thread.
template <int P, bool LIN>
struct PrismVol {
  static constexpr int n = P + 1, m = P + 3, NTN = (P + 1) * (P + 2) / 2, NTQ = (P + 1) * (P + 1);
  static constexpr int NU = NTN * n, NFP = n * n;
  // variables whose flux is projected: LIN leaves out the mass flux (its
  // divergence is L(rho v), formed by the disu kernel)
  static constexpr int NVF = LIN ? 4 : 5, V0 = 5 - NVF;
  static constexpr int SZ_A = 20 * NU;
  // padded strides keep the LDS accesses of both writer and reader free of
  // bank conflicts: T1 rows of NTQ + 1, Z variables NTQ n + 4 apart
  static constexpr int TQS = NTQ + 1, ZVS = NTQ * n + 4;
  static constexpr int SZ_J = 25 * NFP, SZ_T1 = 20 * n * TQS, SZ_Z = 3 * NVF * ZVS;
  static constexpr int EFS = 3 * NFP + 1;  // the 20 fields at the quadrilateral-face points,
  static constexpr int SZ_EF = 20 * EFS;   // odd stride per field (no bank conflicts)
  static constexpr int SZ_JE = SZ_J > SZ_EF ? SZ_J : SZ_EF;
  static constexpr int SZ_B0 = SZ_T1 > SZ_Z ? SZ_T1 : SZ_Z;
  static constexpr int SZ_B1 = SZ_B0 > SZ_J ? SZ_B0 : SZ_J;
  static constexpr int SZ_B = SZ_B1 > SZ_EF ? SZ_B1 : SZ_EF;
  static constexpr int PER_ELEM = SZ_A + SZ_B;
  // with T1 and Z over region A (TOX): the largest of A + (J, EF, S), T1, Z
  static constexpr int per_elem_tox(bool SAA) {
    const int b0 = SAA && SZ_S > SZ_JE ? SZ_S : SZ_JE;
    const int t = SZ_T1 > SZ_Z ? SZ_T1 : SZ_Z;
    return SZ_A + b0 > t ? SZ_A + b0 : t;
  }
  // surface-flux anti-aliasing, one round per face kind: the 20 fields at
  // the two triangles' nodes [2][20][NTN] or along one quadrilateral's first
  // axis at GL(m) [20][m][n] (offset 0); the viscous flux at the face
  // quadrature points [2][4][NTQ] or [4][m][m] (offset SZ_S0)
  static constexpr int SZ_S0 = 40 * NTN > 20 * m * n ? 40 * NTN : 20 * m * n;
  static constexpr int SZ_S = SZ_S0 + (8 * NTQ > 4 * m * m ? 8 * NTQ : 4 * m * m);
  static_assert(SZ_S <= SZ_B, "face quadrature staging fits region B");
};

// sum of a value over an adjacent lane pair (lanes 2i, 2i+1), both lanes get
// the same bits (addition is commutative)
__device__ __forceinline__ float pair_sum(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false);
  return x + __int_as_float(y);
}
__device__ __forceinline__ double pair_sum(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return x + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// AA: flux anti-aliasing; without it the flux is evaluated at the solution
// points and its divergence is taken in strong form, (M1 - M3 M2) F~: the
// derivative blocks minus the lifted normal flux interpolated to the faces.
// SAA: surface-flux anti-aliasing (built with AA only).  The face quadrature
// rules are the volume rule's factors: the conical triangle rule on the two
// triangles and GL(m)^2 on the quadrilaterals.  As for hexahedra, each side
// evaluates its normal viscous flux at the face quadrature points and stores
// its projection onto the flux points: P_T = M_T^-1 T_q^T W on a triangle
// (M_T the triangle mass matrix; lifting the projection reproduces the
// quadrature-point lifting because the rule integrates M_T exactly) and
// P x P on a quadrilateral.
template <int P, typename R, int EB, int NT_, bool BT, bool AA, bool SAA, bool WARP>
__global__ void __launch_bounds__(NT_)
    prism_volume(const Seg one, const BlkRef* __restrict__ bt, const Seg* __restrict__ segs, const bool from_ust,
                 const PrismOps<P, R> op, const PrismTri<P, R>* __restrict__ tri_g, const Gas<R> g,
                 const double eref, const double rho0) {
  // LIN: the mass flux's divergence and the linear energy-flux part come
  // from the disu kernel's L(rho v) (affine elements only)
  constexpr bool LIN = !WARP;
  using C = PrismVol<P, LIN>;
  constexpr int n = C::n, m = C::m, NTN = C::NTN, NTQ = C::NTQ, NU = C::NU, NFP = C::NFP;
  constexpr int NVF = C::NVF, V0 = C::V0;
  using F = PrismCfg<P>;  // face array layout
  // single precision up to p = 3: triangle-plane work one (field, plane) per
  // thread with broadcast operator reads (enough planes fill the workgroup);
  // otherwise one output point per thread
  constexpr bool PL = sizeof(R) == 4 && P <= 3;
  // with flux AA, T1 and Z start at offset 0 over the state and gradients,
  // which are dead after the plane sweep (FP64 at p = 4 keeps them after
  // region A: the plane values held in registers across the barrier spill)
  constexpr bool TOX = !(P >= 4 && sizeof(R) == 8);
  constexpr int PE = AA ? (TOX ? C::per_elem_tox(SAA) : C::PER_ELEM) : C::SZ_A + (PL ? C::SZ_JE : C::SZ_J);
  static_assert(2 * EB * NTQ <= NT_, "two threads per quadrature column");
  using TriL = typename std::conditional<WARP, PrismTri<P, R>, PrismTriOps<P, R>>::type;
  __shared__ TriL tri;
  __shared__ R smem[EB * PE];
  __shared__ R sMet[EB][10];
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  const R* __restrict__ Uf = (const R*)sg.Uf;
  R* __restrict__ Vf = (R*)sg.Vf;
  R* __restrict__ Rp = (R*)sg.Rp;
  const FaceRec* __restrict__ faces = sg.faces;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
  const uint8_t* __restrict__ perms = sg.perms;
  const R* __restrict__ met = (const R*)sg.met;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
#define XS(le) (smem + (le)*PE)            /* [20][NU]                 */
#define JS(le) (smem + (le)*PE + C::SZ_A)  /* [5][5][NFP]              */
#define TS(le) (smem + (le)*PE + (TOX ? 0 : C::SZ_A)) /* [20][n][TQS]  */
#define ZS(le) (smem + (le)*PE + (TOX ? 0 : C::SZ_A)) /* [3][NVF][ZVS] */
#define SS(le) (smem + (le)*PE + C::SZ_A)  /* face quadrature staging   */

  // phase 0: operator tables, state (reference form), metrics, neighbour states
  {
    constexpr int NW = sizeof(TriL) / sizeof(R);
    const R* src = reinterpret_cast<const R*>(tri_g);
    R* dst = reinterpret_cast<R*>(&tri);
    for (int it = tid; it < NW; it += NT_) dst[it] = src[it];
  }
  // face records, face geometry and the permutation table go to LDS first,
  // so the neighbour gather is one global load per value; every thread
  // issues all of its state and gather loads before the first use
  __shared__ FaceRec sFR[EB * 5];
  __shared__ R sFG[EB * 5][4];
  __shared__ uint8_t sPerm[MAX_PERMS * NFP];
  // out-of-range items load from a valid address (the segment's first
  // element) without a select afterwards, so every load stays in flight;
  // their values never reach an output (all stores are guarded)
  for (int it = tid; it < EB * 5; it += NT_) {
    const int slot = slot_base + (e0 + it / 5 < E ? e0 * 5 + it : 0);
    sFR[it] = faces[slot];
#pragma unroll
    for (int k = 0; k < 4; ++k) sFG[it][k] = fgeo[4 * slot + k];
  }
  for (int it = tid; it < sg.nperm * NFP; it += NT_) sPerm[it] = perms[it];
  __shared__ R sV[WARP ? EB : 1][18];  // curved: element vertices
  if constexpr (WARP) {
    const R* __restrict__ vx = (const R*)sg.verts;
    for (int it = tid; it < EB * 18; it += NT_) {
      const int le = it / 18;
      sV[le][it - le * 18] = vx[e0 + le < E ? (size_t)e0 * 18 + it : 0];
    }
  }
  for (int it = tid; it < EB * 10; it += NT_) {
    const int le = it / 10, k = it - le * 10, e = e0 + le;
    sMet[le][k] = met[e < E ? (size_t)e * 10 + k : 0];
  }
  // the state element by element (item r = tid + k NT_ of each element: its
  // LDS position and reference-state shift follow from tid and constants)
  const int nv = E - e0 < EB ? E - e0 : EB;  // valid elements of the batch
  constexpr int NR = (5 * NU + NT_ - 1) / NT_;
  double xs[EB][NR];
#pragma unroll
  for (int le = 0; le < EB; ++le)
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = tid + k * NT_;
      xs[le][k] = U[le < nv && r < 5 * NU ? (size_t)(e0 + le) * 5 * NU + r : 0];
    }
  lds_barrier();
  // neighbour face values: one own flux point per item with its five fields
  // (the element's points in face-array order: two triangles, three
  // quadrilaterals); out-of-range items read the first item's addresses
  constexpr int NG = (EB * F::PPE + NT_ - 1) / NT_;
  R gv[NG][5], gb[NG][5];
  auto face_point = [](int q, int& f, int& r) {
    f = q < 2 * NTN ? q / NTN : 2 + (q - 2 * NTN) / NFP;
    r = q - F::foff(f);
  };
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const int it = tid + k * NT_;
    const int itc = it < EB * F::PPE ? it : 0;
    const int le = itc / F::PPE;
    int f, r;
    face_point(itc - le * F::PPE, f, r);
    const FaceRec fr = sFR[le * 5 + f];
    const R* __restrict__ src = Uf + (size_t)fr.npo * 5 + sPerm[(fr.info >> 1) * NFP + r];
    const int fs = F::fsz(f);
#pragma unroll
    for (int v = 0; v < 5; ++v) gv[k][v] = src[v * fs];
    if constexpr (sizeof(R) == 4) {
#pragma unroll
      for (int v = 0; v < 5; ++v) gb[k][v] = sg.Ub[(size_t)fr.nbr * 5 + v];  // the face base
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int r = tid + k * NT_;
    if (r < 5 * NU) {
      const double sh = r < NU ? rho0 : (r >= 4 * NU ? eref : 0.0);
#pragma unroll
      for (int le = 0; le < EB; ++le) XS(le)[r] = R(xs[le][k] - sh);
    }
  }
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const int it = tid + k * NT_;
    if (it < EB * F::PPE) {
      const int le = it / F::PPE;
      int f, r;
      face_point(it - le * F::PPE, f, r);
      R* dst = JS(le) + f * 5 * NFP + r;
#pragma unroll
      for (int v = 0; v < 5; ++v) dst[v * NFP] = sizeof(R) == 4 ? gv[k][v] + gb[k][v] : gv[k][v];
    }
  }
  lds_barrier();

  // phase 1: jumps C - u^f (eq. FR-conu) at every own flux point, in place
  // over the neighbour values: triangle faces (line interpolation in zeta,
  // one line per thread), quadrilateral faces (triangle-plane interpolation
  // to the edge points): per plane (PL) or per edge point.
  constexpr int NJ_TRI = 5 * NTN, NJ_QUAD = PL ? 5 * n : 5 * 3 * n * n;
  for (int it = tid; it < EB * (NJ_TRI + NJ_QUAD); it += NT_) {
    const int le = it / (NJ_TRI + NJ_QUAD), r0 = it - le * (NJ_TRI + NJ_QUAD);
    const R* X = XS(le);
    if (r0 < NJ_TRI) {
      const int v = r0 / NTN, t = r0 - v * NTN;
      R xm = R(0), xp = R(0);
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const R x = X[v * NU + t + NTN * k];
        xm += op.lb[k] * x;
        xp += op.rb[k] * x;
      }
      const int im = sFR[le * 5].info, ip = sFR[le * 5 + 1].info;
      R* jm = JS(le) + (0 * 5 + v) * NFP + t;
      R* jp = JS(le) + (1 * 5 + v) * NFP + t;
      *jm = ((im & 1) ? R(0.5) + g.beta : R(0.5) - g.beta) * (*jm - xm);
      *jp = ((ip & 1) ? R(0.5) + g.beta : R(0.5) - g.beta) * (*jp - xp);
    } else if constexpr (PL) {
      const int r1 = r0 - NJ_TRI, v = r1 / n, k = r1 - v * n;
      R x[NTN];
#pragma unroll
      for (int t = 0; t < NTN; ++t) x[t] = X[v * NU + t + NTN * k];
#pragma unroll
      for (int ed = 0; ed < 3; ++ed) {
        const R w = (sFR[le * 5 + 2 + ed].info & 1) ? R(0.5) + g.beta : R(0.5) - g.beta;
#pragma unroll
        for (int i = 0; i < n; ++i) {
          R s = R(0);
#pragma unroll
          for (int t = 0; t < NTN; ++t) s += tri.Tedge[ed][i][t] * x[t];
          R* jj = JS(le) + ((2 + ed) * 5 + v) * NFP + i + n * k;
          *jj = w * (*jj - s);
        }
      }
    } else {
      const int r1 = r0 - NJ_TRI, v = r1 / (3 * n * n), r2 = r1 - v * (3 * n * n), ed = r2 / (n * n);
      const int r3 = r2 - ed * (n * n), k = r3 / n, i = r3 - k * n;
      R s = R(0);
#pragma unroll
      for (int t = 0; t < NTN; ++t) s += tri.Tedge[ed][i][t] * X[v * NU + t + NTN * k];
      const int info = sFR[le * 5 + 2 + ed].info;
      R* jj = JS(le) + ((2 + ed) * 5 + v) * NFP + i + n * k;
      *jj = ((info & 1) ? R(0.5) + g.beta : R(0.5) - g.beta) * (*jj - s);
    }
  }
  lds_barrier();

  // phase 2: corrected reference gradient (eq. FR-qfinal): zeta along the
  // lines with the triangle-face lifting; (xi, eta) with the triangle
  // derivative blocks and the quadrilateral-face lifting (per plane or per
  // point, as in phase 1)
  constexpr int NG_Z = 5 * NTN, NG_T = PL ? 5 * n : 5 * n * NTN;
  for (int it = tid; it < EB * (NG_Z + NG_T); it += NT_) {
    const int le = it / (NG_Z + NG_T), r0 = it - le * (NG_Z + NG_T);
    R* X = XS(le);
    const R* J = JS(le);
    if (r0 < NG_Z) {
      const int v = r0 / NTN, t = r0 - v * NTN;
      R x[n];
#pragma unroll
      for (int k = 0; k < n; ++k) x[k] = X[v * NU + t + NTN * k];
      const R jm = J[(0 * 5 + v) * NFP + t], jp = J[(1 * 5 + v) * NFP + t];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        R s = op.liftR[k] * jp - op.liftL[k] * jm;
#pragma unroll
        for (int c = 0; c < n; ++c) s += op.D[k][c] * x[c];
        X[(15 + v) * NU + t + NTN * k] = s;
      }
    } else if constexpr (PL) {
      const int r1 = r0 - NG_Z, v = r1 / n, k = r1 - v * n;
      R x[NTN], jq[3][n];
#pragma unroll
      for (int c = 0; c < NTN; ++c) x[c] = X[v * NU + c + NTN * k];
#pragma unroll
      for (int ed = 0; ed < 3; ++ed)
#pragma unroll
        for (int i = 0; i < n; ++i) jq[ed][i] = J[((2 + ed) * 5 + v) * NFP + i + n * k];
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        R sx = R(0), sy = R(0);
#pragma unroll
        for (int c = 0; c < NTN; ++c) {
          sx += tri.Dxi[t][c] * x[c];
          sy += tri.Deta[t][c] * x[c];
        }
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) {
          R nx, ny;
          edge_normal<R>(ed, nx, ny);
          R l = R(0);
#pragma unroll
          for (int i = 0; i < n; ++i) l += tri.LiftEdge[ed][t][i] * jq[ed][i];
          sx += nx * l;
          sy += ny * l;
        }
        X[(5 + v) * NU + t + NTN * k] = sx;
        X[(10 + v) * NU + t + NTN * k] = sy;
      }
    } else {
      const int r1 = r0 - NG_Z, v = r1 / (n * NTN), r2 = r1 - v * (n * NTN), k = r2 / NTN, t = r2 - k * NTN;
      R sx = R(0), sy = R(0);
#pragma unroll
      for (int c = 0; c < NTN; ++c) {
        const R x = X[v * NU + c + NTN * k];
        sx += tri.Dxi[t][c] * x;
        sy += tri.Deta[t][c] * x;
      }
#pragma unroll
      for (int ed = 0; ed < 3; ++ed) {
        R nx, ny;
        edge_normal<R>(ed, nx, ny);
        R l = R(0);
#pragma unroll
        for (int i = 0; i < n; ++i) l += tri.LiftEdge[ed][t][i] * J[((2 + ed) * 5 + v) * NFP + i + n * k];
        sx += nx * l;
        sy += ny * l;
      }
      X[(5 + v) * NU + t + NTN * k] = sx;
      X[(10 + v) * NU + t + NTN * k] = sy;
    }
  }
  lds_barrier();

  // phase 3: physical gradient q = J^-T q~ (eq. FR-gradcoru)
  for (int it = tid; it < EB * NU; it += NT_) {
    const int le = it / NU, s = it - le * NU;
    R* X = XS(le);
    R M[3][3];  // M[d][c] = (J^-1)_{dc}
    if constexpr (WARP) {
      const int t = s % NTN, k = s / NTN;
      R S[3][3], det;
      wedge_metric(&sV[le][0], tri.nodes[t][0], tri.nodes[t][1], psel(op.x, k), S, det);
      const R id = R(1) / det;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[d][c] = S[d][c] * id;
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[d][c] = sMet[le][3 * d + c];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R g0 = X[(5 + v) * NU + s], g1 = X[(10 + v) * NU + s], g2 = X[(15 + v) * NU + s];
#pragma unroll
      for (int c = 0; c < 3; ++c) X[(5 + c * 5 + v) * NU + s] = M[0][c] * g0 + M[1][c] * g1 + M[2][c] * g2;
    }
  }
  lds_barrier();

  if constexpr (SAA) {
    // phase 4a with surface-flux anti-aliasing.  Triangle round: S1 the 20
    // fields at both triangles' nodes (zeta lines), S2 T_q to the
    // triangle quadrature points and n . f^v there, S3 P_T back to the nodes.
    // Quadrilateral rounds (one per face): S1 the fields at the face's GL
    // points (edge interpolation per plane) and I along the edge, S2 I along
    // zeta and n . f^v at each GL(m)^2 point, S3 P x P back
    __shared__ R sI[m][n];   // rows read with a per-thread index
    __shared__ R sPj[n][m];
    if (tid < m * n) {
      sI[tid / n][tid % n] = op.I[tid / n][tid % n];
      sPj[tid / m][tid % m] = op.Pj[tid / m][tid % m];
    }
    for (int it = tid; it < EB * 20 * NTN; it += NT_) {
      const int le = it / (20 * NTN), r0 = it - le * (20 * NTN), fld = r0 / NTN, t = r0 - fld * NTN;
      const R* X = XS(le) + fld * NU + t;
      R sm = R(0), sp = R(0);
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const R x = X[NTN * k];
        sm += op.lb[k] * x;
        sp += op.rb[k] * x;
      }
      SS(le)[fld * NTN + t] = sm;
      SS(le)[(20 + fld) * NTN + t] = sp;
    }
    lds_barrier();
    for (int it = tid; it < EB * 2 * NTQ; it += NT_) {
      const int le = it / (2 * NTQ), r0 = it - le * (2 * NTQ), side = r0 / NTQ, q = r0 - side * NTQ;
      const R* FT = SS(le) + side * 20 * NTN;
      R w[20];
#pragma unroll
      for (int fld = 0; fld < 20; ++fld) {
        R s = R(0);
#pragma unroll
        for (int t = 0; t < NTN; ++t) s += tri.Tq[q][t] * FT[fld * NTN + t];
        w[fld] = s;
      }
      const int lf = le * 5 + side;
      const R sgn = (sFR[lf].info & 1) ? R(1) : R(-1);
      const R nn[3] = {sgn * sFG[lf][0], sgn * sFG[lf][1], sgn * sFG[lf][2]};
      R u[5], q3[3][5], V[4];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        u[v] = w[v];
#pragma unroll
        for (int d = 0; d < 3; ++d) q3[d][v] = w[5 + d * 5 + v];
      }
      normal_viscous(u, q3, nn, g, V);
      R* VT = SS(le) + C::SZ_S0 + side * 4 * NTQ + q;
#pragma unroll
      for (int k = 0; k < 4; ++k) VT[k * NTQ] = V[k];
    }
    lds_barrier();
    for (int it = tid; it < EB * 8 * NTN; it += NT_) {
      const int le = it / (8 * NTN), r0 = it - le * (8 * NTN), side = r0 / (4 * NTN), r1 = r0 - side * (4 * NTN);
      const int k = r1 / NTN, t = r1 - k * NTN, e = e0 + le;
      if (e >= E) continue;
      const R* VT = SS(le) + C::SZ_S0 + (side * 4 + k) * NTQ;
      R s = R(0);
#pragma unroll
      for (int q = 0; q < NTQ; ++q) s += tri.PT[t][q] * VT[q];
      Vf[(size_t)(sg.po_base + e * F::PPE + side * NTN) * 4 + k * NTN + t] = s;
    }
    // quadrilateral rounds: their S1 overwrites the triangle-node fields (read
    // before the last barrier) and their S2 the triangle viscous fluxes (read
    // above) only after the next barrier
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      for (int it = tid; it < EB * 20 * n; it += NT_) {
        const int le = it / (20 * n), r0 = it - le * (20 * n), fld = r0 / n, k = r0 - fld * n;
        const R* X = XS(le) + fld * NU + NTN * k;
        R xv[NTN];
#pragma unroll
        for (int t = 0; t < NTN; ++t) xv[t] = X[t];
        R y[n];
#pragma unroll
        for (int i = 0; i < n; ++i) {
          R s = R(0);
#pragma unroll
          for (int t = 0; t < NTN; ++t) s += tri.Tedge[ed][i][t] * xv[t];
          y[i] = s;
        }
        R* T = SS(le) + fld * m * n + k;
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) {
          R s = R(0);
#pragma unroll
          for (int i = 0; i < n; ++i) s += op.I[a2][i] * y[i];
          T[a2 * n] = s;
        }
      }
      lds_barrier();
      for (int it = tid; it < EB * m * m; it += NT_) {
        const int le = it / (m * m), r0 = it - le * (m * m), a2 = r0 / m, b2 = r0 - a2 * m;
        R Ib[n];
#pragma unroll
        for (int j = 0; j < n; ++j) Ib[j] = sI[b2][j];
        const R* T = SS(le) + a2 * n;
        R w[20];
#pragma unroll
        for (int fld = 0; fld < 20; ++fld) {
          R s = R(0);
#pragma unroll
          for (int k = 0; k < n; ++k) s += Ib[k] * T[fld * m * n + k];
          w[fld] = s;
        }
        const int lf = le * 5 + 2 + ed;
        const R sgn = (sFR[lf].info & 1) ? R(1) : R(-1);
        const R nn[3] = {sgn * sFG[lf][0], sgn * sFG[lf][1], sgn * sFG[lf][2]};
        R u[5], q3[3][5], V[4];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          u[v] = w[v];
#pragma unroll
          for (int d = 0; d < 3; ++d) q3[d][v] = w[5 + d * 5 + v];
        }
        normal_viscous(u, q3, nn, g, V);
        R* VQ = SS(le) + C::SZ_S0 + a2 * m + b2;
#pragma unroll
        for (int k = 0; k < 4; ++k) VQ[k * m * m] = V[k];
      }
      lds_barrier();
      for (int it = tid; it < EB * 4 * n; it += NT_) {
        const int le = it / (4 * n), r0 = it - le * (4 * n), k = r0 / n, b = r0 - k * n, e = e0 + le;
        if (e >= E) continue;
        R pb[m];
#pragma unroll
        for (int b2 = 0; b2 < m; ++b2) pb[b2] = sPj[b][b2];
        const R* VQ = SS(le) + C::SZ_S0 + k * m * m;
        R z[m];
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) {
          R s = R(0);
#pragma unroll
          for (int b2 = 0; b2 < m; ++b2) s += pb[b2] * VQ[a2 * m + b2];
          z[a2] = s;
        }
        const size_t po = (size_t)(sg.po_base + e * F::PPE + F::foff(2 + ed));
#pragma unroll
        for (int i = 0; i < n; ++i) {
          R s = R(0);
#pragma unroll
          for (int a2 = 0; a2 < m; ++a2) s += op.Pj[i][a2] * z[a2];
          Vf[po * 4 + k * NFP + i + n * b] = s;
        }
      }
    }
    lds_barrier();  // region B is reused below
  } else {
  // phase 4a: normal viscous flux at own flux points (gradcoru_fpts).  With
  // PL the 20 fields are first interpolated to the quadrilateral-face points
  // one (field, plane) per thread into LDS (the jump region, free since the
  // gradient phase)
  if constexpr (PL) {
    for (int it = tid; it < EB * 20 * n; it += NT_) {
      const int le = it / (20 * n), fk = it - le * (20 * n), fld = fk / n, k = fk - fld * n;
      const R* x = XS(le) + fld * NU + NTN * k;
      R xv[NTN];
#pragma unroll
      for (int t = 0; t < NTN; ++t) xv[t] = x[t];
      R* EF = JS(le) + fld * C::EFS;
#pragma unroll
      for (int ed = 0; ed < 3; ++ed)
#pragma unroll
        for (int i = 0; i < n; ++i) {
          R s = R(0);
#pragma unroll
          for (int t = 0; t < NTN; ++t) s += tri.Tedge[ed][i][t] * xv[t];
          EF[ed * NFP + i + n * k] = s;
        }
    }
    lds_barrier();
  }
  constexpr int NV_TRI = NTN, NV_QUAD = 3 * n * n;
  for (int it = tid; it < EB * (NV_TRI + NV_QUAD); it += NT_) {
    const int le = it / (NV_TRI + NV_QUAD), r0 = it - le * (NV_TRI + NV_QUAD), e = e0 + le;
    if (e >= E) continue;
    const R* X = XS(le);
    if (r0 < NV_TRI) {
      const int t = r0;
      R fm[20], fp[20];
#pragma unroll
      for (int fld = 0; fld < 20; ++fld) {
        R sm = R(0), sp = R(0);
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const R x = X[fld * NU + t + NTN * k];
          sm += op.lb[k] * x;
          sp += op.rb[k] * x;
        }
        fm[fld] = sm;
        fp[fld] = sp;
      }
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const R* w = side ? fp : fm;
        const int lf = le * 5 + side, po = sg.po_base + e * F::PPE + side * NTN;
        R nn[3];
        if constexpr (WARP) {
          // own outward unit normal: +-S_zeta / |S_zeta| at the triangle node
          R S[3][3], det;
          wedge_metric(&sV[le][0], tri.nodes[t][0], tri.nodes[t][1], side ? R(1) : R(-1), S, det);
          const R im = rcp(sqrt(S[2][0] * S[2][0] + S[2][1] * S[2][1] + S[2][2] * S[2][2]));
#pragma unroll
          for (int c = 0; c < 3; ++c) nn[c] = (side ? im : -im) * S[2][c];
        } else {
          const R sgn = (sFR[lf].info & 1) ? R(1) : R(-1);
#pragma unroll
          for (int c = 0; c < 3; ++c) nn[c] = sgn * sFG[lf][c];
        }
        R u[5], q[3][5], V[4];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          u[v] = w[v];
#pragma unroll
          for (int d = 0; d < 3; ++d) q[d][v] = w[5 + d * 5 + v];
        }
        normal_viscous(u, q, nn, g, V);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) Vf[(size_t)po * 4 + kk * NTN + t] = V[kk];
      }
    } else {
      const int r1 = r0 - NV_TRI, ed = r1 / (n * n), r2 = r1 - ed * (n * n), k = r2 / n, i = r2 - k * n;
      const int lf = le * 5 + 2 + ed, po = sg.po_base + e * F::PPE + F::foff(2 + ed);
      R nn[3];
      if constexpr (WARP) {
        // own outward unit normal: (nx S_xi + ny S_eta) normalised at the edge point
        R xi, eta, nx, ny, S[3][3], det;
        edge_point(ed, psel(op.x, i), xi, eta);
        edge_normal<R>(ed, nx, ny);
        wedge_metric(&sV[le][0], xi, eta, psel(op.x, k), S, det);
        R vv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[c] = nx * S[0][c] + ny * S[1][c];
        const R im = rcp(sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]));
#pragma unroll
        for (int c = 0; c < 3; ++c) nn[c] = im * vv[c];
      } else {
        const R sgn = (sFR[lf].info & 1) ? R(1) : R(-1);
#pragma unroll
        for (int c = 0; c < 3; ++c) nn[c] = sgn * sFG[lf][c];
      }
      R u[5], q[3][5], V[4];
#pragma unroll
      for (int fld = 0; fld < 20; ++fld) {
        R s = R(0);
        if constexpr (PL) {
          s = JS(le)[fld * C::EFS + ed * NFP + i + n * k];
        } else {
#pragma unroll
          for (int t = 0; t < NTN; ++t) s += tri.Tedge[ed][i][t] * X[fld * NU + t + NTN * k];
        }
        if (fld < 5)
          u[fld] = s;
        else
          q[(fld - 5) / 5][(fld - 5) % 5] = s;
      }
      normal_viscous(u, q, nn, g, V);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) Vf[(size_t)po * 4 + kk * NFP + i + n * k] = V[kk];
    }
  }
  }
  if constexpr (!AA) {
    lds_barrier();  // the face viscous fluxes have read the gradients
    // tdisf at the solution points, in place over the gradients
    for (int it = tid; it < EB * NU; it += NT_) {
      const int le = it / NU, s = it - le * NU;
      R* X = XS(le);
      R u[5], q[3][5], f[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        u[v] = X[v * NU + s];
#pragma unroll
        for (int d = 0; d < 3; ++d) q[d][v] = X[(5 + d * 5 + v) * NU + s];
      }
      point_flux(u, q, g, f);
      const R dj = sMet[le][9];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = V0; v < 5; ++v)
          X[(5 + d * 5 + v) * NU + s] =
              dj * (sMet[le][3 * d] * f[0][v] + sMet[le][3 * d + 1] * f[1][v] + sMet[le][3 * d + 2] * f[2][v]);
    }
    lds_barrier();
    // M2 F~: reference normal flux at the own flux points (JS region, free
    // since the gradient phase): triangle faces from the zeta lines,
    // quadrilateral faces from the triangle planes (per plane where PL)
    constexpr int NQF = PL ? NVF * n : NVF * 3 * n * n;
    for (int it = tid; it < EB * (NVF * NTN + NQF); it += NT_) {
      const int le = it / (NVF * NTN + NQF), r0 = it - le * (NVF * NTN + NQF);
      const R* F = XS(le) + 5 * NU;  // component d of variable v at F[(d * 5 + v) * NU]
      R* NF = JS(le);
      if (r0 < NVF * NTN) {
        const int v = V0 + r0 / NTN, t = r0 - (v - V0) * NTN;
        R fm = R(0), fp = R(0);
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const R x = F[(2 * 5 + v) * NU + t + NTN * k];
          fm += op.lb[k] * x;
          fp += op.rb[k] * x;
        }
        NF[(0 * 5 + v) * NFP + t] = -fm;  // zeta = -1: outward normal -e_zeta
        NF[(1 * 5 + v) * NFP + t] = fp;
      } else if constexpr (PL) {
        const int r1 = r0 - NVF * NTN, v = V0 + r1 / n, k = r1 - (v - V0) * n;
        R fx[NTN], fy[NTN];
#pragma unroll
        for (int t = 0; t < NTN; ++t) {
          fx[t] = F[(0 * 5 + v) * NU + t + NTN * k];
          fy[t] = F[(1 * 5 + v) * NU + t + NTN * k];
        }
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) {
          R nx, ny;
          edge_normal<R>(ed, nx, ny);
#pragma unroll
          for (int i = 0; i < n; ++i) {
            R sx = R(0), sy = R(0);
#pragma unroll
            for (int t = 0; t < NTN; ++t) {
              sx += tri.Tedge[ed][i][t] * fx[t];
              sy += tri.Tedge[ed][i][t] * fy[t];
            }
            NF[((2 + ed) * 5 + v) * NFP + i + n * k] = nx * sx + ny * sy;
          }
        }
      } else {
        const int r1 = r0 - NVF * NTN, v = V0 + r1 / (3 * n * n), r2 = r1 - (v - V0) * (3 * n * n);
        const int ed = r2 / (n * n), r3 = r2 - ed * (n * n), k = r3 / n, i = r3 - k * n;
        R sx = R(0), sy = R(0);
#pragma unroll
        for (int t = 0; t < NTN; ++t) {
          sx += tri.Tedge[ed][i][t] * F[(0 * 5 + v) * NU + t + NTN * k];
          sy += tri.Tedge[ed][i][t] * F[(1 * 5 + v) * NU + t + NTN * k];
        }
        R nx, ny;
        edge_normal<R>(ed, nx, ny);
        NF[((2 + ed) * 5 + v) * NFP + i + n * k] = nx * sx + ny * sy;
      }
    }
    lds_barrier();
    // (M1 - M3 M2) F~: the zeta derivative and triangle-face lifting per
    // line, accumulated over the state slots (dead since the flux phase) ...
    for (int it = tid; it < EB * NVF * NTN; it += NT_) {
      const int le = it / (NVF * NTN), r0 = it - le * (NVF * NTN), v = V0 + r0 / NTN, t = r0 - (v - V0) * NTN;
      const R* F = XS(le) + 5 * NU;
      const R* NF = JS(le);
      R z[n];
#pragma unroll
      for (int c = 0; c < n; ++c) z[c] = F[(2 * 5 + v) * NU + t + NTN * c];
      const R nm = NF[(0 * 5 + v) * NFP + t], np = NF[(1 * 5 + v) * NFP + t];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        R acc = -(op.liftL[k] * nm + op.liftR[k] * np);
#pragma unroll
        for (int c = 0; c < n; ++c) acc += op.D[k][c] * z[c];
        XS(le)[v * NU + t + NTN * k] = acc;
      }
    }
    lds_barrier();
    // ... then the (xi, eta) derivative blocks and quadrilateral-face lifting
    constexpr int NDV = PL ? NVF * n : NVF * NU;
    for (int it = tid; it < EB * NDV; it += NT_) {
      const int le = it / NDV, r0 = it - le * NDV, e = e0 + le;
      if (e >= E) continue;
      const R* F = XS(le) + 5 * NU;
      const R* NF = JS(le);
      if constexpr (PL) {
        const int v = V0 + r0 / n, k = r0 - (v - V0) * n;
        R fx[NTN], fy[NTN], nq[3][n];
#pragma unroll
        for (int c = 0; c < NTN; ++c) {
          fx[c] = F[(0 * 5 + v) * NU + c + NTN * k];
          fy[c] = F[(1 * 5 + v) * NU + c + NTN * k];
        }
#pragma unroll
        for (int ed = 0; ed < 3; ++ed)
#pragma unroll
          for (int i = 0; i < n; ++i) nq[ed][i] = NF[((2 + ed) * 5 + v) * NFP + i + n * k];
#pragma unroll
        for (int t = 0; t < NTN; ++t) {
          R acc = XS(le)[v * NU + t + NTN * k];
          if (LIN && v == 4) acc += g.kap * Rp[(size_t)e * 5 * NU + t + NTN * k];  // kap L(rho v)
#pragma unroll
          for (int c = 0; c < NTN; ++c) acc += tri.Dxi[t][c] * fx[c] + tri.Deta[t][c] * fy[c];
#pragma unroll
          for (int ed = 0; ed < 3; ++ed)
#pragma unroll
            for (int i = 0; i < n; ++i) acc -= tri.LiftEdge[ed][t][i] * nq[ed][i];
          Rp[(size_t)e * 5 * NU + v * NU + t + NTN * k] = acc;
        }
      } else {
        const int v = V0 + r0 / NU, s = r0 - (v - V0) * NU, k = s / NTN, t = s - k * NTN;
        R acc = XS(le)[v * NU + s];
        if (LIN && v == 4) acc += g.kap * Rp[(size_t)e * 5 * NU + s];  // kap L(rho v)
#pragma unroll
        for (int c = 0; c < NTN; ++c)
          acc += tri.Dxi[t][c] * F[(0 * 5 + v) * NU + c + NTN * k] + tri.Deta[t][c] * F[(1 * 5 + v) * NU + c + NTN * k];
#pragma unroll
        for (int ed = 0; ed < 3; ++ed)
#pragma unroll
          for (int i = 0; i < n; ++i) acc -= tri.LiftEdge[ed][t][i] * NF[((2 + ed) * 5 + v) * NFP + i + n * k];
        Rp[(size_t)e * 5 * NU + v * NU + s] = acc;
      }
    }
    return;
  }
  if constexpr (PL && !SAA) lds_barrier();  // every edge point has read its fields
  // phase 4b: triangle-plane interpolation of the 20 fields to the triangle
  // quadrature points (first factor of M7 / M10): one (field, plane) per
  // thread, its N_t values in registers, operator entries read from the LDS
  // copy at wave-uniform addresses (broadcast reads)
  // (at high order SPL threads share a plane, taking alternate outputs, so
  // that more lanes are busy)
  constexpr int SPL = P >= 4 ? 2 : 1;
  auto plane_sweep = [&](const int it, const R* xv) {
    const int le = it / (20 * n * SPL), r0 = it - le * (20 * n * SPL), fk = r0 / SPL, h = r0 - fk * SPL;
    R* T = TS(le) + fk * C::TQS;  // [fld][k][tq]
#pragma unroll
    for (int j = 0; j < (NTQ + SPL - 1) / SPL; ++j) {
      const int tq = SPL * j + h;
      if (tq < NTQ) {
        R s = R(0);
#pragma unroll
        for (int t = 0; t < NTN; ++t) s += tri.Tq[tq][t] * xv[t];
        T[tq] = s;
      }
    }
  };
  auto plane_rows = [&](const int it, R* xv) {
    const int le = it / (20 * n * SPL), r0 = it - le * (20 * n * SPL), fk = r0 / SPL;
    const int fld = fk / n, k = fk - fld * n;
    const R* x = XS(le) + fld * NU + NTN * k;
#pragma unroll
    for (int t = 0; t < NTN; ++t) xv[t] = x[t];
  };
  if constexpr (TOX) {
    // T1 overwrites the state and gradients: every thread reads its plane
    // values into registers before a barrier and writes T1 after it
    constexpr int NIT = (EB * 20 * n * SPL + NT_ - 1) / NT_;
    R xv[NIT][NTN];
#pragma unroll
    for (int k = 0; k < NIT; ++k)
      if (tid + k * NT_ < EB * 20 * n * SPL) plane_rows(tid + k * NT_, xv[k]);
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NIT; ++k)
      if (tid + k * NT_ < EB * 20 * n * SPL) plane_sweep(tid + k * NT_, xv[k]);
  } else {
    for (int it = tid; it < EB * 20 * n * SPL; it += NT_) {
      const int le = it / (20 * n * SPL), r0 = it - le * (20 * n * SPL), fk = r0 / SPL, h = r0 - fk * SPL;
      const int fld = fk / n, k = fk - fld * n;
      const R* x = XS(le) + fld * NU + NTN * k;
      R xv[NTN];
#pragma unroll
      for (int t = 0; t < NTN; ++t) xv[t] = x[t];
      R* T = TS(le) + fk * C::TQS;  // [fld][k][tq]
#pragma unroll
      for (int j = 0; j < (NTQ + SPL - 1) / SPL; ++j) {
        const int tq = SPL * j + h;
        if (tq < NTQ) {
          R s = R(0);
#pragma unroll
          for (int t = 0; t < NTN; ++t) s += tri.Tq[tq][t] * xv[t];
          T[tq] = s;
        }
      }
    }
  }
  lds_barrier();

  // phase 5: line columns over the triangle quadrature points, two threads
  // per column (alternate zeta levels): zeta interpolation, flux (tdisf) and
  // the line part of the projection-divergence; the pair sum completes it
  const bool col = tid < 2 * EB * NTQ;
  const int cc = tid >> 1, half = tid & 1, cle = cc / NTQ, ctq = cc - cle * NTQ;
  R acc[3][NVF][n];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int v = 0; v < NVF; ++v)
#pragma unroll
      for (int k = 0; k < n; ++k) acc[d][v][k] = R(0);
  if (col) {
    const R* T = TS(cle);
    R t1[20][n];
#pragma unroll
    for (int fld = 0; fld < 20; ++fld)
#pragma unroll
      for (int k = 0; k < n; ++k) t1[fld][k] = T[(fld * n + k) * C::TQS + ctq];
    R S[3][3];
    const R dj = sMet[cle][9];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int c = 0; c < 3; ++c) S[d][c] = dj * sMet[cle][3 * d + c];
    R cqx = R(0), cqy = R(0);
    if constexpr (WARP) {
      cqx = tri.qp[ctq][0];
      cqy = tri.qp[ctq][1];
    }
    // thread `half` takes zeta level kq = 2j + half; the operator entries are
    // selected per lane (no divergent branch); for odd m the surplus level of
    // the odd thread repeats level 2j with zero projection weights
#pragma unroll
    for (int j = 0; j < (m + 1) / 2; ++j) {
      const int k0 = 2 * j, k1 = 2 * j + 1 < m ? 2 * j + 1 : 2 * j;
      const bool has1 = 2 * j + 1 < m;
      R wI[n], wP[n], wA[n];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        wI[k] = half ? op.I[k1][k] : op.I[k0][k];
        wP[k] = half ? (has1 ? op.Pj[k][k1] : R(0)) : op.Pj[k][k0];
        wA[k] = half ? (has1 ? op.AP[k][k1] : R(0)) : op.AP[k][k0];
      }
      R u[5], q[3][5], f[3][5];
#pragma unroll
      for (int fld = 0; fld < 20; ++fld) {
        R s = R(0);
#pragma unroll
        for (int k = 0; k < n; ++k) s += wI[k] * t1[fld][k];
        if (fld < 5)
          u[fld] = s;
        else
          q[(fld - 5) / 5][(fld - 5) % 5] = s;
      }
      point_flux(u, q, g, f);
      if constexpr (WARP) {
        R det;
        wedge_metric(&sV[cle][0], cqx, cqy, half ? op.xq[k1] : op.xq[k0], S, det);  // det J J^-1 here
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = V0; v < 5; ++v) {
          const R ft = S[d][0] * f[0][v] + S[d][1] * f[1][v] + S[d][2] * f[2][v];
#pragma unroll
          for (int k = 0; k < n; ++k) acc[d][v - V0][k] += (d == 2 ? wA[k] : wP[k]) * ft;
        }
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int v = 0; v < NVF; ++v)
#pragma unroll
      for (int k = 0; k < n; ++k) acc[d][v][k] = pair_sum(acc[d][v][k]);
  lds_barrier();  // every column has read T1; Z may now overwrite it
  if (col) {
    R* Z = ZS(cle);
    // both threads of a pair hold the same sums; each writes half the values
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < NVF; ++v)
#pragma unroll
        for (int k = 0; k < n; ++k)
          if (((d * NVF + v) * n + k) % 2 == half) Z[(d * NVF + v) * C::ZVS + ctq * n + k] = acc[d][v][k];
  }
  lds_barrier();

  // phase 6: triangle-plane projection-divergence: one (variable, plane) per
  // thread, its 3 N_tq line-projected flux values in registers, operator
  // entries read from the LDS copy at wave-uniform addresses; LIN: the
  // energy residual takes kap L(rho v) (row 0, from the disu kernel)
  for (int it = tid; it < EB * NVF * n * SPL; it += NT_) {
    const int le = it / (NVF * n * SPL), r0 = it - le * (NVF * n * SPL), vk = r0 / SPL, h = r0 - vk * SPL;
    const int vv = vk / n, k = vk - vv * n, e = e0 + le, v = vv + V0;
    if (e >= E) continue;
    const R* Z = ZS(le);
    R z0[NTQ], z1[NTQ], z2[NTQ];
#pragma unroll
    for (int tq = 0; tq < NTQ; ++tq) {
      z0[tq] = Z[(0 * NVF + vv) * C::ZVS + tq * n + k];
      z1[tq] = Z[(1 * NVF + vv) * C::ZVS + tq * n + k];
      z2[tq] = Z[(2 * NVF + vv) * C::ZVS + tq * n + k];
    }
#pragma unroll
    for (int j = 0; j < (NTN + SPL - 1) / SPL; ++j) {
      const int t = SPL * j + h;
      if (t < NTN) {
        R s = (LIN && v == 4) ? g.kap * Rp[(size_t)e * 5 * NU + t + NTN * k] : R(0);
#pragma unroll
        for (int tq = 0; tq < NTQ; ++tq) {
          s += tri.APxi[t][tq] * z0[tq];
          s += tri.APeta[t][tq] * z1[tq];
          s += tri.PT[t][tq] * z2[tq];
        }
        Rp[(size_t)e * 5 * NU + v * NU + t + NTN * k] = s;
      }
    }
  }
#undef XS
#undef JS
#undef TS
#undef ZS
#undef SS
}

// -------------------------------------------------------------- surface
// With surface-flux anti-aliasing (SAA) the common flux is lifted through
// its projection onto the flux points (P_T on the triangles, P x P on the
// quadrilaterals): the part linear in the two sides' values at the flux
// points, the Rusanov flux at the face quadrature points from the
// interpolated pair of states (T_q on the triangles, I x I on the
// quadrilaterals).  The triangle rule is not symmetric, so both sides of a
// triangle face must see the same nodes: the library requires the identity
// point permutation there.
template <int P, typename R, int EB, int NT_, bool BT, bool SAA, bool WARP>
__global__ void __launch_bounds__(NT_)
    prism_surface(const Seg one, const BlkRef* __restrict__ bt, const Seg* __restrict__ segs, const int rk,
                  const PrismOps<P, R> op, const PrismTri<P, R>* __restrict__ tri, const Gas<R> g) {
  using C = PrismCfg<P>;
  constexpr int n = C::n, m = C::m, NT = C::NT, NTQ = C::NTQ, NU = C::NU, NFP = C::NFP;
  constexpr bool LIN = !WARP, FB = sizeof(R) == 4;
  // SAA staging per face: the L state and uL - uR [10][NFP], later the Rusanov
  // flux at a quadrilateral's quadrature points [5][m][m] (sW); a
  // quadrilateral's states along its first axis at GL(m) [10][m][n] (sT);
  // the Rusanov flux at a triangle's quadrature points [5][NTQ] (sFt)
  constexpr int SW = 10 * NFP > 5 * m * m ? 10 * NFP : 5 * m * m, ST = 10 * m * n, SF = 5 * NTQ;
  __shared__ R sD[EB * 25 * NFP];
  __shared__ R sLift[3][NT][n];
  __shared__ R sW[SAA ? EB * 5 * SW : 1];
  __shared__ R sT[SAA ? EB * 3 * ST : 1];
  __shared__ R sFt[SAA ? EB * 2 * SF : 1];
  __shared__ R sTq[SAA ? NTQ : 1][NT];
  __shared__ R sPT[SAA ? NT : 1][NTQ];
  __shared__ R sI[SAA ? m : 1][n];
  __shared__ R sPj[SAA ? n : 1][m];
  __shared__ R sFG[SAA ? EB * 5 : 1][4];
  __shared__ int sInfo[SAA ? EB * 5 : 1];
  __shared__ R sV[WARP ? EB : 1][18];              // curved: element vertices
  __shared__ R sDetU[WARP ? EB : 1][WARP ? NU : 1];  // curved: det J at the solution points
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const R* __restrict__ Uf = (const R*)sg.Uf;
  const R* __restrict__ Vf = (const R*)sg.Vf;
  const R* __restrict__ Rp = (const R*)sg.Rp;
  const FaceRec* __restrict__ faces = sg.faces;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
  const uint8_t* __restrict__ perms = sg.perms;
  const double* __restrict__ detj = sg.detj;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
  // edge lifting table, staged in LDS for the per-point lift below
  for (int it = tid; it < 3 * NT * n; it += NT_) (&sLift[0][0][0])[it] = (&tri->LiftEdge[0][0][0])[it];
  if constexpr (WARP) {
    const R* __restrict__ vx = (const R*)sg.verts;
    for (int it = tid; it < EB * 18; it += NT_) {
      const int le = it / 18;
      sV[le][it - le * 18] = vx[e0 + le < E ? (size_t)e0 * 18 + it : 0];
    }
    __syncthreads();
  }
  if constexpr (SAA) {
    for (int it = tid; it < NTQ * NT; it += NT_) {
      (&sTq[0][0])[it] = (&tri->Tq[0][0])[it];
      (&sPT[0][0])[it] = (&tri->PT[0][0])[it];
    }
    if (tid < m * n) {
      sI[tid / n][tid % n] = op.I[tid / n][tid % n];
      sPj[tid / m][tid % m] = op.Pj[tid / m][tid % m];
    }
  }
  // comm_flux: common normal flux at every own flux point, times +-mag
  // (with SAA: its linear part, and the pair of states to LDS)
  // one own flux point per item, the element's points in face-array order
  // (two triangles, three quadrilaterals)
  for (int it = tid; it < EB * C::PPE; it += NT_) {
    const int le = it / C::PPE, q = it - le * C::PPE, e = e0 + le;
    if (e >= E) continue;
    const int f = q < 2 * NT ? q / NT : 2 + (q - 2 * NT) / NFP, r = q - C::foff(f);
    const int slot = slot_base + e * 5 + f;
    const FaceRec fr = faces[slot];
    const int rr = perms[(fr.info >> 1) * NFP + r];
    const bool left = fr.info & 1;
    // this face's points in the face arrays: own and paired
    const int fs = C::fsz(f);
    const size_t po = (size_t)(sg.po_base + e * C::PPE + q - r);
    R uo[5], un[5], jn[5], Vo[4], Vn[4], F[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      uo[v] = Uf[po * 5 + v * fs + r];
      un[v] = Uf[(size_t)fr.npo * 5 + v * fs + rr];
    }
    // u_nbr - u_own from the face bases and deviations (single precision),
    // before the states themselves are formed
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if constexpr (FB) {
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
      Vo[k] = Vf[po * 4 + k * fs + r];
      Vn[k] = Vf[(size_t)fr.npo * 4 + k * fs + rr];
    }
    R nL[3] = {fgeo[4 * slot], fgeo[4 * slot + 1], fgeo[4 * slot + 2]};
    R mag = fgeo[4 * slot + 3];
    if constexpr (WARP) {
      // own area factor and outward normal at this flux point; the L side's
      // normal is the opposite of the R side's own
      R S[3][3], det, vv[3];
      if (f < 2) {
        wedge_metric(&sV[le][0], tri->nodes[r][0], tri->nodes[r][1], f ? R(1) : R(-1), S, det);
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[c] = f ? S[2][c] : -S[2][c];
      } else {
        R xi, eta, nx, ny;
        edge_point(f - 2, psel(op.x, r % n), xi, eta);
        edge_normal<R>(f - 2, nx, ny);
        wedge_metric(&sV[le][0], xi, eta, psel(op.x, r / n), S, det);
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[c] = nx * S[0][c] + ny * S[1][c];
      }
      mag = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
      const R im = left ? rcp(mag) : -rcp(mag);
#pragma unroll
      for (int c = 0; c < 3; ++c) nL[c] = im * vv[c];
    }
    if constexpr (SAA) {
      face_flux_linear<R, LIN>(jn, Vo, Vn, nL, left, g, F);
      R* W = sW + (le * 5 + f) * SW + r;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        W[v * NFP] = left ? uo[v] : un[v];
        W[(5 + v) * NFP] = left ? -jn[v] : jn[v];
      }
      if (r == 0) {
        sInfo[le * 5 + f] = fr.info;
#pragma unroll
        for (int k = 0; k < 3; ++k) sFG[le * 5 + f][k] = nL[k];
        sFG[le * 5 + f][3] = mag;
      }
    } else {
      face_flux<R, LIN>(uo, un, jn, Vo, Vn, nL, left, g, F);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sD[(le * 5 + f) * 5 * NFP + v * NFP + r] = mag * F[v];
  }
  if constexpr (SAA) {
    __syncthreads();
    // triangles: Rusanov at the quadrature points (T_q of the pair);
    // quadrilaterals: the pair along the first axis to GL(m)
    constexpr int NA = 2 * NTQ + 3 * 10 * n;
    for (int it = tid; it < EB * NA; it += NT_) {
      const int le = it / NA, r0 = it - le * NA;
      if (e0 + le >= E) continue;
      if (r0 < 2 * NTQ) {
        const int f = r0 / NTQ, q = r0 - f * NTQ, lf = le * 5 + f;
        const R* W = sW + lf * SW;
        R uL[5], jl[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          R sl = R(0), sj = R(0);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            sl += sTq[q][t] * W[v * NFP + t];
            sj += sTq[q][t] * W[(5 + v) * NFP + t];
          }
          uL[v] = sl;
          jl[v] = sj;
        }
        const R nL[3] = {sFG[lf][0], sFG[lf][1], sFG[lf][2]};
        R F[5];
        rusanov_jump<R, true>(uL, jl, nL, g, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sFt[(le * 2 + f) * SF + v * NTQ + q] = F[v];
      } else {
        const int r1 = r0 - 2 * NTQ, ed = r1 / (10 * n), r2 = r1 - ed * (10 * n), fld = r2 / n, k = r2 - fld * n;
        const R* W = sW + (le * 5 + 2 + ed) * SW + fld * NFP + n * k;
        R y[n];
#pragma unroll
        for (int i = 0; i < n; ++i) y[i] = W[i];
        R* T = sT + (le * 3 + ed) * ST + fld * m * n + k;
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) {
          R s = R(0);
#pragma unroll
          for (int i = 0; i < n; ++i) s += op.I[a2][i] * y[i];
          T[a2 * n] = s;
        }
      }
    }
    __syncthreads();
    // triangles: P_T of the Rusanov flux, added; quadrilaterals: the pair
    // along zeta to GL(m) and Rusanov at each quadrature point (over the
    // quadrilateral states, read in the previous pass)
    constexpr int NB = 2 * 5 * NT + 3 * m * m;
    for (int it = tid; it < EB * NB; it += NT_) {
      const int le = it / NB, r0 = it - le * NB;
      if (e0 + le >= E) continue;
      if (r0 < 10 * NT) {
        const int f = r0 / (5 * NT), r1 = r0 - f * (5 * NT), v = r1 / NT, t = r1 - v * NT, lf = le * 5 + f;
        const R* Ft = sFt + (le * 2 + f) * SF + v * NTQ;
        R s = R(0);
#pragma unroll
        for (int q = 0; q < NTQ; ++q) s += sPT[t][q] * Ft[q];
        const R sc = (sInfo[lf] & 1) ? sFG[lf][3] : -sFG[lf][3];
        sD[lf * 5 * NFP + v * NFP + t] += sc * s;
      } else {
        const int r1 = r0 - 10 * NT, ed = r1 / (m * m), r2 = r1 - ed * (m * m), a2 = r2 / m, b2 = r2 - a2 * m;
        const int lf = le * 5 + 2 + ed;
        R Ib[n];
#pragma unroll
        for (int j = 0; j < n; ++j) Ib[j] = sI[b2][j];
        const R* T = sT + (le * 3 + ed) * ST + a2 * n;
        R uL[5], jl[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          R sl = R(0), sj = R(0);
#pragma unroll
          for (int k = 0; k < n; ++k) {
            sl += Ib[k] * T[v * m * n + k];
            sj += Ib[k] * T[(5 + v) * m * n + k];
          }
          uL[v] = sl;
          jl[v] = sj;
        }
        const R nL[3] = {sFG[lf][0], sFG[lf][1], sFG[lf][2]};
        R F[5];
        rusanov_jump<R, true>(uL, jl, nL, g, F);
        R* FQ = sW + lf * SW + a2 * m + b2;
#pragma unroll
        for (int v = 0; v < 5; ++v) FQ[v * m * m] = F[v];
      }
    }
    __syncthreads();
    // quadrilaterals: P x P of the Rusanov flux, added
    for (int it = tid; it < EB * 3 * 5 * n; it += NT_) {
      const int le = it / (15 * n), r0 = it - le * (15 * n), ed = r0 / (5 * n), r1 = r0 - ed * (5 * n);
      const int v = r1 / n, b = r1 - v * n, lf = le * 5 + 2 + ed;
      if (e0 + le >= E) continue;
      R pb[m];
#pragma unroll
      for (int b2 = 0; b2 < m; ++b2) pb[b2] = sPj[b][b2];
      const R* FQ = sW + lf * SW + v * m * m;
      R z[m];
#pragma unroll
      for (int a2 = 0; a2 < m; ++a2) {
        R s = R(0);
#pragma unroll
        for (int b2 = 0; b2 < m; ++b2) s += pb[b2] * FQ[a2 * m + b2];
        z[a2] = s;
      }
      const R sc = (sInfo[lf] & 1) ? sFG[lf][3] : -sFG[lf][3];
      R* D = sD + lf * 5 * NFP + v * NFP + n * b;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        R s = R(0);
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) s += op.Pj[i][a2] * z[a2];
        D[i] += sc * s;
      }
    }
  }
  if constexpr (WARP) {
    for (int it = tid; it < EB * NU; it += NT_) {
      const int le = it / NU, s = it - le * NU;
      R S[3][3], det;
      wedge_metric(&sV[le][0], tri->nodes[s % NT][0], tri->nodes[s % NT][1], psel(op.x, s / NT), S, det);
      sDetU[le][s] = det;
    }
  }
  __syncthreads();
  // tdivtconf + negdivconf, one output point per thread (coalesced state
  // and residual access)
  for (int it = tid; it < EB * 5 * NU; it += NT_) {
    const int le = it / (5 * NU), r0 = it - le * (5 * NU), v = r0 / NU, s = r0 - v * NU, e = e0 + le;
    if (e >= E) continue;
    const int k = s / NT, t = s - k * NT;
    const R* D = sD + le * 25 * NFP + v * NFP;
    R acc = Rp[(size_t)e * 5 * NU + r0] + psel(op.liftL, k) * D[0 * 5 * NFP + t] + psel(op.liftR, k) * D[1 * 5 * NFP + t];
#pragma unroll
    for (int ed = 0; ed < 3; ++ed)
#pragma unroll
      for (int i = 0; i < n; ++i) acc += sLift[ed][t][i] * D[(2 + ed) * 5 * NFP + i + n * k];
    rk_store(sg, rk, (size_t)e * 5 * NU + r0, -double(acc) / (WARP ? double(sDetU[le][s]) : detj[e]));
  }
}

// ------------------------------------------------------------ host side
template <int P, typename R>
static PrismOps<P, R> make_prism_ops(const HostOps& h) {
  PrismOps<P, R> o;
  constexpr int n = P + 1, m = P + 3;
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < n; ++i) o.I[a][i] = R(h.I[a * n + i]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) o.D[i][j] = R(h.D[i * n + j]);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < m; ++a) {
      o.Pj[i][a] = R(h.P[i * m + a]);
      o.AP[i][a] = R(h.AP[i * m + a]);
    }
  for (int i = 0; i < n; ++i) {
    o.lb[i] = R(h.lb[i]);
    o.rb[i] = R(h.rb[i]);
    o.liftL[i] = R(h.liftL[i]);
    o.liftR[i] = R(h.liftR[i]);
    o.x[i] = R(h.x[i]);
  }
  for (int a = 0; a < m; ++a) o.xq[a] = R(h.xq[a]);
  return o;
}

template <int P, typename R>
static void pack_tri(const Tri& T, PrismTri<P, R>* o) {
  constexpr int n = P + 1, NT = (P + 1) * (P + 2) / 2, NTQ = (P + 1) * (P + 1);
  for (int q = 0; q < NTQ; ++q)
    for (int t = 0; t < NT; ++t) o->Tq[q][t] = R(T.Tq[q * NT + t]);
  for (int a = 0; a < NT; ++a)
    for (int b = 0; b < NT; ++b) {
      o->Dxi[a][b] = R(T.Dxi[a * NT + b]);
      o->Deta[a][b] = R(T.Deta[a * NT + b]);
    }
  for (int t = 0; t < NT; ++t)
    for (int q = 0; q < NTQ; ++q) {
      o->PT[t][q] = R(T.PT[t * NTQ + q]);
      o->APxi[t][q] = R(T.APxi[t * NTQ + q]);
      o->APeta[t][q] = R(T.APeta[t * NTQ + q]);
    }
  for (int e = 0; e < 3; ++e) {
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < NT; ++t) o->Tedge[e][i][t] = R(T.Tedge[(e * n + i) * NT + t]);
    for (int t = 0; t < NT; ++t)
      for (int i = 0; i < n; ++i) o->LiftEdge[e][t][i] = R(T.LiftEdge[(e * NT + t) * n + i]);
  }
  for (int t = 0; t < NT; ++t)
    for (int d = 0; d < 2; ++d) o->nodes[t][d] = R(T.nodes[2 * t + d]);
  for (int q = 0; q < NTQ; ++q)
    for (int d = 0; d < 2; ++d) o->qp[q][d] = R(T.qp[2 * q + d]);
}

template <int P>
static void pack_disu(const RefElem& r, PrismDisuTab<P>* o) {
  constexpr int n = P + 1, NT = (P + 1) * (P + 2) / 2;
  const Tri& T = r.tri;
  for (int i = 0; i < n; ++i) {
    o->lb[i] = r.line.lb[i];
    o->rb[i] = r.line.rb[i];
    for (int j = 0; j < n; ++j) o->D[i][j] = r.line.D[i * n + j];
  }
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < NT; ++t) o->Tedge[e][i][t] = T.Tedge[(e * n + i) * NT + t];
  for (int a = 0; a < NT; ++a)
    for (int b = 0; b < NT; ++b) {
      o->Dxi[a][b] = T.Dxi[a * NT + b];
      o->Deta[a][b] = T.Deta[a * NT + b];
    }
}

template <int P, typename R>
static size_t prism_bytes_t() {
  return prism_disu_offset<P, R>() + sizeof(PrismDisuTab<P>);
}

template <int P, typename R>
static void prism_pack_t(const RefElem& r, void* dst) {
  pack_tri<P, R>(r.tri, (PrismTri<P, R>*)dst);
  pack_disu<P>(r, (PrismDisuTab<P>*)((char*)dst + prism_disu_offset<P, R>()));
}

// the device table of one order and precision: the prism operators in the
// working precision, then the double-precision disu operators
size_t prism_ops_bytes(int p, int prec) {
  const bool d = prec == 0;
  switch (p) {
    case 1: return d ? prism_bytes_t<1, double>() : prism_bytes_t<1, float>();
    case 2: return d ? prism_bytes_t<2, double>() : prism_bytes_t<2, float>();
    case 3: return d ? prism_bytes_t<3, double>() : prism_bytes_t<3, float>();
    case 4: return d ? prism_bytes_t<4, double>() : prism_bytes_t<4, float>();
  }
  return 0;
}

void prism_ops_pack(const RefElem& r, int prec, void* dst) {
  const bool d = prec == 0;
  switch (r.p) {
    case 1: d ? prism_pack_t<1, double>(r, dst) : prism_pack_t<1, float>(r, dst); break;
    case 2: d ? prism_pack_t<2, double>(r, dst) : prism_pack_t<2, float>(r, dst); break;
    case 3: d ? prism_pack_t<3, double>(r, dst) : prism_pack_t<3, float>(r, dst); break;
    case 4: d ? prism_pack_t<4, double>(r, dst) : prism_pack_t<4, float>(r, dst); break;
  }
}

// launch shapes of the volume kernel: two threads per quadrature column
template <int P, bool DBL>
struct PrismLaunch;
template <> struct PrismLaunch<1, false> { static constexpr int EB = 8, NT = 64; };   // 64 column threads
template <> struct PrismLaunch<2, false> { static constexpr int EB = 7, NT = 128; };  // 126
template <> struct PrismLaunch<3, false> { static constexpr int EB = 4, NT = 128; };  // 128
template <> struct PrismLaunch<4, false> { static constexpr int EB = 1, NT = 64; };   // 50 (one-wave groups:
                                                                                      // 12 % faster than 2)
template <> struct PrismLaunch<1, true> { static constexpr int EB = 8, NT = 64; };
template <> struct PrismLaunch<2, true> { static constexpr int EB = 3, NT = 64; };    // 54
template <> struct PrismLaunch<3, true> { static constexpr int EB = 2, NT = 64; };    // 64
template <> struct PrismLaunch<4, true> { static constexpr int EB = 1, NT = 64; };    // 50

// elements per workgroup of the disu kernel (256 threads)
constexpr int PRISM_DISU_EB = 8;
// elements per workgroup of the interface kernel (256 threads)
template <int P, bool DBL, bool SAA = false>
struct PrismSurf {
  // surface-flux anti-aliasing stages the face quadrature data in LDS: half
  // the elements per workgroup
  static constexpr int EB = SAA ? 2 : 4;
};

template <int P, typename R, bool BT>
static void prism_launch(const TypeArgs& a, const int grid[3], hipStream_t st) {
  const PrismOps<P, R> op = make_prism_ops<P, R>(*a.ops);
  // affine prisms take the mass flux and the linear energy-flux part from
  // the double-precision L(rho v) of the disu kernel
  const bool lin = !a.warp;
  const Gas<R> g = make_gas<R>(*a.gas, lin);
  const PrismTri<P, R>* tri = (const PrismTri<P, R>*)a.dops;
  const PrismDisuTab<P>* dtab = (const PrismDisuTab<P>*)((const char*)a.dops + prism_disu_offset<P, R>());
  constexpr bool dbl = sizeof(R) == 8;
  constexpr int EB = PrismLaunch<P, dbl>::EB, NT = PrismLaunch<P, dbl>::NT;
  constexpr int EBA = PRISM_DISU_EB, NTA = 256, EBC = PrismSurf<P, dbl>::EB, NTC = 256;
  const double eref = a.gas->pref / (a.gas->gamma - 1.0), rho0 = a.gas->rho_ref;
  if ((a.stage & 1) && grid[K_DISU] > 0)
    hipLaunchKernelGGL((prism_disu<P, R, EBA, NTA, BT>), dim3(grid[K_DISU]), dim3(NTA), 0, st, a.one, a.bt[K_DISU],
                       a.segs, a.from_ust, dtab, eref, rho0, lin);
  // curved prisms (single meshes only; flux anti-aliasing, general metric)
  if constexpr (!BT) {
    if (a.warp) {
      if ((a.stage & 2) && grid[K_VOLUME] > 0)
        hipLaunchKernelGGL((prism_volume<P, R, EB, NT, false, true, false, true>), dim3(grid[K_VOLUME]), dim3(NT), 0,
                           st, a.one, a.bt[K_VOLUME], a.segs, a.from_ust, op, tri, g, eref, rho0);
      if ((a.stage & 4) && grid[K_SURFACE] > 0)
        hipLaunchKernelGGL((prism_surface<P, R, EBC, NTC, false, false, true>), dim3(grid[K_SURFACE]), dim3(NTC), 0,
                           st, a.one, a.bt[K_SURFACE], a.segs, a.rk, op, tri, g);
      return;
    }
  }
  if ((a.stage & 2) && grid[K_VOLUME] > 0) {
    // surface-flux anti-aliasing is built together with flux anti-aliasing
    // only (the paper's "full AA"); the library rejects it without
    if (a.saa)
      hipLaunchKernelGGL((prism_volume<P, R, EB, NT, BT, true, true, false>), dim3(grid[K_VOLUME]), dim3(NT), 0, st, a.one,
                         a.bt[K_VOLUME], a.segs, a.from_ust, op, tri, g, eref, rho0);
    else if (a.aa)
      hipLaunchKernelGGL((prism_volume<P, R, EB, NT, BT, true, false, false>), dim3(grid[K_VOLUME]), dim3(NT), 0, st, a.one,
                         a.bt[K_VOLUME], a.segs, a.from_ust, op, tri, g, eref, rho0);
    else
      hipLaunchKernelGGL((prism_volume<P, R, EB, NT, BT, false, false, false>), dim3(grid[K_VOLUME]), dim3(NT), 0, st,
                         a.one, a.bt[K_VOLUME], a.segs, a.from_ust, op, tri, g, eref, rho0);
  }
  if ((a.stage & 4) && grid[K_SURFACE] > 0) {
    if (a.saa)
      hipLaunchKernelGGL((prism_surface<P, R, PrismSurf<P, dbl, true>::EB, NTC, BT, true, false>), dim3(grid[K_SURFACE]),
                         dim3(NTC), 0, st, a.one, a.bt[K_SURFACE], a.segs, a.rk, op, tri, g);
    else
      hipLaunchKernelGGL((prism_surface<P, R, EBC, NTC, BT, false, false>), dim3(grid[K_SURFACE]), dim3(NTC), 0, st, a.one,
                         a.bt[K_SURFACE], a.segs, a.rk, op, tri, g);
  }
}

template <int P, typename R>
static hipError_t prism_rhs_t(const TypeArgs& a, hipStream_t st) {
  constexpr bool dbl = sizeof(R) == 8;
  const int ebs[3] = {PRISM_DISU_EB, PrismLaunch<P, dbl>::EB,
                      a.saa ? PrismSurf<P, dbl, true>::EB : PrismSurf<P, dbl>::EB};
  const bool bt = a.bt[0] && a.bt[1] && a.bt[2] && a.segs;
  int grid[3];
  for (int k = 0; k < 3; ++k) grid[k] = bt ? a.nblk[k] : (a.one.E + ebs[k] - 1) / ebs[k];
  if (bt)
    prism_launch<P, R, true>(a, grid, st);
  else
    prism_launch<P, R, false>(a, grid, st);
  return hipGetLastError();
}

template <int P>
static int prism_surf_elems(bool d, bool saa) {
  return d ? (saa ? PrismSurf<P, true, true>::EB : PrismSurf<P, true>::EB)
           : (saa ? PrismSurf<P, false, true>::EB : PrismSurf<P, false>::EB);
}

int prism_block_elems(int p, int prec, int k, bool saa) {
  if (k == K_DISU) return PRISM_DISU_EB;
  const bool d = prec == 0;
  if (k == K_SURFACE) {
    switch (p) {
      case 1: return prism_surf_elems<1>(d, saa);
      case 2: return prism_surf_elems<2>(d, saa);
      case 3: return prism_surf_elems<3>(d, saa);
      case 4: return prism_surf_elems<4>(d, saa);
    }
    return 0;
  }
  switch (p) {
    case 1: return d ? PrismLaunch<1, true>::EB : PrismLaunch<1, false>::EB;
    case 2: return d ? PrismLaunch<2, true>::EB : PrismLaunch<2, false>::EB;
    case 3: return d ? PrismLaunch<3, true>::EB : PrismLaunch<3, false>::EB;
    case 4: return d ? PrismLaunch<4, true>::EB : PrismLaunch<4, false>::EB;
  }
  return 0;
}

hipError_t prism_rhs(const TypeArgs& a, int prec, hipStream_t st) {
  const bool d = prec == 0;
  switch (a.p) {
    case 1: return d ? prism_rhs_t<1, double>(a, st) : prism_rhs_t<1, float>(a, st);
    case 2: return d ? prism_rhs_t<2, double>(a, st) : prism_rhs_t<2, float>(a, st);
    case 3: return d ? prism_rhs_t<3, double>(a, st) : prism_rhs_t<3, float>(a, st);
    case 4: return d ? prism_rhs_t<4, double>(a, st) : prism_rhs_t<4, float>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fr
