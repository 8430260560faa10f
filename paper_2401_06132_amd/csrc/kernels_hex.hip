// Fused flux-reconstruction kernels for hexahedra (gfx950).
//
// The paper's kernel groups (section 6.1, figure NSAAKG) become three
// kernels per right-hand side:
//   hex_disu     group 1: disu (eq. FR-disu) -- solution at the flux points
//   hex_volume   groups 2+3: con_u, tgradpcoru, tgradcoru, gradcoru,
//                gradcoru_fpts, uqpts, gradcoru_qpts, tdisf, tdivtpcorf;
//                every intermediate stays in LDS/registers; the outputs are
//                the normal viscous flux at the element's own flux points and
//                the volume part of the transformed divergence
//   hex_surface  groups 4+5: comm_flux, tdivtconf, negdivconf
// The anti-aliasing operators are applied by sum factorisation (section 4):
// M7 = I (x) I (x) I and, combined with the DG divergence (M1 - M3 M2) M9,
// the projection-divergence of component d is AP along d and P along the
// other two directions, where P = W_u^-1 I^T W_q and AP = -W_u^-1 Dq^T W_q
// (summation-by-parts form of the GL collocation operators).
//
// Threads work on "lines": a thread holds the n (or m) values of one 1-D line
// of one field in registers and applies a 1-D operator whose entries are
// wave-uniform (kernel-argument constants).  The column phase keeps one
// (x,y) quadrature column per thread and runs the z direction on the fly:
// interpolate the 20 fields (state + gradient), evaluate the flux, and
// accumulate the z projection, so the quadrature-point data never exists as
// a whole.  A workgroup owns EB elements; element data is contiguous in HBM
// (element-major layout), so every global load/store is coalesced.
#include "fr_device.h"
#include "fr_kernels.h"

namespace fr {

template <int P, typename R>
struct HexOps {
  static constexpr int n = P + 1, m = P + 3;
  R I[m][n];   // l_i at GL(m)
  R D[n][n];   // l_j' at the solution points
  R Pj[n][m];  // projection
  R AP[n][m];  // projection + divergence
  R APu[n][n]; // divergence at the solution points (no anti-aliasing)
  R lb[n], rb[n], liftL[n], liftR[n];
  R x[n], xq[m];  // GL(n) solution and GL(m) quadrature nodes
};

// Curved hexahedra: the trilinear map of the eight vertices X (vertex
// a + 2b + 4c at reference corner (2a-1, 2b-1, 2c-1)).  At reference point
// (xi, eta, zeta): the columns J_c = dx/dxi_c (bilinear interpolations of the
// four edge vectors along c), the cofactor rows S_d = J_{d+1} x J_{d+2}
// (S = det J J^-1, the metric terms of the transformed flux and of the
// normals) and det J = J_0 . S_0.
template <typename R>
__device__ __forceinline__ void trilinear_metric(const R* X, R xi, R eta, R zeta, R S[3][3], R& det) {
  const R xm = R(1) - xi, xp = R(1) + xi, ym = R(1) - eta, yp = R(1) + eta, zm = R(1) - zeta, zp = R(1) + zeta;
  R J[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    J[0][i] = R(0.125) * (ym * zm * (X[3 + i] - X[i]) + yp * zm * (X[9 + i] - X[6 + i]) +
                          ym * zp * (X[15 + i] - X[12 + i]) + yp * zp * (X[21 + i] - X[18 + i]));
    J[1][i] = R(0.125) * (xm * zm * (X[6 + i] - X[i]) + xp * zm * (X[9 + i] - X[3 + i]) +
                          xm * zp * (X[18 + i] - X[12 + i]) + xp * zp * (X[21 + i] - X[15 + i]));
    J[2][i] = R(0.125) * (xm * ym * (X[12 + i] - X[i]) + xp * ym * (X[15 + i] - X[3 + i]) +
                          xm * yp * (X[18 + i] - X[6 + i]) + xp * yp * (X[21 + i] - X[9 + i]));
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

// reference coordinates of the point with index i along axis ax and
// tangential indices (a, b) on the grid g (tangential axes in increasing order)
template <typename R>
__device__ __forceinline__ void grid_point(int ax, R xi_ax, R ta, R tb, R& x, R& y, R& z) {
  x = ax == 0 ? xi_ax : ta;
  y = ax == 1 ? xi_ax : (ax == 0 ? ta : tb);
  z = ax == 2 ? xi_ax : tb;
}

template <int P>
struct HexCfg {
  static constexpr int n = P + 1, m = P + 3, NU = n * n * n, NFP = n * n;
  static constexpr int SZ_X = 20 * NU;  // state (5) + gradients (15)
  static constexpr int SZ_J = 30 * NFP; // jumps C - u^f, 6 faces x 5 vars
  static constexpr int SZ_Z = 15 * m * m * n;
  static constexpr int SZ_A = (SZ_X + SZ_J > SZ_Z) ? SZ_X + SZ_J : SZ_Z;
  static constexpr int SZ_T1 = 20 * m * n * n;
  static constexpr int PER_ELEM = SZ_A + SZ_T1;
};

// index of the point with coordinate index i along axis ax and tangential
// indices (a, b) (tangential axes in increasing order)
template <int n>
__device__ __forceinline__ int hex_pt(int ax, int i, int a, int b) {
  return ax == 0 ? i + n * (a + n * b) : (ax == 1 ? a + n * (i + n * b) : a + n * (b + n * i));
}

// select v[idx] for a lane-varying idx from a compile-time array (no
// dynamic indexing into kernel arguments)
template <int N, typename R>
__device__ __forceinline__ R sel(const R (&v)[N], int idx) {
  R r = v[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = idx == k ? v[k] : r;
  return r;
}

// ----------------------------------------------------------------- disu
// Operators of the disu kernel, always in double precision.
template <int P>
struct HexDisuOps {
  static constexpr int n = P + 1;
  double lb[n], rb[n];  // l_i(-1), l_i(+1)
  double D[n][n];       // l_j' at the solution points
};

// Group 1: the solution at the flux points (eq. FR-disu), interpolated in
// double precision from the state in reference form.  Single precision
// stores each face as a base (its value at the face's first flux point,
// rounded to float) and the deviations from it, so that a face jump
// u_nbr - u_own = (b_nbr - b_own) + (d_nbr - d_own) keeps the digits that
// the O(1) values themselves lose.
// LIN: also the central DG divergence of the mass flux in double precision,
//   L(rho v) = sum_d D_d (S m)_d,  S = det J J^-1,
// the strong form (M1 - M3 M2) (S m) plus the lift of the own trace (exact
// for affine elements: the projected polynomial flux is itself), written
// to row 0 of the volume residual.  DIAG (diagonal metric): (S m)_d is
// S_dd m_d, n terms per point instead of 3n.
// LDS: the state with its x lines padded to an odd length (n even), so that
// the lanes of a wave walking x lines hit different banks.
template <int P, typename R, int EB, int NT, bool BT, bool DIAG>
__global__ void __launch_bounds__(NT) hex_disu(const Seg one, const BlkRef* __restrict__ bt,
                                               const Seg* __restrict__ segs, const bool from_ust,
                                               const HexDisuOps<P> op, const double eref, const double rho0,
                                               const bool lin) {
  using C = HexCfg<P>;
  constexpr int n = C::n, NU = C::NU, NFP = C::NFP;
  constexpr int LX = n + 1 - (n & 1), NUP = LX * n * n;  // padded x line, padded field
  constexpr bool FB = sizeof(R) == 4;
  __shared__ double sU[EB * 5 * NUP];
  __shared__ double sS[EB][9];
  __shared__ double sB[FB ? EB : 1][6][5];  // single precision: the face bases, rounded
  __shared__ double sD[n][n];  // D, read with a per-thread row index
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  R* __restrict__ Uf = (R*)sg.Uf;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
  constexpr int NS = (EB * 5 * NU + NT - 1) / NT;
  // point (i, a, b) of field v of element le in LDS
  auto at = [](int le, int v, int i, int a, int b) { return (le * 5 + v) * NUP + i + LX * (a + n * b); };
  double xs[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int it = tid + k * NT;
    const bool ok = it < EB * 5 * NU && e0 + it / (5 * NU) < E;
    xs[k] = U[ok ? (size_t)e0 * 5 * NU + it : 0];
  }
  if (tid < n * n) sD[tid / n][tid % n] = op.D[tid / n][tid % n];
  if (lin && tid < EB * 9) {
    // S = det J J^-1 from the element metrics [J^-1 (row-major), det J]
    const int le = tid / 9, k = tid - le * 9;
    const R* __restrict__ met = (const R*)sg.met;
    const size_t e = e0 + le < E ? (size_t)(e0 + le) : 0;
    sS[le][k] = double(met[e * 10 + 9]) * double(met[e * 10 + k]);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int it = tid + k * NT;
    if (it < EB * 5 * NU) {
      const int le = it / (5 * NU), r = it - le * (5 * NU), v = r / NU, pt = r - v * NU;
      double x = xs[k];
      if (v == 4) x -= eref;
      if (v == 0) x -= rho0;
      sU[at(le, v, pt % n, (pt / n) % n, pt / (n * n))] = x;
    }
  }
  lds_barrier();
  if constexpr (FB) {
    // the face bases: the values at the first flux point (a = b = 0)
    for (int it = tid; it < EB * 15; it += NT) {
      const int le = it / 15, r0 = it - le * 15, ax = r0 / 5, v = r0 - ax * 5, e = e0 + le;
      double bm = 0.0, bp = 0.0;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double x = sU[ax == 0 ? at(le, v, i, 0, 0) : (ax == 1 ? at(le, v, 0, i, 0) : at(le, v, 0, 0, i))];
        bm += op.lb[i] * x;
        bp += op.rb[i] * x;
      }
      const float fm = float(bm), fp = float(bp);
      sB[le][2 * ax][v] = double(fm);
      sB[le][2 * ax + 1][v] = double(fp);
      if (e < E) {
        const size_t s0 = (size_t)(slot_base + e * 6 + 2 * ax);
        sg.Ub[s0 * 5 + v] = fm;
        sg.Ub[(s0 + 1) * 5 + v] = fp;
      }
    }
    lds_barrier();
  }
  // one line (axis, flux point) per item, all five fields along it
  for (int it = tid; it < EB * 3 * NFP; it += NT) {
    const int le = it / (3 * NFP), r0 = it - le * (3 * NFP), ax = r0 / NFP, r = r0 - ax * NFP;
    const int a = r % n, b = r / n, e = e0 + le;
    if (e >= E) continue;
    const int si = ax == 0 ? 1 : (ax == 1 ? LX : LX * n);
    const double* X = sU + le * 5 * NUP + (ax == 0 ? LX * (a + n * b) : (ax == 1 ? a + LX * n * b : a + LX * b));
    R* __restrict__ um = Uf + (size_t)(sg.po_base + (e * 6 + 2 * ax) * NFP) * 5 + r;
    R* __restrict__ up = um + 5 * NFP;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double xm = 0.0, xp = 0.0;
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double x = X[v * NUP + i * si];
        xm += op.lb[i] * x;
        xp += op.rb[i] * x;
      }
      if constexpr (FB) {
        xm -= sB[le][2 * ax][v];
        xp -= sB[le][2 * ax + 1][v];
      }
      um[v * NFP] = R(xm);
      up[v * NFP] = R(xp);
    }
  }
  if (!lin) return;
  R* __restrict__ Rp = (R*)sg.Rp;
  for (int it = tid; it < EB * NU; it += NT) {
    const int le = it / NU, s = it - le * NU, e = e0 + le;
    if (e >= E) continue;
    const int i = s % n, j = (s / n) % n, k = s / (n * n);
    const int ix[3] = {i, j, k};
    // the line through the point along each axis: start and stride in LDS
    const int lb[3] = {LX * (j + n * k), i + LX * n * k, i + LX * j}, ls[3] = {1, LX, LX * n};
    const double* M = sU + le * 5 * NUP + NUP;  // momentum components
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double ad = 0.0;
#pragma unroll
      for (int q = 0; q < n; ++q) {
        const int o = lb[d] + q * ls[d];
        if constexpr (DIAG) {
          ad += sD[ix[d]][q] * M[d * NUP + o];
        } else {
          const double sm = sS[le][3 * d] * M[o] + sS[le][3 * d + 1] * M[NUP + o] + sS[le][3 * d + 2] * M[2 * NUP + o];
          ad += sD[ix[d]][q] * sm;
        }
      }
      acc += DIAG ? sS[le][4 * d] * ad : ad;
    }
    Rp[(size_t)e * 5 * NU + s] = R(acc);
  }
}

// --------------------------------------------------------------- volume
// LDS per element, in the order the phases use it:
//   region A, offset 0: the state + gradients (20 fields at the solution
//     points); region B, after A: the neighbour face states (and the
//     surface-flux AA staging);
//   offset 0: the x-interpolated fields T1, written over A and B once every
//     thread holds its x rows in registers (the state and gradients are dead
//     after the x sweep);
//   offset 0: the z-projected flux Z, written after every column has read
//     T1; the y-projected residual Y is written inside Z, each thread into
//     the Z entries that only it reads.
// The footprint is the largest of A + B, T1 and Z (p = 3: 2160 values
// instead of 3440 with separate regions).  Measured at 48^3 (volume group):
// FP32 p = 3 with 7 elements per workgroup 0.736 -> 0.627 ms, FP32 p = 4
// 1.51 -> 1.24 ms, FP64 p = 3 1.89 -> 1.51 ms.  At p = 4 in FP64, with
// surface-flux AA or curved, T1 stays after region A and Y after Z (the
// footprint is the larger of A + B + T1 and Z + Y): the x rows held in
// registers there spill (FP64: 4.29 -> 4.54 ms).
template <int P, bool LIN>
struct HexVol {
  static constexpr int n = P + 1, m = P + 3, NU = n * n * n, NFP = n * n;
  // variables whose flux is projected: LIN leaves out the mass flux (its
  // divergence is L(rho v), formed by the disu kernel)
  static constexpr int NVF = LIN ? 4 : 5, V0 = 5 - NVF;
  static constexpr int SZ_X = 20 * NU, SZ_Y = 2 * NVF * m * n * n;
  static constexpr int SZ_A = SZ_X > SZ_Y ? SZ_X : SZ_Y;
  // x-interpolated fields T1 [20][m][TPS]; at p = 4 the rows of n^2 are
  // padded to n^2 + 1 so that the quadrature columns of a wave read
  // different banks (measured at 48^3: 1% faster in FP32, 4% in FP64; at
  // p = 3 the unpadded rows are faster)
  static constexpr int TPS = P >= 4 ? NFP + 1 : NFP;
  static constexpr int SZ_T1 = 20 * m * TPS, SZ_Z = 3 * NVF * m * m * n, SZ_J = 30 * NFP;
  // surface-flux anti-aliasing, per axis: face values interpolated along the
  // first tangential axis [2][20][m][n], viscous flux at the face
  // quadrature points [2][4][m][m]
  static constexpr int SZ_ST = 2 * 20 * m * n, SZ_S = SZ_ST + 2 * 4 * m * m;
  // T1 over region A and Y inside Z (TOX), or T1 after region A and Y after
  // Z; at p = 4 in FP64, with surface-flux AA (SAA) or curved (WARP) the
  // registers that hold the x rows across the barrier spill
  template <typename R, bool SAA, bool WARP>
  static constexpr bool tox() { return !(P >= 4 && (sizeof(R) == 8 || SAA || WARP)); }
  // per element with flux anti-aliasing; SAA: with surface-flux AA staging
  static constexpr int per_elem(bool SAA, bool TOX) {
    const int b0 = SAA && SZ_S > SZ_J ? SZ_S : SZ_J;
    const int b = TOX || b0 > SZ_T1 ? b0 : SZ_T1;
    const int t = TOX ? (SZ_T1 > SZ_Z ? SZ_T1 : SZ_Z) : SZ_Z + SZ_Y;
    return SZ_A + b > t ? SZ_A + b : t;
  }
};

// Loads of one batch of EB elements, held in registers: the state, face
// records, face geometry and metrics first (independent loads), then the
// neighbour face states (gathered through face records in LDS).  Every
// thread issues all of its loads before the first use.  The state is
// loaded element by element (item r = tid + k NT of each element), so the
// LDS position and the reference-state shift of an item follow from tid and
// compile-time constants; the gather takes one neighbour flux point per item
// with its five fields.
template <int P, typename R, int EB, int NT, bool LIN>
struct HexVolLoads {
  using C = HexVol<P, LIN>;
  static constexpr int NU = C::NU, NFP = C::NFP;
  static constexpr int NR = (5 * NU + NT - 1) / NT;         // state items per element
  static constexpr int NG = (EB * 6 * NFP + NT - 1) / NT;   // neighbour flux points
  static constexpr int NF = (EB * 6 + NT - 1) / NT;
  static constexpr int NM = (EB * 10 + NT - 1) / NT;
  double xs[EB][NR];
  R gv[NG][5];
  FaceRec fr[NF];
  R fg[NF][4];
  R mt[NM];

  // branch-free: an out-of-range item loads from a valid address (the
  // segment's first element) and its value is never used for an output (every
  // store of the kernel is guarded by the element count), so no select
  // follows the load and the compiler can keep all loads in flight
  __device__ __forceinline__ void load(const double* __restrict__ U, const FaceRec* __restrict__ faces,
                                       const R* __restrict__ fgeo, const R* __restrict__ met, int e0, int E,
                                       int slot_base, int tid) {
    const int nv = E - e0 < EB ? E - e0 : EB;  // valid elements of the batch
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int it = tid + k * NT;
      const bool ok = it < nv * 6;
      const int slot = slot_base + (ok ? e0 * 6 + it : 0);
      fr[k] = faces[slot];
#pragma unroll
      for (int c = 0; c < 4; ++c) fg[k][c] = fgeo[4 * slot + c];
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int it = tid + k * NT;
      mt[k] = met[it < nv * 10 ? (size_t)e0 * 10 + it : 0];
    }
#pragma unroll
    for (int le = 0; le < EB; ++le)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int r = tid + k * NT;
        xs[le][k] = U[le < nv && r < 5 * NU ? (size_t)(e0 + le) * 5 * NU + r : 0];
      }
  }
  __device__ __forceinline__ void put_faces(FaceRec* sFR, R (*sFG)[4], int tid) const {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int it = tid + k * NT;
      if (it < EB * 6) {
        sFR[it] = fr[k];
#pragma unroll
        for (int c = 0; c < 4; ++c) sFG[it][c] = fg[k][c];
      }
    }
  }
  // face records of out-of-range elements are those of a valid slot, so
  // every gathered address is valid; only in-range values are ever used.
  // Single precision adds the neighbour face's base.
  __device__ __forceinline__ void gather(const R* __restrict__ Uf, const float* __restrict__ Ub,
                                         const FaceRec* sFR, const uint8_t* sPerm, int tid) {
    R gb[NG][5];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int it = tid + k * NT;
      const int itc = it < EB * 6 * NFP ? it : 0;
      const int lf = itc / NFP, r = itc - lf * NFP;  // lf = le * 6 + f
      const FaceRec q = sFR[lf];
      const R* __restrict__ src = Uf + (size_t)q.npo * 5 + sPerm[(q.info >> 1) * NFP + r];
#pragma unroll
      for (int v = 0; v < 5; ++v) gv[k][v] = src[v * NFP];
      if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int v = 0; v < 5; ++v) gb[k][v] = Ub[(size_t)q.nbr * 5 + v];
      }
    }
    if constexpr (sizeof(R) == 4) {
#pragma unroll
      for (int k = 0; k < NG; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) gv[k][v] += gb[k][v];
    }
  }
  // state in reference form, metrics and neighbour states to LDS (pe: LDS
  // values per element)
  __device__ __forceinline__ void put_elems(R* smem, R (*sMet)[10], double eref, double rho0, int pe,
                                            int tid) const {
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int it = tid + k * NT;
      if (it < EB * 10) sMet[it / 10][it % 10] = mt[k];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = tid + k * NT;
      if (r < 5 * NU) {
        const double sh = r < NU ? rho0 : (r >= 4 * NU ? eref : 0.0);
#pragma unroll
        for (int le = 0; le < EB; ++le) smem[le * pe + r] = R(xs[le][k] - sh);
      }
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int it = tid + k * NT;
      if (it < EB * 6 * NFP) {
        const int lf = it / NFP, r = it - lf * NFP, le = lf / 6, f = lf - le * 6;
        R* dst = smem + le * pe + C::SZ_A + f * 5 * NFP + r;
#pragma unroll
        for (int v = 0; v < 5; ++v) dst[v * NFP] = gv[k][v];
      }
    }
  }
};

// AA: flux anti-aliasing (quadrature GL(p+3)^3); without it the flux is
// evaluated at the solution points and its divergence uses -W^-1 D^T W
// along each direction (exact for the GL solution points).
// SAA: surface-flux anti-aliasing (face quadrature GL(p+3)^2).  With the
// flux points moved to the face quadrature points, the lifting of face data
// factorises into the projection P x P onto the GL(n)^2 flux points followed
// by the lifting of those (the GL(m) rule integrates l_u L_f exactly).  The
// common solution is linear in the two sides' states and the LDG viscous
// flux is linear in the two sides' normal viscous fluxes, so the projected
// common solution is the common solution of the flux-point states, and each
// side may project its own viscous flux: this kernel evaluates n . f^v at
// the face quadrature points (from the solution and corrected gradient
// interpolated there) and stores its projection at the flux points.  Only
// the Rusanov flux, nonlinear in the pair, is left to the interface kernel.
template <int P, typename R, int EB, int NT, bool DIAG, bool BT, bool AA, bool SAA, bool WARP>
__global__ void __launch_bounds__(NT)
    hex_volume(const Seg one, const BlkRef* __restrict__ bt, const Seg* __restrict__ segs, const bool from_ust,
               const HexOps<P, R> op, const Gas<R> g, const double eref, const double rho0) {
  // LIN: the mass flux's divergence and the linear energy-flux part come
  // from the disu kernel's L(rho v) (affine elements only)
  constexpr bool LIN = !WARP;
  using C = HexVol<P, LIN>;
  constexpr int n = C::n, m = C::m, NU = C::NU, NFP = C::NFP, NVF = C::NVF, V0 = C::V0;
  constexpr int SZ_BN = SAA && C::SZ_S > C::SZ_J ? C::SZ_S : C::SZ_J;  // region B without AA
  constexpr bool TOX = C::template tox<R, SAA, WARP>();
  constexpr int PE = AA ? C::per_elem(SAA, TOX) : C::SZ_A + SZ_BN;
  static_assert(EB * m * m <= NT, "one quadrature column per thread");
  __shared__ R smem[EB * PE];
  __shared__ R sMet[EB][10];
  __shared__ FaceRec sFR[EB * 6];
  __shared__ R sFG[EB * 6][4];
  __shared__ uint8_t sPerm[MAX_PERMS * NFP];
  __shared__ R sI[m][n];  // interpolation rows, read with a per-thread row index
  __shared__ R sV[WARP ? EB : 1][24];  // curved: element vertices
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const double* __restrict__ U = from_ust ? sg.ust : sg.U;
  const R* __restrict__ Uf = (const R*)sg.Uf;
  R* __restrict__ Vf = (R*)sg.Vf;
  R* __restrict__ Rp = (R*)sg.Rp;
  const FaceRec* __restrict__ faces = sg.faces;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
  const R* __restrict__ met = (const R*)sg.met;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
#define XS(le) (smem + (le)*PE)            /* [20][NU]                     */
#define YS(le) (smem + (le)*PE + (TOX ? 0 : C::SZ_Z)) /* [2][NVF][m][YB][n] */
#define JS(le) (smem + (le)*PE + C::SZ_A)  /* [6][5][NFP] neighbour u^f    */
#define TS(le) (smem + (le)*PE + (TOX ? 0 : C::SZ_A)) /* [20][m][TPS]      */
#define ZS(le) (smem + (le)*PE)            /* [3][NVF][m][m][n]            */
#define SS(le) (smem + (le)*PE + C::SZ_A)  /* [2][20][m][n], [2][4][m][m]  */

  // phase 0: state (reference form), metrics, neighbour states at own
  // faces.  Face records, face geometry and the permutation table go to LDS
  // first, so the neighbour gather is one global load per value.
  for (int it = tid; it < sg.nperm * NFP; it += NT) sPerm[it] = sg.perms[it];
  if (tid < m * n) sI[tid / n][tid % n] = op.I[tid / n][tid % n];
  HexVolLoads<P, R, EB, NT, LIN> ld;
  ld.load(U, faces, fgeo, met, e0, E, slot_base, tid);
  ld.put_faces(sFR, sFG, tid);
  if constexpr (WARP) {
    const R* __restrict__ vx = (const R*)sg.verts;
    for (int it = tid; it < EB * 24; it += NT) {
      const int le = it / 24;
      sV[le][it - le * 24] = vx[e0 + le < E ? (size_t)e0 * 24 + it : 0];
    }
  }
  lds_barrier();
  ld.gather(Uf, sg.Ub, sFR, sPerm, tid);
  ld.put_elems(smem, sMet, eref, rho0, PE, tid);
  lds_barrier();
  const FaceRec* cFR = sFR;
  const R (*cFG)[4] = sFG;

  // phase 1: per axis and line: own face values, jumps C - u^f (eq. FR-conu:
  // L side (1/2 + beta)(u_nbr - u_own), R side (1/2 - beta)(u_nbr - u_own)),
  // and the corrected gradient D u + lift (eq. FR-qfinal).  With a diagonal
  // metric the J^-T scaling of eq. FR-gradcoru is applied here as well.
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int si = ax == 0 ? 1 : (ax == 1 ? n : n * n);
    const int sa = ax == 0 ? n : 1, sb = ax == 2 ? n : n * n;
    for (int it = tid; it < EB * 5 * NFP; it += NT) {
      const int le = it / (5 * NFP), r0 = it - le * (5 * NFP), v = r0 / NFP, r = r0 - v * NFP;
      const int a = r % n, b = r / n;
      R* X = XS(le);
      const int base = a * sa + b * sb;
      R x[n];
#pragma unroll
      for (int i = 0; i < n; ++i) x[i] = X[v * NU + base + i * si];
      R xm = R(0), xp = R(0);
#pragma unroll
      for (int i = 0; i < n; ++i) {
        xm += op.lb[i] * x[i];
        xp += op.rb[i] * x[i];
      }
      const int im = cFR[le * 6 + 2 * ax].info, ip = cFR[le * 6 + 2 * ax + 1].info;
      const R jm = ((im & 1) ? R(0.5) + g.beta : R(0.5) - g.beta) * (JS(le)[((2 * ax) * 5 + v) * NFP + r] - xm);
      const R jp = ((ip & 1) ? R(0.5) + g.beta : R(0.5) - g.beta) * (JS(le)[((2 * ax + 1) * 5 + v) * NFP + r] - xp);
      const R sc = DIAG ? sMet[le][4 * ax] : R(1);
#pragma unroll
      for (int i = 0; i < n; ++i) {
        R s = op.liftR[i] * jp - op.liftL[i] * jm;
#pragma unroll
        for (int c = 0; c < n; ++c) s += op.D[i][c] * x[c];
        X[(5 + ax * 5 + v) * NU + base + i * si] = sc * s;
      }
    }
  }
  lds_barrier();

  if (!DIAG) {
    // phase 2: physical gradient q = J^-T q~ (eq. FR-gradcoru), in place
    for (int it = tid; it < EB * NU; it += NT) {
      const int le = it / NU, s = it - le * NU;
      R* X = XS(le);
      R M[3][3];  // M[d][c] = (J^-1)_{dc}
      if constexpr (WARP) {
        R S[3][3], det;
        trilinear_metric(&sV[le][0], sel(op.x, s % n), sel(op.x, (s / n) % n), sel(op.x, s / (n * n)), S, det);
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
  }

  if constexpr (SAA) {
    // phase 3a with surface-flux anti-aliasing, one axis (two faces) at a
    // time: S1 interpolates the 20 fields to the face (normal direction) and
    // along the first tangential axis to GL(m); S2 along the second and
    // evaluates n . f^v at each face quadrature point; S3 projects it back to
    // the flux points (P along the second axis, then the first)
    __shared__ R sPj[n][m];  // read with a per-thread row index
    if (tid < n * m) sPj[tid / m][tid % m] = op.Pj[tid / m][tid % m];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      for (int it = tid; it < EB * 40 * n; it += NT) {
        const int le = it / (40 * n), r0 = it - le * (40 * n), side = r0 / (20 * n), r1 = r0 - side * (20 * n);
        const int fld = r1 / n, b = r1 - fld * n;
        const R* X = XS(le) + fld * NU;
        R y[n];
#pragma unroll
        for (int a = 0; a < n; ++a) {
          R s = R(0);
#pragma unroll
          for (int i = 0; i < n; ++i) s += (side ? op.rb[i] : op.lb[i]) * X[hex_pt<n>(ax, i, a, b)];
          y[a] = s;
        }
        R* T = SS(le) + (side * 20 + fld) * m * n + b;
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) {
          R s = R(0);
#pragma unroll
          for (int a = 0; a < n; ++a) s += op.I[a2][a] * y[a];
          T[a2 * n] = s;
        }
      }
      lds_barrier();
      for (int it = tid; it < EB * 2 * m * m; it += NT) {
        const int le = it / (2 * m * m), r0 = it - le * (2 * m * m), side = r0 / (m * m), r1 = r0 - side * (m * m);
        const int a2 = r1 / m, b2 = r1 - a2 * m;
        R Ib[n];
#pragma unroll
        for (int j = 0; j < n; ++j) Ib[j] = sI[b2][j];
        const R* T = SS(le) + (side * 20 * m + a2) * n;
        R w[20];
#pragma unroll
        for (int fld = 0; fld < 20; ++fld) {
          R s = R(0);
#pragma unroll
          for (int b = 0; b < n; ++b) s += Ib[b] * T[fld * m * n + b];
          w[fld] = s;
        }
        const int lf = le * 6 + 2 * ax + side;
        const R sgn = (cFR[lf].info & 1) ? R(1) : R(-1);
        const R nn[3] = {sgn * cFG[lf][0], sgn * cFG[lf][1], sgn * cFG[lf][2]};
        R u[5], q[3][5], V[4];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          u[v] = w[v];
#pragma unroll
          for (int d = 0; d < 3; ++d) q[d][v] = w[5 + d * 5 + v];
        }
        normal_viscous(u, q, nn, g, V);
        R* VQ = SS(le) + C::SZ_ST + side * 4 * m * m + a2 * m + b2;
#pragma unroll
        for (int k = 0; k < 4; ++k) VQ[k * m * m] = V[k];
      }
      lds_barrier();
      // the next axis's S1 writes T (read above, before the barrier) and its
      // S2 writes VQ only after the next barrier
      for (int it = tid; it < EB * 8 * n; it += NT) {
        const int le = it / (8 * n), r0 = it - le * (8 * n), side = r0 / (4 * n), r1 = r0 - side * (4 * n);
        const int k = r1 / n, b = r1 - k * n, e = e0 + le;
        if (e >= E) continue;
        R pb[m];
#pragma unroll
        for (int b2 = 0; b2 < m; ++b2) pb[b2] = sPj[b][b2];
        const R* VQ = SS(le) + C::SZ_ST + (side * 4 + k) * m * m;
        R z[m];
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) {
          R s = R(0);
#pragma unroll
          for (int b2 = 0; b2 < m; ++b2) s += pb[b2] * VQ[a2 * m + b2];
          z[a2] = s;
        }
        const size_t po = (size_t)(sg.po_base + (e * 6 + 2 * ax + side) * NFP);
#pragma unroll
        for (int a = 0; a < n; ++a) {
          R s = R(0);
#pragma unroll
          for (int a2 = 0; a2 < m; ++a2) s += op.Pj[a][a2] * z[a2];
          Vf[po * 4 + k * NFP + a + n * b] = s;
        }
      }
    }
    lds_barrier();  // region B is reused below
  } else {
  // phase 3a: gradcoru_fpts + normal viscous flux at the own flux points
  for (int it = tid; it < EB * 3 * NFP; it += NT) {
    const int le = it / (3 * NFP), r0 = it - le * (3 * NFP), ax = r0 / NFP, r = r0 - ax * NFP;
    const int a = r % n, b = r / n, e = e0 + le;
    if (e >= E) continue;
    const int si = ax == 0 ? 1 : (ax == 1 ? n : n * n);
    const int base = ax == 0 ? n * a + n * n * b : (ax == 1 ? a + n * n * b : a + n * b);
    const R* X = XS(le);
    R fm[20], fp[20];
#pragma unroll
    for (int fld = 0; fld < 20; ++fld) {
      R sm = R(0), sp = R(0);
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const R x = X[fld * NU + base + i * si];
        sm += op.lb[i] * x;
        sp += op.rb[i] * x;
      }
      fm[fld] = sm;
      fp[fld] = sp;
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const R* w = side ? fp : fm;
      const int lf = le * 6 + 2 * ax + side, po = sg.po_base + (e * 6 + 2 * ax + side) * NFP;
      R nn[3];
      if constexpr (WARP) {
        // own outward unit normal at this flux point: +-S_ax / |S_ax|
        R px, py, pz, S[3][3], det;
        grid_point(ax, side ? R(1) : R(-1), sel(op.x, a), sel(op.x, b), px, py, pz);
        trilinear_metric(&sV[le][0], px, py, pz, S, det);
        const R im = rcp(sqrt(S[ax][0] * S[ax][0] + S[ax][1] * S[ax][1] + S[ax][2] * S[ax][2]));
#pragma unroll
        for (int c = 0; c < 3; ++c) nn[c] = (side ? im : -im) * S[ax][c];
      } else {
        const R sgn = (cFR[lf].info & 1) ? R(1) : R(-1);
#pragma unroll
        for (int c = 0; c < 3; ++c) nn[c] = sgn * cFG[lf][c];
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
      for (int k = 0; k < 4; ++k) Vf[(size_t)po * 4 + k * NFP + r] = V[k];
    }
  }
  }
  if constexpr (!AA) {
    // no anti-aliasing: transformed flux at each solution point, in place
    // over the gradients (tdisf), then its divergence (M1 - M3 M2) as
    // -W^-1 D^T W along each direction
    __shared__ R sAPu[n][n];  // read with a per-thread row index
    if (tid < n * n) sAPu[tid / n][tid % n] = op.APu[tid / n][tid % n];
    lds_barrier();  // the face viscous fluxes have read the gradients
    for (int it = tid; it < EB * NU; it += NT) {
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
        for (int v = V0; v < 5; ++v) {
          const R ft = DIAG ? sMet[le][4 * d] * f[d][v]
                            : sMet[le][3 * d] * f[0][v] + sMet[le][3 * d + 1] * f[1][v] + sMet[le][3 * d + 2] * f[2][v];
          X[(5 + d * 5 + v) * NU + s] = dj * ft;
        }
    }
    lds_barrier();
    for (int it = tid; it < EB * NVF * NU; it += NT) {
      const int le = it / (NVF * NU), r1 = it - le * (NVF * NU), v = V0 + r1 / NU, s = r1 - (v - V0) * NU;
      const int e = e0 + le;
      if (e >= E) continue;
      const int i = s % n, j = (s / n) % n, k = s / (n * n);
      const R* F = XS(le) + 5 * NU + v * NU;  // component d at F + d * 5 NU
      R acc = R(0);
      if (LIN && v == 4) acc = g.kap * Rp[(size_t)e * 5 * NU + s];  // kap L(rho v)
#pragma unroll
      for (int c = 0; c < n; ++c) {
        acc += sAPu[i][c] * F[0 * 5 * NU + c + n * (j + n * k)];
        acc += sAPu[j][c] * F[1 * 5 * NU + i + n * (c + n * k)];
        acc += sAPu[k][c] * F[2 * 5 * NU + i + n * (j + n * c)];
      }
      Rp[(size_t)e * 5 * NU + v * NU + s] = acc;
    }
    return;
  }
  // phase 3b: x interpolation of the 20 fields (first factor of M7 / M10).
  // Over region A (TOX) every thread reads its x rows into registers before
  // a barrier and writes T1 after it.
  if constexpr (TOX) {
    constexpr int NIT = (EB * 20 * NFP + NT - 1) / NT;
    R x[NIT][n];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = tid + k * NT;
      if (it < EB * 20 * NFP) {
        const int le = it / (20 * NFP), r0 = it - le * (20 * NFP), fld = r0 / NFP, r = r0 - fld * NFP;
#pragma unroll
        for (int i = 0; i < n; ++i) x[k][i] = XS(le)[fld * NU + i + n * r];
      }
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = tid + k * NT;
      if (it < EB * 20 * NFP) {
        const int le = it / (20 * NFP), r0 = it - le * (20 * NFP), fld = r0 / NFP, r = r0 - fld * NFP;
        const int j = r % n, l = r / n;
        R* T = TS(le) + (fld * m) * C::TPS + j * n + l;
#pragma unroll
        for (int a = 0; a < m; ++a) {
          R s = R(0);
#pragma unroll
          for (int i = 0; i < n; ++i) s += op.I[a][i] * x[k][i];
          T[a * C::TPS] = s;
        }
      }
    }
  } else {
    for (int it = tid; it < EB * 20 * NFP; it += NT) {
      const int le = it / (20 * NFP), r0 = it - le * (20 * NFP), fld = r0 / NFP, r = r0 - fld * NFP;
      const int j = r % n, l = r / n;
      R x[n];
#pragma unroll
      for (int i = 0; i < n; ++i) x[i] = XS(le)[fld * NU + i + n * r];
      R* T = TS(le) + (fld * m) * C::TPS + j * n + l;
#pragma unroll
      for (int a = 0; a < m; ++a) {
        R s = R(0);
#pragma unroll
        for (int i = 0; i < n; ++i) s += op.I[a][i] * x[i];
        T[a * C::TPS] = s;
      }
    }
  }
  lds_barrier();

  // phase 4: one quadrature column (a, b) per thread: y interpolation, then
  // for each z level: z interpolation (uqpts, gradcoru_qpts), the flux
  // (tdisf, eq. FR-tdisfq) and the z factor of the projection-divergence
  const bool col = tid < EB * m * m;
  const int cle = tid / (m * m), cr = tid - cle * (m * m), ca = cr / m, cb = cr - ca * m;
  R acc[3][NVF][n];
  if (col) {
    R Ib[n];
#pragma unroll
    for (int j = 0; j < n; ++j) Ib[j] = sI[cb][j];
    R t2[20][n];
    const R* T = TS(cle) + ca * C::TPS;
#pragma unroll
    for (int fld = 0; fld < 20; ++fld) {
#pragma unroll
      for (int l = 0; l < n; ++l) t2[fld][l] = R(0);
#pragma unroll
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int l = 0; l < n; ++l) t2[fld][l] += Ib[j] * T[fld * m * C::TPS + j * n + l];
    }
    R S[3][3];
    const R dj = sMet[cle][9];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int c = 0; c < 3; ++c) S[d][c] = DIAG ? (d == c ? dj * sMet[cle][4 * d] : R(0)) : dj * sMet[cle][3 * d + c];
    const R qx = WARP ? sel(op.xq, ca) : R(0), qy = WARP ? sel(op.xq, cb) : R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < NVF; ++v)
#pragma unroll
        for (int l = 0; l < n; ++l) acc[d][v][l] = R(0);
    // the z levels in a loop (not unrolled), so that the operator entries of
    // one level are live at a time.  Fully unrolled, the FP64 constants of
    // all levels spill out of the scalar registers (p = 3 at 48^3: 1.81 ->
    // 1.49 ms as a loop); in single precision the loop is 2% faster at p = 3
    // and 4 (smaller code).  FP64 at p = 4 stays unrolled (the loop was 5%
    // slower there).
    constexpr int KQ_UNROLL = sizeof(R) == 8 && P >= 4 ? m : 1;
#pragma unroll KQ_UNROLL
    for (int kq = 0; kq < m; ++kq) {
      R u[5], q[3][5], f[3][5];
#pragma unroll
      for (int fld = 0; fld < 20; ++fld) {
        R s = R(0);
#pragma unroll
        for (int l = 0; l < n; ++l) s += op.I[kq][l] * t2[fld][l];
        if (fld < 5)
          u[fld] = s;
        else
          q[(fld - 5) / 5][(fld - 5) % 5] = s;
      }
      point_flux(u, q, g, f);
      if constexpr (WARP) {
        R det;
        trilinear_metric(&sV[cle][0], qx, qy, op.xq[kq], S, det);  // det J J^-1 at this point
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = V0; v < 5; ++v) {
          const R ft = DIAG ? S[d][d] * f[d][v] : S[d][0] * f[0][v] + S[d][1] * f[1][v] + S[d][2] * f[2][v];
#pragma unroll
          for (int l = 0; l < n; ++l) acc[d][v - V0][l] += (d == 2 ? op.AP[l][kq] : op.Pj[l][kq]) * ft;
        }
    }
  }
  lds_barrier();  // every column has read T1; Z may now overwrite it
  if (col) {
    R* Z = ZS(cle);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < NVF; ++v)
#pragma unroll
        for (int l = 0; l < n; ++l) Z[(((d * NVF + v) * m + ca) * m + cb) * n + l] = acc[d][v][l];
  }
  lds_barrier();

  // phase 5: y projection: X' = P_y X, Y' = AP_y Y + P_y Z.  Inside Z
  // (TOX), Y[d][v][a][j][l] takes the place of Z[d][v][a][j][l], which only
  // this thread reads (into registers, before it writes).
  constexpr int YB = TOX ? m : n;
  for (int it = tid; it < EB * NVF * m * n; it += NT) {
    const int le = it / (NVF * m * n), r0 = it - le * (NVF * m * n);
    const int v = r0 / (m * n), r1 = r0 - v * (m * n), a = r1 / n, l = r1 - a * n;
    const R* Z = ZS(le);
    R zx[m], zy[m], zz[m];
#pragma unroll
    for (int b = 0; b < m; ++b) {
      zx[b] = Z[(((0 * NVF + v) * m + a) * m + b) * n + l];
      zy[b] = Z[(((1 * NVF + v) * m + a) * m + b) * n + l];
      zz[b] = Z[(((2 * NVF + v) * m + a) * m + b) * n + l];
    }
    R* Y = YS(le);
#pragma unroll
    for (int j = 0; j < n; ++j) {
      R sx = R(0), sy = R(0);
#pragma unroll
      for (int b = 0; b < m; ++b) {
        sx += op.Pj[j][b] * zx[b];
        sy += op.AP[j][b] * zy[b];
        sy += op.Pj[j][b] * zz[b];
      }
      Y[(((0 * NVF + v) * m + a) * YB + j) * n + l] = sx;
      Y[(((1 * NVF + v) * m + a) * YB + j) * n + l] = sy;
    }
  }
  lds_barrier();

  // phase 6: x projection: R_vol = AP_x X' + P_x Y'; LIN: the energy
  // residual takes kap L(rho v) (row 0, from the disu kernel), which also
  // is the mass residual
  for (int it = tid; it < EB * NVF * NFP; it += NT) {
    const int le = it / (NVF * NFP), r0 = it - le * (NVF * NFP), v = r0 / NFP, r = r0 - v * NFP;
    const int j = r % n, l = r / n, e = e0 + le;
    if (e >= E) continue;
    R lin[n];
    if (LIN && v + V0 == 4) {
#pragma unroll
      for (int i = 0; i < n; ++i) lin[i] = Rp[(size_t)e * 5 * NU + i + n * (j + n * l)];
    }
    const R* Y = YS(le);
    R y0[m], y1[m];
#pragma unroll
    for (int a = 0; a < m; ++a) {
      y0[a] = Y[(((0 * NVF + v) * m + a) * YB + j) * n + l];
      y1[a] = Y[(((1 * NVF + v) * m + a) * YB + j) * n + l];
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
      R s = (LIN && v + V0 == 4) ? g.kap * lin[i] : R(0);
#pragma unroll
      for (int a = 0; a < m; ++a) {
        s += op.AP[i][a] * y0[a];
        s += op.Pj[i][a] * y1[a];
      }
      Rp[(size_t)e * 5 * NU + (v + V0) * NU + i + n * (j + n * l)] = s;
    }
  }
#undef XS
#undef YS
#undef JS
#undef TS
#undef ZS
#undef SS
}

// -------------------------------------------------------------- surface
// Face records, face geometry, the permutation table, the lifting weights
// and det J are staged in LDS; the volume residual is prefetched before the
// first barrier; every flux point's own and neighbour loads are issued
// branch-free (out-of-range items read a valid address and are dropped).
//
// With surface-flux anti-aliasing (SAA) the common flux is wanted at the
// GL(m)^2 face quadrature points and lifted from there, which equals lifting
// its projection P x P onto the flux points.  The part of the common flux
// that is linear in the two sides' values (LDG viscous flux, penalty) is
// projected already (the viscous fluxes arrive projected from the volume
// kernel; the states are face polynomials of degree p) and is evaluated at
// the flux points; the Rusanov flux is evaluated at the quadrature points
// from the interpolated pair of states and projected back.
template <int P, typename R, int EB, int NT, bool BT, bool SAA, bool WARP>
__global__ void __launch_bounds__(NT)
    hex_surface(const Seg one, const BlkRef* __restrict__ bt, const Seg* __restrict__ segs, const int rk,
                const HexOps<P, R> op, const Gas<R> g) {
  using C = HexCfg<P>;
  constexpr int n = C::n, m = C::m, NU = C::NU, NFP = C::NFP;
  constexpr int NI = (EB * 6 * NFP + NT - 1) / NT;  // flux points per thread
  constexpr int NL = (EB * 5 * NU + NT - 1) / NT;   // solution values per thread
  constexpr bool LIN = !WARP, FB = sizeof(R) == 4;
  // SAA staging per face: the L state and the jump uL - uR at the flux
  // points [10][NFP], later the Rusanov flux at the quadrature points
  // [5][m][m] (sW); both interpolated along the first tangential axis
  // [10][m][n] (sT)
  constexpr int SW = 10 * NFP > 5 * m * m ? 10 * NFP : 5 * m * m, ST = 10 * m * n;
  __shared__ R sD[EB * 30 * NFP];
  __shared__ R sW[SAA ? EB * 6 * SW : 1];
  __shared__ R sT[SAA ? EB * 6 * ST : 1];
  __shared__ R sI[SAA ? m : 1][n];  // rows read with a per-thread index
  __shared__ R sPj[SAA ? n : 1][m];
  __shared__ FaceRec sFR[EB * 6];
  __shared__ R sFG[EB * 6][4];
  __shared__ uint8_t sPerm[MAX_PERMS * NFP];
  __shared__ R sLift[2][n];
  __shared__ double sDet[EB];
  __shared__ R sV[WARP ? EB : 1][24];              // curved: element vertices
  __shared__ R sDetU[WARP ? EB : 1][WARP ? NU : 1];  // curved: det J at the solution points
  int e0;
  const Seg sg = seg_of<BT>(one, bt, segs, EB, e0);
  const R* __restrict__ Uf = (const R*)sg.Uf;
  const R* __restrict__ Vf = (const R*)sg.Vf;
  const R* __restrict__ Rp = (const R*)sg.Rp;
  const FaceRec* __restrict__ faces = sg.faces;
  const R* __restrict__ fgeo = (const R*)sg.fgeo;
  const int E = sg.E, slot_base = sg.slot_base, tid = threadIdx.x;
  for (int it = tid; it < EB * 6; it += NT) {
    const int slot = slot_base + (e0 + it / 6 < E ? e0 * 6 + it : 0);
    sFR[it] = faces[slot];
#pragma unroll
    for (int c = 0; c < 4; ++c) sFG[it][c] = fgeo[4 * slot + c];
  }
  for (int it = tid; it < sg.nperm * NFP; it += NT) sPerm[it] = sg.perms[it];
  if (tid < n) {
    sLift[0][tid] = op.liftL[tid];
    sLift[1][tid] = op.liftR[tid];
  }
  if (tid < EB) sDet[tid] = sg.detj[e0 + tid < E ? e0 + tid : 0];
  if constexpr (WARP) {
    const R* __restrict__ vx = (const R*)sg.verts;
    for (int it = tid; it < EB * 24; it += NT) {
      const int le = it / 24;
      sV[le][it - le * 24] = vx[e0 + le < E ? (size_t)e0 * 24 + it : 0];
    }
  }
  if constexpr (SAA) {
    if (tid < m * n) {
      sI[tid / n][tid % n] = op.I[tid / n][tid % n];
      sPj[tid / m][tid % m] = op.Pj[tid / m][tid % m];
    }
  }
  R rp[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int it = tid + k * NT;
    const bool ok = it < EB * 5 * NU && e0 + it / (5 * NU) < E;
    rp[k] = Rp[ok ? (size_t)e0 * 5 * NU + it : 0];
  }
  lds_barrier();
  // comm_flux: common normal flux at every own flux point, times mag.  The
  // jump u_nbr - u_own comes from the face bases and deviations (single
  // precision) before the states themselves are formed.
  {
    R uo[NI][5], un[NI][5], jn[NI][5], Vo[NI][4], Vn[NI][4];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int it = tid + q * NT;
      const int itc = it < EB * 6 * NFP ? it : 0;
      const int le = itc / (6 * NFP), r0 = itc - le * (6 * NFP), f = r0 / NFP, r = r0 - f * NFP;
      const int ls = e0 + le < E ? (e0 + le) * 6 + f : 0, slot = slot_base + ls;
      const size_t po = (size_t)(sg.po_base + ls * NFP);
      const FaceRec fr = sFR[le * 6 + f];
      const int rr = sPerm[(fr.info >> 1) * NFP + r];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        uo[q][v] = Uf[po * 5 + v * NFP + r];
        un[q][v] = Uf[(size_t)fr.npo * 5 + v * NFP + rr];
      }
      if constexpr (FB) {
#pragma unroll
        for (int v = 0; v < 5; ++v) jn[q][v] = sg.Ub[(size_t)fr.nbr * 5 + v];  // neighbour base
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const float bo = sg.Ub[(size_t)slot * 5 + v];
          const R d = un[q][v] - uo[q][v];
          const R bn = jn[q][v];
          jn[q][v] = (bn - bo) + d;
          uo[q][v] += bo;
          un[q][v] += bn;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Vo[q][k] = Vf[po * 4 + k * NFP + r];
        Vn[q][k] = Vf[(size_t)fr.npo * 4 + k * NFP + rr];
      }
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int it = tid + q * NT;
      if (it >= EB * 6 * NFP) continue;
      const int le = it / (6 * NFP), r0 = it - le * (6 * NFP), f = r0 / NFP, r = r0 - f * NFP;
      const int lf = le * 6 + f;
      const bool left = sFR[lf].info & 1;
      if constexpr (!FB) {
#pragma unroll
        for (int v = 0; v < 5; ++v) jn[q][v] = un[q][v] - uo[q][v];
      }
      R nL[3] = {sFG[lf][0], sFG[lf][1], sFG[lf][2]};
      R mag = sFG[lf][3];
      if constexpr (WARP) {
        // own area factor and outward normal at this flux point; the L side's
        // normal is the opposite of the R side's own
        const int ax = f >> 1, side = f & 1;
        R px, py, pz, S[3][3], det;
        grid_point(ax, side ? R(1) : R(-1), sel(op.x, r % n), sel(op.x, r / n), px, py, pz);
        trilinear_metric(&sV[le][0], px, py, pz, S, det);
        mag = sqrt(S[ax][0] * S[ax][0] + S[ax][1] * S[ax][1] + S[ax][2] * S[ax][2]);
        const R im = (side == (left ? 1 : 0)) ? rcp(mag) : -rcp(mag);
#pragma unroll
        for (int c = 0; c < 3; ++c) nL[c] = im * S[ax][c];
      }
      R D[5];
      if constexpr (SAA) {
        face_flux_linear<R, LIN>(jn[q], Vo[q], Vn[q], nL, left, g, D);
        // stage the L state and uL - uR for the Rusanov flux at the face
        // quadrature points
        R* W = sW + lf * SW + r;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          W[v * NFP] = left ? uo[q][v] : un[q][v];
          W[(5 + v) * NFP] = left ? -jn[q][v] : jn[q][v];
        }
      } else {
        face_flux<R, LIN>(uo[q], un[q], jn[q], Vo[q], Vn[q], nL, left, g, D);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) sD[lf * 5 * NFP + v * NFP + r] = mag * D[v];
    }
  }
  if constexpr (WARP) {
    for (int it = tid; it < EB * NU; it += NT) {
      const int le = it / NU, s = it - le * NU;
      R S[3][3], det;
      trilinear_metric(&sV[le][0], sel(op.x, s % n), sel(op.x, (s / n) % n), sel(op.x, s / (n * n)), S, det);
      sDetU[le][s] = det;
    }
  }
  lds_barrier();
  if constexpr (SAA) {
    // the pair of states along the first tangential axis to GL(m)
    for (int it = tid; it < EB * 60 * n; it += NT) {
      const int lf = it / (10 * n), r0 = it - lf * (10 * n), fld = r0 / n, b = r0 - fld * n;
      if (e0 + lf / 6 >= E) continue;
      const R* W = sW + lf * SW + fld * NFP + n * b;
      R y[n];
#pragma unroll
      for (int a = 0; a < n; ++a) y[a] = W[a];
      R* T = sT + lf * ST + fld * m * n + b;
#pragma unroll
      for (int a2 = 0; a2 < m; ++a2) {
        R s = R(0);
#pragma unroll
        for (int a = 0; a < n; ++a) s += op.I[a2][a] * y[a];
        T[a2 * n] = s;
      }
    }
    lds_barrier();
    // along the second axis, then the Rusanov flux at each quadrature point
    // (over the states: sW is free once the pass above has read it)
    for (int it = tid; it < EB * 6 * m * m; it += NT) {
      const int lf = it / (m * m), r0 = it - lf * (m * m), a2 = r0 / m, b2 = r0 - a2 * m;
      if (e0 + lf / 6 >= E) continue;
      R Ib[n];
#pragma unroll
      for (int j = 0; j < n; ++j) Ib[j] = sI[b2][j];
      const R* T = sT + lf * ST + a2 * n;
      R uL[5], jl[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        R sl = R(0), sj = R(0);
#pragma unroll
        for (int b = 0; b < n; ++b) {
          sl += Ib[b] * T[v * m * n + b];
          sj += Ib[b] * T[(5 + v) * m * n + b];
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
    lds_barrier();
    // projection to the flux points, added to the linear part
    for (int it = tid; it < EB * 30 * n; it += NT) {
      const int lf = it / (5 * n), r0 = it - lf * (5 * n), v = r0 / n, b = r0 - v * n;
      if (e0 + lf / 6 >= E) continue;
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
      const R sc = (sFR[lf].info & 1) ? sFG[lf][3] : -sFG[lf][3];
      R* D = sD + lf * 5 * NFP + v * NFP + n * b;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        R s = R(0);
#pragma unroll
        for (int a2 = 0; a2 < m; ++a2) s += op.Pj[a][a2] * z[a2];
        D[a] += sc * s;
      }
    }
    lds_barrier();
  }
  // tdivtconf (lift of the common flux, DG correction) + negdivconf
  double val[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int it = tid + k * NT;
    const int itc = it < EB * 5 * NU ? it : 0;
    const int le = itc / (5 * NU), r0 = itc - le * (5 * NU), v = r0 / NU, s = r0 - v * NU;
    const int i = s % n, j = (s / n) % n, kk = s / (n * n);
    const R* D = sD + le * 30 * NFP + v * NFP;
    R acc = rp[k];
    acc += sLift[0][i] * D[0 * 5 * NFP + j + n * kk] + sLift[1][i] * D[1 * 5 * NFP + j + n * kk];
    acc += sLift[0][j] * D[2 * 5 * NFP + i + n * kk] + sLift[1][j] * D[3 * 5 * NFP + i + n * kk];
    acc += sLift[0][kk] * D[4 * 5 * NFP + i + n * j] + sLift[1][kk] * D[5 * 5 * NFP + i + n * j];
    const double dj = WARP ? double(sDetU[le][s]) : sDet[le];
    val[k] = -double(acc) / dj;
  }
  rk_store_block<NL, NT>(sg, rk, e0, E, 5 * NU, EB * 5 * NU, tid, val);
}

// ------------------------------------------------------------ launchers
template <int P, typename R>
static HexOps<P, R> make_hex_ops(const HostOps& h) {
  HexOps<P, R> o;
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
    for (int j = 0; j < n; ++j) o.APu[i][j] = R(h.APu[i * n + j]);
    o.x[i] = R(h.x[i]);
  }
  for (int a = 0; a < m; ++a) o.xq[a] = R(h.xq[a]);
  return o;
}


// launch shapes of the volume kernel: EB elements per workgroup, NT threads,
// with EB * m^2 <= NT (one quadrature column per thread); the LDS footprint
// (EB elements) bounds the workgroups per CU, and the shapes below were the
// fastest of those measured at 48^3
template <int P, bool DBL>
struct HexLaunch;
template <> struct HexLaunch<1, false> { static constexpr int EB = 4, NT = 64; };   // 64 columns
template <> struct HexLaunch<2, false> { static constexpr int EB = 5, NT = 128; };  // 125
template <> struct HexLaunch<3, false> { static constexpr int EB = 5, NT = 256; };  // 180 (4 waves: measured
                                                                                    // 12 % faster than 3)
template <> struct HexLaunch<4, false> { static constexpr int EB = 1, NT = 64; };   // 49 (one-wave groups:
                                                                                    // 8 % faster than 2 elements)
template <> struct HexLaunch<1, true> { static constexpr int EB = 4, NT = 64; };
template <> struct HexLaunch<2, true> { static constexpr int EB = 2, NT = 64; };    // 50
template <> struct HexLaunch<3, true> { static constexpr int EB = 1, NT = 64; };    // 36
template <> struct HexLaunch<4, true> { static constexpr int EB = 1, NT = 64; };    // 49

// with flux anti-aliasing (AA) the footprint of the overlaid LDS regions
// fits more elements per workgroup in FP32.  BASE: the affine kernel without
// surface-flux AA.  p = 3: 6 elements per 256 threads (216 quadrature
// columns); at 168 VGPRs and 48 KB of LDS three workgroups share a CU (three
// waves per SIMD): 0.59 -> 0.51 ms at 48^3 against 7 elements (two
// workgroups per CU; 5 elements: 0.54 ms).  p = 4: 5 elements per 256
// threads (245 columns): 1.18 -> 1.13 ms against one-element one-wave
// groups.  The surface-AA and curved kernels keep 7 elements (p = 3) and
// one-wave groups (p = 4).
template <int P, bool DBL, bool AA, bool BASE = true>
struct HexVolLaunch : HexLaunch<P, DBL> {};
template <> struct HexVolLaunch<3, false, true, true> { static constexpr int EB = 6, NT = 256; };
template <> struct HexVolLaunch<3, false, true, false> { static constexpr int EB = 7, NT = 256; };
template <> struct HexVolLaunch<4, false, true, true> { static constexpr int EB = 5, NT = 256; };

// elements per workgroup of the disu kernel (256 threads; at 48^3, FP32
// p = 3: 4 elements 0.099 ms, 8 elements 0.107 ms, 16 elements 0.142 ms)
constexpr int HEX_DISU_EB = 4;
// elements per workgroup of the interface kernel (256 threads): at most two
// flux points and about five solution values per thread
template <int P, bool DBL, bool SAA = false>
struct HexSurf {
  // surface-flux anti-aliasing stages the face quadrature data in LDS: half
  // the elements per workgroup
  static constexpr int EB0 = (DBL ? 8 : 16) >> (P - 1);
  static constexpr int EB = SAA ? (EB0 > 1 ? EB0 / 2 : 1) : EB0;
};

template <int P, typename R, bool BT, bool DIAG, bool AA, bool SAA, bool WARP = false>
static void hex_volume_launch(const TypeArgs& a, int nb, const HexOps<P, R>& op, const Gas<R>& g, double eref,
                              hipStream_t st) {
  constexpr bool dbl = sizeof(R) == 8;
  using L = HexVolLaunch<P, dbl, AA, !SAA && !WARP>;
  constexpr int EB = L::EB, NT = L::NT;
  hipLaunchKernelGGL((hex_volume<P, R, EB, NT, DIAG, BT, AA, SAA, WARP>), dim3(nb), dim3(NT), 0, st, a.one,
                     a.bt[K_VOLUME], a.segs, a.from_ust, op, g, eref, a.gas->rho_ref);
}

// surface-flux anti-aliasing is built together with flux anti-aliasing only
// (the paper's "full AA"); the library rejects it without
template <int P, typename R, bool BT, bool DIAG>
static void hex_volume_dispatch(const TypeArgs& a, int nb, const HexOps<P, R>& op, const Gas<R>& g, double eref,
                                hipStream_t st) {
  if (a.saa)
    hex_volume_launch<P, R, BT, DIAG, true, true>(a, nb, op, g, eref, st);
  else if (a.aa)
    hex_volume_launch<P, R, BT, DIAG, true, false>(a, nb, op, g, eref, st);
  else
    hex_volume_launch<P, R, BT, DIAG, false, false>(a, nb, op, g, eref, st);
}

template <int P>
static HexDisuOps<P> make_disu_ops(const HostOps& h) {
  HexDisuOps<P> o;
  constexpr int n = P + 1;
  for (int i = 0; i < n; ++i) {
    o.lb[i] = h.lb[i];
    o.rb[i] = h.rb[i];
    for (int j = 0; j < n; ++j) o.D[i][j] = h.D[i * n + j];
  }
  return o;
}

template <int P, typename R, bool BT>
static void hex_launch(const TypeArgs& a, const int grid[3], hipStream_t st) {
  const HexOps<P, R> op = make_hex_ops<P, R>(*a.ops);
  // affine elements take the mass flux and the linear energy-flux part from
  // the double-precision L(rho v) of the disu kernel
  const bool lin = !a.warp;
  const Gas<R> g = make_gas<R>(*a.gas, lin);
  constexpr bool dbl = sizeof(R) == 8;
  constexpr int EBA = HEX_DISU_EB, NTA = 256, NTC = 256;
  const double eref = a.gas->pref / (a.gas->gamma - 1.0);
  if ((a.stage & 1) && grid[K_DISU] > 0) {
    if (a.diag && !a.warp)
      hipLaunchKernelGGL((hex_disu<P, R, EBA, NTA, BT, true>), dim3(grid[K_DISU]), dim3(NTA), 0, st, a.one,
                         a.bt[K_DISU], a.segs, a.from_ust, make_disu_ops<P>(*a.ops), eref, a.gas->rho_ref, lin);
    else
      hipLaunchKernelGGL((hex_disu<P, R, EBA, NTA, BT, false>), dim3(grid[K_DISU]), dim3(NTA), 0, st, a.one,
                         a.bt[K_DISU], a.segs, a.from_ust, make_disu_ops<P>(*a.ops), eref, a.gas->rho_ref, lin);
  }
  // curved hexahedra (single meshes only; flux anti-aliasing, general metric)
  if constexpr (!BT) {
    if (a.warp) {
      if ((a.stage & 2) && grid[K_VOLUME] > 0)
        hex_volume_launch<P, R, false, false, true, false, true>(a, grid[K_VOLUME], op, g, eref, st);
      if ((a.stage & 4) && grid[K_SURFACE] > 0)
        hipLaunchKernelGGL((hex_surface<P, R, HexSurf<P, dbl>::EB, NTC, false, false, true>), dim3(grid[K_SURFACE]),
                           dim3(NTC), 0, st, a.one, a.bt[K_SURFACE], a.segs, a.rk, op, g);
      return;
    }
  }
  if ((a.stage & 2) && grid[K_VOLUME] > 0) {
    if (a.diag)
      hex_volume_dispatch<P, R, BT, true>(a, grid[K_VOLUME], op, g, eref, st);
    else
      hex_volume_dispatch<P, R, BT, false>(a, grid[K_VOLUME], op, g, eref, st);
  }
  if ((a.stage & 4) && grid[K_SURFACE] > 0) {
    if (a.saa)
      hipLaunchKernelGGL((hex_surface<P, R, HexSurf<P, dbl, true>::EB, NTC, BT, true, false>),
                         dim3(grid[K_SURFACE]), dim3(NTC), 0, st, a.one, a.bt[K_SURFACE], a.segs, a.rk, op, g);
    else
      hipLaunchKernelGGL((hex_surface<P, R, HexSurf<P, dbl>::EB, NTC, BT, false, false>), dim3(grid[K_SURFACE]),
                         dim3(NTC), 0, st, a.one, a.bt[K_SURFACE], a.segs, a.rk, op, g);
  }
}

template <int P, typename R>
static hipError_t hex_rhs_t(const TypeArgs& a, hipStream_t st) {
  constexpr bool dbl = sizeof(R) == 8;
  const int ebs[3] = {HEX_DISU_EB,
                      a.aa ? (a.saa || a.warp ? HexVolLaunch<P, dbl, true, false>::EB : HexVolLaunch<P, dbl, true>::EB)
                           : HexVolLaunch<P, dbl, false>::EB,
                      a.saa ? HexSurf<P, dbl, true>::EB : HexSurf<P, dbl>::EB};
  const bool bt = a.bt[0] && a.bt[1] && a.bt[2] && a.segs;
  int grid[3];
  for (int k = 0; k < 3; ++k) grid[k] = bt ? a.nblk[k] : (a.one.E + ebs[k] - 1) / ebs[k];
  if (bt)
    hex_launch<P, R, true>(a, grid, st);
  else
    hex_launch<P, R, false>(a, grid, st);
  return hipGetLastError();
}

template <int P>
static int hex_surf_elems(bool d, bool saa) {
  return d ? (saa ? HexSurf<P, true, true>::EB : HexSurf<P, true>::EB)
           : (saa ? HexSurf<P, false, true>::EB : HexSurf<P, false>::EB);
}

template <int P>
static int hex_vol_elems(bool d, bool aa, bool saa) {
  if (!aa) return d ? HexVolLaunch<P, true, false>::EB : HexVolLaunch<P, false, false>::EB;
  return d ? (saa ? HexVolLaunch<P, true, true, false>::EB : HexVolLaunch<P, true, true>::EB)
           : (saa ? HexVolLaunch<P, false, true, false>::EB : HexVolLaunch<P, false, true>::EB);
}

int hex_block_elems(int p, int prec, int k, bool aa, bool saa) {
  if (k == K_DISU) return HEX_DISU_EB;
  const bool d = prec == 0;
  if (k == K_SURFACE) {
    switch (p) {
      case 1: return hex_surf_elems<1>(d, saa);
      case 2: return hex_surf_elems<2>(d, saa);
      case 3: return hex_surf_elems<3>(d, saa);
      case 4: return hex_surf_elems<4>(d, saa);
    }
    return 0;
  }
  switch (p) {
    case 1: return hex_vol_elems<1>(d, aa, saa);
    case 2: return hex_vol_elems<2>(d, aa, saa);
    case 3: return hex_vol_elems<3>(d, aa, saa);
    case 4: return hex_vol_elems<4>(d, aa, saa);
  }
  return 0;
}

hipError_t hex_rhs(const TypeArgs& a, int prec, hipStream_t st) {
  const bool d = prec == 0;
  switch (a.p) {
    case 1: return d ? hex_rhs_t<1, double>(a, st) : hex_rhs_t<1, float>(a, st);
    case 2: return d ? hex_rhs_t<2, double>(a, st) : hex_rhs_t<2, float>(a, st);
    case 3: return d ? hex_rhs_t<3, double>(a, st) : hex_rhs_t<3, float>(a, st);
    case 4: return d ? hex_rhs_t<4, double>(a, st) : hex_rhs_t<4, float>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fr
