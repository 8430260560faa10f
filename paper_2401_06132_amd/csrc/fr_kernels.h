// Interface between the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fr_device.h"
#include "fr_host.h"

namespace fr {

// host copies of the 1-D (and triangle) operator factors of one element type
struct HostOps {
  const double *I = nullptr, *D = nullptr, *P = nullptr, *AP = nullptr, *APu = nullptr;
  const double *lb = nullptr, *rb = nullptr, *liftL = nullptr, *liftR = nullptr;
  const Tri* tri = nullptr;
  const RefElem* ref = nullptr;
  const double *x = nullptr, *xq = nullptr;  // GL(n) and GL(m) nodes
};

struct GasHost {
  double gamma, prandtl, mu, pref, beta, tau;
  double rho_ref = 0.0;  // reference density (0: none)
};

// Device constants of the physics.  lin: the element type takes the mass
// flux and the linear energy-flux part from the double-precision L(rho v)
// (affine elements); the energy split needs a reference density.
template <typename R>
inline Gas<R> make_gas(const GasHost& g, bool lin) {
  Gas<R> o;
  o.gamma = R(g.gamma);
  o.gm1 = R(g.gamma - 1.0);
  o.mu = R(g.mu);
  o.muh = R(g.mu * g.gamma / g.prandtl);
  o.pref = R(g.pref);
  o.eref = R(g.pref / (g.gamma - 1.0));
  const double href = g.gamma * g.pref / (g.gamma - 1.0);
  o.href = R(href);
  o.beta = R(g.beta);
  o.tau = R(g.tau);
  o.rho0 = R(g.rho_ref);
  const bool split = lin && g.rho_ref > 0.0;
  o.kap = split ? R(href / g.rho_ref) : R(0);
  o.hc0 = split ? R(0) : R(href);
  return o;
}

// One segment: the elements of one type of one mesh, with every per-mesh
// array the kernels touch.  A launch covers either a single segment (passed
// by value) or a list of segments in device memory addressed through a
// per-workgroup table, so that one launch advances many independent meshes.
struct Seg {
  double* U = nullptr;    // state at the solution points [E][5][N_u] (RK: u_n)
  double* ust = nullptr;  // RK stage state (input of stages 2-4)
  double* acc = nullptr;  // RK accumulator
  double* du = nullptr;   // right-hand side output (plain evaluation)
  void* Uf = nullptr;     // face states (precision R), per mesh: slot s holds
                          // [5][npts(s)] from value 5 po(s), po(s) the slot's
                          // first point (npts: n^2 on quadrilaterals, n(n+1)/2
                          // on triangles); single precision: deviations from
                          // the face base
  float* Ub = nullptr;    // single precision: face bases [slot][5] (value at
                          // the face's first flux point); null in double
  float* fbar = nullptr;  // single precision, tetrahedra and pyramids: the
                          // element's constant transformed flux [E][3][4]
  void* Vf = nullptr;     // normal viscous fluxes, per mesh: [4][npts(s)] from
                          // value 4 po(s)
  void* Rp = nullptr;     // volume divergence [E][5][N_u] (precision R)
  const FaceRec* faces = nullptr;
  const void* fgeo = nullptr;      // [slot][4]: L-side unit normal, own area factor (R)
  const uint8_t* perms = nullptr;  // [perm][n^2]
  const void* met = nullptr;       // [E][10]: J^-1 (row-major), det J   (R)
  const double* detj = nullptr;    // [E]
  double dt = 0.0;                 // RK time step of this mesh
  int32_t E = 0;                   // elements in the segment
  int32_t slot_base = 0;           // first face slot of this type in the mesh
  int32_t po_base = 0;             // first point of that slot in the face arrays
  int32_t nperm = 0;               // face-point permutations in perms (<= MAX_PERMS)
  const void* verts = nullptr;     // curved hexahedra: [E][8][3] element vertices (R)
};

// largest number of distinct face-point permutations a mesh may use (the
// fused kernels stage the table in LDS; box meshes use at most 3)
constexpr int MAX_PERMS = 16;

// workgroup -> (segment, first element of the segment)
struct BlkRef {
  int32_t seg, e0;
};

// kernels of one right-hand side, in launch order
enum { K_DISU = 0, K_VOLUME = 1, K_SURFACE = 2 };

// everything one element type needs for a right-hand-side evaluation
struct TypeArgs {
  int p = 0;
  int stage = 7;        // bit 0: disu, bit 1: volume group, bit 2: interface group
  bool diag = false;    // every element has a diagonal Jacobian
  bool from_ust = false;  // disu/volume read Seg::ust instead of Seg::U
  bool aa = true;       // flux anti-aliasing (false: flux at the solution points)
  bool saa = false;     // surface-flux anti-aliasing (only together with aa)
  bool warp = false;    // curved hexahedra: per-point metrics from Seg::verts
  int rk = -1;          // -1: surface writes du; 0..3: fused classical RK4 stage
  Seg one;              // the segment when bt is null
  const BlkRef* bt[3] = {nullptr, nullptr, nullptr};  // per-kernel workgroup tables
  int nblk[3] = {0, 0, 0};                            // workgroups per kernel
  const Seg* segs = nullptr;                          // device segment list
  const void* dops = nullptr;  // device copy of the prism operator tables (R)
  const HostOps* ops = nullptr;
  const GasHost* gas = nullptr;
};

hipError_t hex_rhs(const TypeArgs& a, int prec, hipStream_t st);
hipError_t prism_rhs(const TypeArgs& a, int prec, hipStream_t st);
// elements per workgroup of kernel k (K_DISU, K_VOLUME, K_SURFACE)
int hex_block_elems(int p, int prec, int k, bool aa, bool saa);
int prism_block_elems(int p, int prec, int k, bool saa);
// size in bytes of the prism operator table for order p and precision prec,
// and its packing into host memory (uploaded once per context)
size_t prism_ops_bytes(int p, int prec);
void prism_ops_pack(const RefElem& r, int prec, void* dst);
// tetrahedra and pyramids (etype 2, 3): dense operator tables (device copy)
// and the kernels
size_t dense_ops_bytes(int etype, int p, int prec);
void dense_ops_pack(const RefElem& r, int prec, void* dst);
hipError_t dense_rhs(int etype, const TypeArgs& a, int prec, hipStream_t st);

// element-wise RK4 stage update: acc += a k; ust = u0 + b k  (first stage:
// acc = u0 + a k)
hipError_t rk_stage(int64_t n, const double* u0, const double* k, double* acc, double* ust, double a, double b,
                    int first, hipStream_t st);

// fills the device's LDS with v (test support: see fr_fill_lds)
hipError_t lds_fill(float v, hipStream_t st);

// Taylor-Green initial state at the solution points of E affine elements:
// x = org_e + J_e xi_u (geo: [E][12] = org, J row-major; ref: [N_u][3])
hipError_t tgv_init(int64_t E, int nu, const double* geo, const double* ref, double gamma, double p0, double* U,
                    hipStream_t st);

// locate this workgroup's segment and first element: BT (batched launch)
// reads the workgroup table, otherwise the single segment passed by value
template <bool BT>
__device__ __forceinline__ Seg seg_of(const Seg& one, const BlkRef* bt, const Seg* segs, int EB, int& e0) {
  if constexpr (BT) {
    const BlkRef b = bt[blockIdx.x];
    e0 = b.e0;
    return segs[b.seg];
  } else {
    e0 = blockIdx.x * EB;
    return one;
  }
}

// write the right-hand side value k of state entry i, or apply the classical
// RK4 stage rk to it:  k1..k4 at u_n, u_n + dt/2 k1, u_n + dt/2 k2, u_n + dt k3;
// u_{n+1} = u_n + dt/6 (k1 + 2 k2 + 2 k3 + k4)
__device__ __forceinline__ void rk_store(const Seg& s, int rk, size_t i, double k) {
  if (rk < 0) {
    s.du[i] = k;
    return;
  }
  const double dt = s.dt;
  if (rk == 3) {
    s.U[i] = s.acc[i] + (dt / 6) * k;
    return;
  }
  const double u = s.U[i];
  const double a = rk == 0 ? dt / 6 : dt / 3;
  const double b = rk == 2 ? dt : dt / 2;
  s.acc[i] = (rk == 0 ? u : s.acc[i]) + a * k;
  s.ust[i] = u + b * k;
}

// rk_store for the NL values a thread holds: item it = tid + k NT of a
// workgroup covering elements [e0, e0 + elems) with per elements values,
// valid while it < total and its element < E.  In an RK stage every state
// load is issued before the first store.
template <int NL, int NT>
__device__ __forceinline__ void rk_store_block(const Seg& s, int rk, int e0, int E, int per, int total, int tid,
                                               const double (&val)[NL]) {
  size_t idx[NL];
  bool ok[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int it = tid + k * NT;
    ok[k] = it < total && e0 + it / per < E;
    idx[k] = ok[k] ? (size_t)e0 * per + it : 0;
  }
  if (rk < 0) {
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (ok[k]) s.du[idx[k]] = val[k];
    return;
  }
  const double dt = s.dt;
  if (rk == 3) {
    double a[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) a[k] = s.acc[idx[k]];
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (ok[k]) s.U[idx[k]] = a[k] + (dt / 6) * val[k];
    return;
  }
  const double ca = rk == 0 ? dt / 6 : dt / 3;
  const double cb = rk == 2 ? dt : dt / 2;
  double u[NL], a[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    u[k] = s.U[idx[k]];
    a[k] = rk == 0 ? u[k] : s.acc[idx[k]];
  }
#pragma unroll
  for (int k = 0; k < NL; ++k)
    if (ok[k]) {
      s.acc[idx[k]] = a[k] + ca * val[k];
      s.ust[idx[k]] = u[k] + cb * val[k];
    }
}

}  // namespace fr
