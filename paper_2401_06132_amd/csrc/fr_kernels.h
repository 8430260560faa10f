// Interface between the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fr_device.h"
#include "fr_host.h"

namespace fr {

// host copies of the 1-D (and triangle) operator factors of one element type
struct HostOps {
  const double *I = nullptr, *D = nullptr, *P = nullptr, *AP = nullptr;
  const double *lb = nullptr, *rb = nullptr, *liftL = nullptr, *liftR = nullptr;
  const Tri* tri = nullptr;
  const RefElem* ref = nullptr;
};

struct GasHost {
  double gamma, prandtl, mu, pref, beta, tau;
};

// everything one element type needs for a right-hand-side evaluation
struct TypeArgs {
  int p = 0;
  int64_t E = 0;          // elements of this type
  int64_t slot_base = 0;  // first face slot of this type
  int stage = 7;          // bit 0: disu, bit 1: volume group, bit 2: interface group
  bool diag = false;      // every element of this type has a diagonal Jacobian
  const double* U = nullptr;  // state of this type (E x 5 x N_u)
  double* du = nullptr;
  void* Uf = nullptr;  // face states   [slot][5][n^2]   (precision R)
  void* Vf = nullptr;  // normal viscous fluxes [slot][4][n^2]
  void* Rp = nullptr;  // volume divergence of this type (E x 5 x N_u, precision R)
  const FaceRec* faces = nullptr;
  const void* fgeo = nullptr;     // [slot][4]: L-side unit normal, area factor (R)
  const uint8_t* perms = nullptr; // [perm][n^2]
  const void* met = nullptr;      // [E][10]: J^-1 (row-major), det J   (R)
  const double* detj = nullptr;   // [E]
  const void* dops = nullptr;     // device copy of the prism operator tables (R)
  const HostOps* ops = nullptr;
  const GasHost* gas = nullptr;
};

hipError_t hex_rhs(const TypeArgs& a, int prec, hipStream_t st);
hipError_t prism_rhs(const TypeArgs& a, int prec, hipStream_t st);
// size in bytes of the prism operator table for order p and precision prec,
// and its packing into host memory (uploaded once per context)
size_t prism_ops_bytes(int p, int prec);
void prism_ops_pack(const RefElem& r, int prec, void* dst);

// element-wise RK4 stage update: acc += a k; ust = u0 + b k  (first stage:
// acc = u0 + a k)
hipError_t rk_stage(int64_t n, const double* u0, const double* k, double* acc, double* ust, double a, double b,
                    int first, hipStream_t st);

}  // namespace fr
