// Plain (unfused, dense-operator, FP64) path: host-side state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fr_device.h"
#include "fr_host.h"

namespace fr {

// dense composite operators of section 2.2 for one element type (row-major)
struct PlainOps {
  int nu = 0, nf = 0, nq = 0;
  std::vector<double> M0;  // nf x nu                 disu, gradcoru_fpts
  std::vector<double> G1;  // 3nu x nu   M4 - M6 M0   tgradpcoru
  std::vector<double> M6;  // 3nu x nf                tgradcoru
  std::vector<double> M7;  // nq x nu                 qptsu, gradcoru_qpts
  std::vector<double> K;   // nu x 3nq   (M1 - M3 M2) M9   tdivpcorf
  std::vector<double> M3;  // nu x nf                 tdivtconf
  std::vector<double> LV;  // nu x 3nu   [Lv_0 | Lv_1 | Lv_2]: the divergence L(rho v)
                           //            of the linear energy-flux part
};

// per own flux point: the paired point and which side is L
struct PlainFace {
  int32_t nbr_elem;
  int16_t nbr_fpt;
  int8_t nbr_type;
  int8_t is_left;
};

struct PlainTypes {
  int64_t E[NTYPES];      // elements per type
  int64_t off_f[NTYPES];  // offset of each type block in the flux-point arrays (5 values per point)
  int64_t nf[NTYPES];     // flux points per element
  int64_t f0[NTYPES];     // first flat flux point of each type (types in order)
};

// element type of flat flux point i
__host__ __device__ inline int plain_type_of(const PlainTypes& ty, int64_t i) {
  int t = 0;
  for (int u = 1; u < NTYPES; ++u)
    if (i >= ty.f0[u]) t = u;
  return t;
}

struct PlainCtx {
  PlainOps ops[NTYPES];
  PlainTypes ty;
  Gas<double> gas;
  double beta = 0.5, eref = 0.0, rho0 = 0.0;
  int64_t state_off[NTYPES] = {};
  void* blas = nullptr;
  // device
  double *dM0[NTYPES] = {}, *dG1[NTYPES] = {}, *dM6[NTYPES] = {};
  double *dM7[NTYPES] = {}, *dK[NTYPES] = {}, *dM3[NTYPES] = {}, *dLV[NTYPES] = {};
  double *W = nullptr, *Uf = nullptr, *Cf = nullptr, *Q = nullptr, *Qf = nullptr, *Uq = nullptr, *Qq = nullptr;
  double *Df = nullptr, *fgeo = nullptr;
  double *jinv[NTYPES] = {}, *detj[NTYPES] = {};
  PlainFace* faces = nullptr;
};

void build_plain_ops(const RefElem& r, PlainOps& o);
hipError_t plain_rhs(PlainCtx& P, const double* U, double* du, hipStream_t st);
bool plain_create_handle(void** h);
void plain_destroy_handle(void* h);

}  // namespace fr
