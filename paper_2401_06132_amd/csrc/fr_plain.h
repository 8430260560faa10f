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
};

// per own flux point: the paired point and which side is L
struct PlainFace {
  int32_t nbr_elem;
  int16_t nbr_fpt;
  int8_t nbr_type;
  int8_t is_left;
};

struct PlainTypes {
  int64_t E[2];      // elements per type
  int64_t off_f[2];  // offset of each type block in the flux-point arrays (5 values per point)
  int64_t nf[2];     // flux points per element
};

struct PlainCtx {
  PlainOps ops[2];
  PlainTypes ty;
  Gas<double> gas;
  double beta = 0.5, eref = 0.0;
  int64_t state_off[2] = {0, 0};
  void* blas = nullptr;
  // device
  double *dM0[2] = {nullptr, nullptr}, *dG1[2] = {nullptr, nullptr}, *dM6[2] = {nullptr, nullptr};
  double *dM7[2] = {nullptr, nullptr}, *dK[2] = {nullptr, nullptr}, *dM3[2] = {nullptr, nullptr};
  double *W = nullptr, *Uf = nullptr, *Cf = nullptr, *Q = nullptr, *Qf = nullptr, *Uq = nullptr, *Qq = nullptr;
  double *Df = nullptr, *fgeo = nullptr;
  double *jinv[2] = {nullptr, nullptr}, *detj[2] = {nullptr, nullptr};
  PlainFace* faces = nullptr;
};

void build_plain_ops(const RefElem& r, PlainOps& o);
hipError_t plain_rhs(PlainCtx& P, const double* U, double* du, hipStream_t st);
bool plain_create_handle(void** h);
void plain_destroy_handle(void* h);

}  // namespace fr
