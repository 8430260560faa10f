// C ABI implementation (host): context, mesh, device buffers and the
// right-hand-side / RK4 drivers.  See include/fr.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_host.h"
#include "fr_kernels.h"
#include "fr_plain.h"

// Per-call work buffers of the fused form: face values Uf [slot][5][points],
// transformed face fluxes Vf [slot][4][points], residual partials Rp (state
// layout) and, in single precision, the face bases Ub [slot][5] and the
// constant transformed flux fbar [E][12] of the dense types.  None needs to
// start at any particular value: every call writes each before reading it.
struct Work {
  enum { UF, VF, RP, UB, FBAR, N = FBAR + fr::NTYPES };
  void* ptr[N] = {};
};

struct fr_ctx {
  fr_physics ph;
  hipStream_t st = nullptr;
  std::string err;
  bool mesh_ok = false, dev_ok = false;
  int p = 0;
  fr::RefElem ref[fr::NTYPES];
  bool has[fr::NTYPES] = {};
  fr::Mesh M;
  int64_t off[fr::NTYPES] = {}, n_state = 0;
  bool diag[fr::NTYPES] = {};  // all Jacobians of the type are diagonal
  fr::HostOps hops[fr::NTYPES];
  fr::GasHost gas;
  // device buffers
  double* d_state = nullptr;  // internal state
  double* d_rk = nullptr;     // RK buffers: stage state, accumulator (+ stage derivative, plain form)
  void* d_fgeo = nullptr;
  fr::FaceRec* d_faces = nullptr;
  uint8_t* d_perms = nullptr;
  void* d_met[fr::NTYPES] = {};
  double* d_detj[fr::NTYPES] = {};
  void* d_pops = nullptr;  // prism triangle tables
  void* d_dops[fr::NTYPES] = {};  // dense operator tables (tetrahedra, pyramids)
  void* d_verts[2] = {nullptr, nullptr};  // curved meshes: element vertices [E][nv][3]
  fr::PlainCtx* plain = nullptr;  // unfused comparison path
  Work w;  // per-call work buffers of the fused form (allocated on first use)
  bool work_ok = false;
};

// Work buffers of fr_rhs_noalloc: one copy of this array per GPU, held from
// the library's load until the process ends.  In host code the name is a
// host-side stand-in; the device address comes from hipGetSymbolAddress, once
// per device (scratch_on_device below), and only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[FR_NOALLOC_MAX_BYTES];

namespace {

fr_status fail(fr_ctx* c, fr_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(c, FR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t rsize(const fr_ctx* c) { return c->ph.prec == FR_PREC_FP64 ? 8 : 4; }

template <typename T>
void put(std::vector<unsigned char>& buf, const std::vector<double>& v, size_t n) {
  buf.resize(n * sizeof(T));
  T* p = reinterpret_cast<T*>(buf.data());
  for (size_t i = 0; i < n; ++i) p[i] = T(v[i]);
}

void to_real(const fr_ctx* c, const std::vector<double>& v, std::vector<unsigned char>& buf) {
  if (rsize(c) == 8)
    put<double>(buf, v, v.size());
  else
    put<float>(buf, v, v.size());
}

fr_status setup_plain(fr_ctx* c) {
  const fr::Mesh& M = c->M;
  fr::PlainCtx* P = new (std::nothrow) fr::PlainCtx();
  if (!P) return fail(c, FR_ENOMEM, "host allocation");
  c->plain = P;
  if (!fr::plain_create_handle(&P->blas)) return fail(c, FR_EDEVICE, "rocblas_create_handle failed");
  P->beta = c->ph.ldg_beta;
  P->eref = c->ph.pref / (c->ph.gamma - 1.0);
  // the plain path takes the same reference state and energy-flux split as
  // the fused kernels (its mass flux stays in the dense products)
  P->rho0 = c->gas.rho_ref;
  P->gas = fr::make_gas<double>(c->gas, true);
  int64_t nftot = 0, nqmax = 0;
  for (int t = 0; t < fr::NTYPES; ++t) {
    P->ty.E[t] = M.nel[t];
    P->ty.nf[t] = c->ref[t].nf;
    P->ty.off_f[t] = 5 * nftot;
    P->ty.f0[t] = nftot;
    nftot += M.nel[t] * c->ref[t].nf;
    P->state_off[t] = c->off[t];
    if (!c->has[t]) continue;
    fr::build_plain_ops(c->ref[t], P->ops[t]);
    const fr::PlainOps& o = P->ops[t];
    nqmax = std::max<int64_t>(nqmax, M.nel[t] * o.nq);
    struct {
      double** d;
      const std::vector<double>* h;
    } up[] = {{&P->dM0[t], &o.M0}, {&P->dG1[t], &o.G1}, {&P->dM6[t], &o.M6}, {&P->dM7[t], &o.M7},
              {&P->dK[t], &o.K},   {&P->dM3[t], &o.M3},  {&P->dLV[t], &o.LV}};
    for (auto& x : up) {
      HIPCHK(hipMalloc(x.d, sizeof(double) * x.h->size()));
      HIPCHK(hipMemcpy(*x.d, x.h->data(), sizeof(double) * x.h->size(), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMalloc(&P->jinv[t], sizeof(double) * 9 * M.nel[t]));
    HIPCHK(hipMemcpy(P->jinv[t], M.jinv[t].data(), sizeof(double) * 9 * M.nel[t], hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&P->detj[t], sizeof(double) * M.nel[t]));
    HIPCHK(hipMemcpy(P->detj[t], M.detj[t].data(), sizeof(double) * M.nel[t], hipMemcpyHostToDevice));
  }
  // per flux point neighbour records and L-side normals (the paper's n^(f))
  std::vector<fr::PlainFace> pf(nftot);
  std::vector<double> geo(4 * nftot);
  int64_t base[fr::NTYPES];
  for (int t = 0; t < fr::NTYPES; ++t) base[t] = P->ty.f0[t];
  auto type_of = [&](int64_t s) {
    int t = 0;
    for (int u = 1; u < fr::NTYPES; ++u)
      if (M.nel[u] > 0 && s >= M.slot_base[u]) t = u;
    return t;
  };
  for (int64_t s = 0; s < M.nslots; ++s) {
    int t = type_of(s);
    int64_t e = (s - M.slot_base[t]) / fr::kFacesOf[t];
    int f = int((s - M.slot_base[t]) % fr::kFacesOf[t]);
    int64_t o = M.nbr_slot[s];
    int to = type_of(o);
    int64_t eo = (o - M.slot_base[to]) / fr::kFacesOf[to];
    int fo = int((o - M.slot_base[to]) % fr::kFacesOf[to]);
    const std::vector<int>& pm = M.perms[M.perm_id[s]];
    for (int q = 0; q < c->ref[t].face_npts[f]; ++q) {
      int64_t i = base[t] + e * c->ref[t].nf + c->ref[t].face_start[f] + q;
      pf[i].nbr_elem = (int32_t)eo;
      pf[i].nbr_fpt = (int16_t)(c->ref[to].face_start[fo] + pm[q]);
      pf[i].nbr_type = (int8_t)to;
      pf[i].is_left = (int8_t)M.is_left[s];
      for (int d = 0; d < 3; ++d) geo[4 * i + d] = M.nrm[3 * s + d];
      geo[4 * i + 3] = M.mag[s];
    }
  }
  HIPCHK(hipMalloc(&P->faces, sizeof(fr::PlainFace) * nftot));
  HIPCHK(hipMemcpy(P->faces, pf.data(), sizeof(fr::PlainFace) * nftot, hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&P->fgeo, sizeof(double) * 4 * nftot));
  HIPCHK(hipMemcpy(P->fgeo, geo.data(), sizeof(double) * 4 * nftot, hipMemcpyHostToDevice));
  const size_t d8 = sizeof(double);
  HIPCHK(hipMalloc(&P->W, d8 * c->n_state));
  HIPCHK(hipMalloc(&P->Q, d8 * 3 * c->n_state));
  HIPCHK(hipMalloc(&P->Uf, d8 * 5 * nftot));
  HIPCHK(hipMalloc(&P->Cf, d8 * 5 * nftot));
  HIPCHK(hipMalloc(&P->Df, d8 * 5 * nftot));
  HIPCHK(hipMalloc(&P->Qf, d8 * 15 * nftot));
  HIPCHK(hipMalloc(&P->Uq, d8 * 5 * nqmax));
  HIPCHK(hipMalloc(&P->Qq, d8 * 15 * nqmax));
  return FR_OK;
}

void free_plain(fr_ctx* c) {
  fr::PlainCtx* P = c->plain;
  if (!P) return;
  void* bufs[] = {P->W, P->Uf, P->Cf, P->Q, P->Qf, P->Uq, P->Qq, P->Df, P->fgeo, P->faces};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int t = 0; t < fr::NTYPES; ++t) {
    void* tb[] = {P->dM0[t], P->dG1[t], P->dM6[t], P->dM7[t], P->dK[t], P->dM3[t], P->dLV[t], P->jinv[t], P->detj[t]};
    for (void* b : tb)
      if (b) (void)hipFree(b);
  }
  fr::plain_destroy_handle(P->blas);
  delete P;
  c->plain = nullptr;
}

fr_status ensure_device(fr_ctx* c) {
  if (c->dev_ok) return FR_OK;
  if (!c->mesh_ok) return fail(c, FR_ESTATE, "no mesh");
  if (c->ph.form == FR_FORM_PLAIN) {
    HIPCHK(hipMalloc(&c->d_state, sizeof(double) * c->n_state));
    HIPCHK(hipMemsetAsync(c->d_state, 0, sizeof(double) * c->n_state, c->st));
    HIPCHK(hipMalloc(&c->d_rk, sizeof(double) * c->n_state * 3));
    fr_status s = setup_plain(c);
    if (s != FR_OK) return s;
    c->dev_ok = true;
    return FR_OK;
  }
  const fr::Mesh& M = c->M;
  const int nfp = (c->p + 1) * (c->p + 1);
  const int64_t S = M.nslots;
  HIPCHK(hipMalloc(&c->d_state, sizeof(double) * c->n_state));
  HIPCHK(hipMemsetAsync(c->d_state, 0, sizeof(double) * c->n_state, c->st));
  HIPCHK(hipMalloc(&c->d_rk, sizeof(double) * c->n_state * 2));  // stage state, accumulator
  // faces
  std::vector<fr::FaceRec> fr(S);
  std::vector<double> geo(4 * S);
  for (int64_t s = 0; s < S; ++s) {
    fr[s].nbr = (int32_t)M.nbr_slot[s];
    fr[s].info = (M.perm_id[s] << 1) | (M.is_left[s] ? 1 : 0);
    fr[s].npo = (int32_t)M.slot_po[M.nbr_slot[s]];
    fr[s].pad = 0;
    for (int d = 0; d < 3; ++d) geo[4 * s + d] = M.nrm[3 * s + d];
    geo[4 * s + 3] = M.mag[s];
  }
  HIPCHK(hipMalloc(&c->d_faces, sizeof(fr::FaceRec) * S));
  HIPCHK(hipMemcpyAsync(c->d_faces, fr.data(), sizeof(fr::FaceRec) * S, hipMemcpyHostToDevice, c->st));
  std::vector<unsigned char> buf;
  to_real(c, geo, buf);
  HIPCHK(hipMalloc(&c->d_fgeo, buf.size()));
  HIPCHK(hipMemcpyAsync(c->d_fgeo, buf.data(), buf.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  std::vector<uint8_t> perms(M.perms.size() * nfp, 0);
  for (size_t k = 0; k < M.perms.size(); ++k)
    for (size_t r = 0; r < M.perms[k].size(); ++r) perms[k * nfp + r] = (uint8_t)M.perms[k][r];
  HIPCHK(hipMalloc(&c->d_perms, perms.size()));
  HIPCHK(hipMemcpy(c->d_perms, perms.data(), perms.size(), hipMemcpyHostToDevice));
  for (int t = 0; t < fr::NTYPES; ++t) {
    if (!c->has[t]) continue;
    const int64_t E = M.nel[t];
    std::vector<double> met(10 * E);
    for (int64_t e = 0; e < E; ++e) {
      for (int k = 0; k < 9; ++k) met[10 * e + k] = M.jinv[t][9 * e + k];
      met[10 * e + 9] = M.detj[t][e];
    }
    to_real(c, met, buf);
    HIPCHK(hipMalloc(&c->d_met[t], buf.size()));
    HIPCHK(hipMemcpy(c->d_met[t], buf.data(), buf.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&c->d_detj[t], sizeof(double) * E));
    HIPCHK(hipMemcpy(c->d_detj[t], M.detj[t].data(), sizeof(double) * E, hipMemcpyHostToDevice));
  }
  if (c->has[1]) {
    size_t nb = fr::prism_ops_bytes(c->p, c->ph.prec);
    std::vector<unsigned char> pb(nb);
    fr::prism_ops_pack(c->ref[1], c->ph.prec, pb.data());
    HIPCHK(hipMalloc(&c->d_pops, nb));
    HIPCHK(hipMemcpy(c->d_pops, pb.data(), nb, hipMemcpyHostToDevice));
  }
  if (M.curved)
    for (int t = 0; t < 2; ++t) {
      if (!c->has[t]) continue;
      to_real(c, M.verts[t], buf);
      HIPCHK(hipMalloc(&c->d_verts[t], buf.size()));
      HIPCHK(hipMemcpy(c->d_verts[t], buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
  for (int t = 2; t < fr::NTYPES; ++t) {
    if (!c->has[t]) continue;
    size_t nb = fr::dense_ops_bytes(t, c->p, c->ph.prec);
    std::vector<unsigned char> pb(nb);
    fr::dense_ops_pack(c->ref[t], c->ph.prec, pb.data());
    HIPCHK(hipMalloc(&c->d_dops[t], nb));
    HIPCHK(hipMemcpy(c->d_dops[t], pb.data(), nb, hipMemcpyHostToDevice));
  }
  c->dev_ok = true;
  return FR_OK;
}

// Sizes in bytes of the fused form's per-call work buffers (slot k of
// Work::ptr): face values, transformed face fluxes, residual partials and,
// in single precision, the face bases and the dense types' constant
// transformed flux.  Returns the total with every buffer 256-byte aligned.
int64_t work_bytes(const fr_ctx* c, int64_t bytes[Work::N]) {
  const int64_t rs = (int64_t)rsize(c), S = c->M.nslots, NP = c->M.npts;
  bytes[Work::UF] = rs * 5 * NP;
  bytes[Work::VF] = rs * 4 * NP;
  bytes[Work::RP] = rs * c->n_state;
  bytes[Work::UB] = rs == 4 ? (int64_t)sizeof(float) * S * 5 : 0;
  for (int t = 0; t < fr::NTYPES; ++t)
    bytes[Work::FBAR + t] = rs == 4 && t >= 2 ? (int64_t)sizeof(float) * 12 * c->M.nel[t] : 0;
  int64_t tot = 0;
  for (int k = 0; k < Work::N; ++k) tot += (bytes[k] + 255) / 256 * 256;
  return tot;
}

// the device address of `scratch` on the current device, looked up on the
// first call there and kept per device ordinal
hipError_t scratch_on_device(void** out) {
  static std::mutex mu;
  static void* addr[256] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

// the context's own work buffers, allocated on first use
fr_status ensure_work(fr_ctx* c) {
  if (c->work_ok) return FR_OK;
  int64_t b[Work::N];
  work_bytes(c, b);
  for (int k = 0; k < Work::N; ++k)
    if (b[k] > 0) HIPCHK(hipMalloc(&c->w.ptr[k], (size_t)b[k]));
  c->work_ok = true;
  return FR_OK;
}

// the segment of element type t: caller's u/du for a plain evaluation, the
// internal state and RK buffers otherwise; work buffers from w
fr::Seg seg_of_type(fr_ctx* c, int t, const double* u, double* du, const Work& w) {
  fr::Seg s;
  const int64_t o = c->off[t];
  s.U = const_cast<double*>(u ? u : c->d_state) + o;
  s.du = du ? du + o : nullptr;
  s.ust = c->d_rk + o;
  s.acc = c->d_rk + c->n_state + o;
  s.Uf = w.ptr[Work::UF];
  s.Ub = (float*)w.ptr[Work::UB];
  s.Vf = w.ptr[Work::VF];
  s.Rp = (char*)w.ptr[Work::RP] + rsize(c) * o;
  s.faces = c->d_faces;
  s.fgeo = c->d_fgeo;
  s.perms = c->d_perms;
  s.met = c->d_met[t];
  s.detj = c->d_detj[t];
  s.E = (int32_t)c->M.nel[t];
  s.slot_base = (int32_t)c->M.slot_base[t];
  s.po_base = c->M.nel[t] > 0 ? (int32_t)c->M.slot_po[c->M.slot_base[t]] : 0;
  s.nperm = (int32_t)c->M.perms.size();
  s.verts = t < 2 ? c->d_verts[t] : nullptr;
  s.fbar = (float*)w.ptr[Work::FBAR + t];
  return s;
}

fr::TypeArgs type_args(fr_ctx* c, int t, const fr::Seg& s, int stage) {
  fr::TypeArgs a;
  a.p = c->p;
  a.stage = stage;
  a.diag = c->diag[t];
  a.one = s;
  a.dops = t >= 2 ? c->d_dops[t] : c->d_pops;
  a.warp = c->M.curved && t < 2;
  a.ops = &c->hops[t];
  a.gas = &c->gas;
  return a;
}

// one right-hand side (rk < 0: du = R(u)) or one fused RK4 stage rk on the
// internal state (u, du unused); work buffers from w, else the context's own
fr_status launch_rhs(fr_ctx* c, const double* u, double* du, int mask = 7, int rk = -1, double dt = 0.0,
                     const Work* w = nullptr) {
  if (c->ph.form == FR_FORM_PLAIN) {
    hipError_t e = fr::plain_rhs(*c->plain, u, du, c->st);
    if (e != hipSuccess) return fail(c, FR_EDEVICE, std::string("plain path: ") + hipGetErrorString(e));
    return FR_OK;
  }
  if (!w) {
    fr_status s = ensure_work(c);
    if (s != FR_OK) return s;
    w = &c->w;
  }
  for (int stage = 1; stage <= 4; stage <<= 1)
    if (mask & stage)
    for (int t = 0; t < fr::NTYPES; ++t) {
      if (!c->has[t]) continue;
      fr::TypeArgs a = type_args(c, t, seg_of_type(c, t, rk < 0 ? u : nullptr, rk < 0 ? du : nullptr, *w), stage);
      a.one.dt = dt;
      a.rk = rk;
      a.from_ust = rk > 0;
      a.aa = c->ph.flux_aa != 0;
      a.saa = c->ph.surface_aa != 0;
      hipError_t e = t == 0   ? fr::hex_rhs(a, c->ph.prec, c->st)
                     : t == 1 ? fr::prism_rhs(a, c->ph.prec, c->st)
                              : fr::dense_rhs(t, a, c->ph.prec, c->st);
      if (e != hipSuccess) return fail(c, FR_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
  return FR_OK;
}

// operator pointers, per-type flags and the state layout of a new mesh
fr_status setup_ctx_mesh(fr_ctx* c) {
  for (int t = 0; t < fr::NTYPES; ++t) {
    c->has[t] = c->M.nel[t] > 0;
    const fr::RefElem& r = c->ref[t];
    fr::HostOps& h = c->hops[t];
    h.I = r.line.I.data();
    h.D = r.line.D.data();
    h.P = r.line.P.data();
    h.AP = r.line.AP.data();
    h.APu = r.line.APu.data();
    h.lb = r.line.lb.data();
    h.rb = r.line.rb.data();
    h.liftL = r.line.liftL.data();
    h.liftR = r.line.liftR.data();
    h.tri = &r.tri;
    h.ref = &r;
    h.x = r.line.x.data();
    h.xq = r.line.xq.data();
  }
  for (int t = 0; t < fr::NTYPES; ++t) {
    bool d = c->has[t] && !c->M.curved;
    for (int64_t e = 0; e < c->M.nel[t] && d; ++e) {
      const double* A = &c->M.jac[t][9 * e];
      d = A[1] == 0 && A[2] == 0 && A[3] == 0 && A[5] == 0 && A[6] == 0 && A[7] == 0;
    }
    c->diag[t] = d;
  }
  c->off[0] = 0;
  for (int t = 1; t < fr::NTYPES; ++t) c->off[t] = c->off[t - 1] + c->M.nel[t - 1] * 5 * c->ref[t - 1].nu;
  c->n_state = c->off[fr::NTYPES - 1] + c->M.nel[fr::NTYPES - 1] * 5 * c->ref[fr::NTYPES - 1].nu;
  // the kernels index slots, face points and elements with 32-bit integers
  if (c->M.nslots >= (int64_t)1 << 31 || c->M.npts >= (int64_t)1 << 31)
    return fail(c, FR_EINVAL, "mesh too large: face slots or face points exceed 2^31");
  c->mesh_ok = true;
  return FR_OK;
}

}  // namespace

extern "C" {

void fr_physics_default(fr_physics* ph) {
  if (!ph) return;
  ph->gamma = 1.4;
  ph->prandtl = 0.71;
  ph->mu = 1.0 / 1600.0;
  ph->ldg_beta = 0.5;
  ph->ldg_tau = 0.1;
  ph->pref = 0.0;
  ph->rho_ref = 0.0;
  ph->prec = FR_PREC_FP64;
  ph->form = FR_FORM_FUSED;
  ph->flux_aa = 1;
  ph->surface_aa = 0;
}

fr_status fr_create(const fr_physics* ph, void* stream, fr_ctx** out) {
  if (!ph || !out) return FR_EINVAL;
  *out = nullptr;
  if (!(ph->gamma > 1.0) || !(ph->prandtl > 0.0) || !(ph->mu >= 0.0) || !(ph->ldg_tau >= 0.0) ||
      !std::isfinite(ph->ldg_beta) || !std::isfinite(ph->pref) || !(ph->rho_ref >= 0.0) ||
      !std::isfinite(ph->rho_ref) || ph->prec < 0 || ph->prec > 1 || ph->form < 0 ||
      ph->form > 1 || ph->flux_aa < 0 || ph->flux_aa > 1 || ph->surface_aa < 0 || ph->surface_aa > 1)
    return FR_EINVAL;
  if (ph->form == FR_FORM_PLAIN && ph->prec != FR_PREC_FP64) return FR_EUNSUPPORTED;
  if (ph->form == FR_FORM_PLAIN && (!ph->flux_aa || ph->surface_aa)) return FR_EUNSUPPORTED;
  if (ph->surface_aa && !ph->flux_aa) return FR_EUNSUPPORTED;
  fr_ctx* c = new (std::nothrow) fr_ctx();
  if (!c) return FR_ENOMEM;
  c->ph = *ph;
  c->st = (hipStream_t)stream;
  c->gas = {ph->gamma, ph->prandtl, ph->mu, ph->pref, ph->ldg_beta, ph->ldg_tau, ph->rho_ref};
  *out = c;
  return FR_OK;
}

fr_status fr_mesh_box(fr_ctx* c, int nx, int ny, int nz, double lo, double hi, int p, int kind) {
  if (!c) return FR_EINVAL;
  if (c->mesh_ok) return fail(c, FR_ESTATE, "mesh already built");
  if (nx < 1 || ny < 1 || nz < 1 || !(hi > lo) || kind < 0 || kind >= fr::kNumKinds)
    return fail(c, FR_EINVAL, "bad mesh size");
  if (p < 1 || p > 4) return fail(c, FR_EUNSUPPORTED, "order must be 1..4");
  if ((kind == FR_MESH_HEX_PYR_TET || kind == FR_MESH_HEX_PRISM_PYR_TET) && nz < 3)
    return fail(c, FR_EINVAL, "meshes with transition cells: nz >= 3");
  if (fr::kind_dense(kind) && c->ph.surface_aa)
    return fail(c, FR_EUNSUPPORTED, "tetrahedra and pyramids: no surface-flux anti-aliasing");
  if (fr::kind_curved(kind) && (c->ph.form != FR_FORM_FUSED || !c->ph.flux_aa || c->ph.surface_aa))
    return fail(c, FR_EUNSUPPORTED, "curved elements: fused form with flux anti-aliasing only");
  try {
    c->p = p;
    for (int t = 0; t < fr::NTYPES; ++t) fr::build_ref(t, p, c->ref[t]);
    const fr::RefElem* refs[fr::NTYPES] = {&c->ref[0], &c->ref[1], &c->ref[2], &c->ref[3]};
    std::string e = fr::build_box_mesh(nx, ny, nz, lo, hi, p, kind, refs, c->M);
    if (!e.empty()) return fail(c, FR_EINVAL, e);
    if ((int)c->M.perms.size() > fr::MAX_PERMS) return fail(c, FR_EUNSUPPORTED, "too many face permutations");
    if (c->ph.surface_aa && !fr::prism_tri_faces_aligned(c->M))
      return fail(c, FR_EUNSUPPORTED, "surface-flux anti-aliasing needs aligned prism triangle faces");
  } catch (const std::exception& ex) {
    return fail(c, FR_EINVAL, ex.what());
  }
  return setup_ctx_mesh(c);
}

fr_status fr_mesh_elements(fr_ctx* c, int p, const int64_t* n_elem, const double* const* verts,
                           const double* period) {
  if (!c) return FR_EINVAL;
  if (c->mesh_ok) return fail(c, FR_ESTATE, "mesh already built");
  if (!n_elem || !verts) return fail(c, FR_EINVAL, "null argument");
  if (p < 1 || p > 4) return fail(c, FR_EUNSUPPORTED, "order must be 1..4");
  int64_t total = 0;
  for (int t = 0; t < fr::NTYPES; ++t) {
    if (n_elem[t] < 0 || (n_elem[t] > 0 && !verts[t])) return fail(c, FR_EINVAL, "bad element count or vertex array");
    if (n_elem[t] > ((int64_t)1 << 30)) return fail(c, FR_EINVAL, "too many elements");
    total += n_elem[t];
  }
  if (total == 0) return fail(c, FR_EINVAL, "no elements");
  if ((n_elem[2] > 0 || n_elem[3] > 0) && c->ph.surface_aa)
    return fail(c, FR_EUNSUPPORTED, "tetrahedra and pyramids: no surface-flux anti-aliasing");
  try {
    c->p = p;
    for (int t = 0; t < fr::NTYPES; ++t) fr::build_ref(t, p, c->ref[t]);
    const fr::RefElem* refs[fr::NTYPES] = {&c->ref[0], &c->ref[1], &c->ref[2], &c->ref[3]};
    std::string e = fr::build_element_mesh(p, n_elem, verts, period, refs, c->M);
    if (!e.empty()) return fail(c, FR_EINVAL, e);
    if ((int)c->M.perms.size() > fr::MAX_PERMS) return fail(c, FR_EUNSUPPORTED, "too many face permutations");
    if (c->ph.surface_aa && !fr::prism_tri_faces_aligned(c->M))
      return fail(c, FR_EUNSUPPORTED, "surface-flux anti-aliasing needs aligned prism triangle faces");
  } catch (const std::exception& ex) {
    return fail(c, FR_EINVAL, ex.what());
  }
  return setup_ctx_mesh(c);
}

fr_status fr_layout(const fr_ctx* c, int64_t* nh, int64_t* np, int64_t* ns) {
  if (!c) return FR_EINVAL;
  if (!c->mesh_ok) return FR_ESTATE;
  if (nh) *nh = c->M.nel[0];
  if (np) *np = c->M.nel[1];
  if (ns) *ns = c->n_state;
  return FR_OK;
}

fr_status fr_type_count(const fr_ctx* c, int etype, int64_t* n_elem) {
  if (!c || !n_elem || etype < 0 || etype >= fr::NTYPES) return FR_EINVAL;
  if (!c->mesh_ok) return FR_ESTATE;
  *n_elem = c->M.nel[etype];
  return FR_OK;
}

fr_status fr_upts_coords(const fr_ctx* c, double* xyz) {
  if (!c || !xyz) return FR_EINVAL;
  if (!c->mesh_ok) return FR_ESTATE;
  int64_t k = 0;
  for (int t = 0; t < fr::NTYPES; ++t) {
    const fr::RefElem& r = c->ref[t];
    for (int64_t e = 0; e < c->M.nel[t]; ++e) {
      for (int u = 0; u < r.nu; ++u) fr::map_point(c->M, t, e, &r.upts[3 * u], &xyz[3 * (k + u)]);
      k += r.nu;
    }
  }
  return FR_OK;
}

fr_status fr_rhs(fr_ctx* c, const double* u, double* du) {
  if (!c) return FR_EINVAL;
  if (!u || !du) return fail(c, FR_EINVAL, "null buffer");
  if (u == du) return fail(c, FR_EINVAL, "u and du must not alias");
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  return launch_rhs(c, u, du);
}

fr_status fr_rhs_noalloc(fr_ctx* c, const double* u, double* du) {
  if (!c) return FR_EINVAL;
  if (!u || !du) return fail(c, FR_EINVAL, "null buffer");
  if (u == du) return fail(c, FR_EINVAL, "u and du must not alias");
  if (!c->mesh_ok) return fail(c, FR_ESTATE, "no mesh");
  if (c->ph.form != FR_FORM_FUSED)
    return fail(c, FR_EUNSUPPORTED, "fr_rhs_noalloc: the plain form keeps its work buffers in the context");
  int64_t b[Work::N];
  const int64_t need = work_bytes(c, b);
  if (need > (int64_t)FR_NOALLOC_MAX_BYTES)
    return fail(c, FR_EINVAL, "fr_rhs_noalloc: this mesh needs " + std::to_string(need) +
                                  " bytes of work buffers; the static scratch holds " +
                                  std::to_string((long long)FR_NOALLOC_MAX_BYTES));
  if (!c->dev_ok)
    return fail(c, FR_ESTATE, "fr_rhs_noalloc: mesh data not on the device yet (fr_set_state uploads it)");
  void* base = nullptr;
  HIPCHK(scratch_on_device(&base));
  Work w;
  char* q = (char*)base;
  for (int k = 0; k < Work::N; ++k) {
    w.ptr[k] = b[k] > 0 ? q : nullptr;
    q += (b[k] + 255) / 256 * 256;
  }
  return launch_rhs(c, u, du, 7, -1, 0.0, &w);
}

fr_status fr_rhs_stages(fr_ctx* c, const double* u, double* du, int mask) {
  if (!c) return FR_EINVAL;
  if (!u || !du || mask < 1 || mask > 7) return fail(c, FR_EINVAL, "bad arguments");
  if (u == du) return fail(c, FR_EINVAL, "u and du must not alias");
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  return launch_rhs(c, u, du, mask);
}

fr_status fr_set_state(fr_ctx* c, const double* u, int on_device) {
  if (!c) return FR_EINVAL;
  if (!u) return fail(c, FR_EINVAL, "null buffer");
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  HIPCHK(hipMemcpyAsync(c->d_state, u, sizeof(double) * c->n_state,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
  if (!on_device) HIPCHK(hipStreamSynchronize(c->st));
  return FR_OK;
}

fr_status fr_get_state(fr_ctx* c, double* u, int on_device) {
  if (!c) return FR_EINVAL;
  if (!u) return fail(c, FR_EINVAL, "null buffer");
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  HIPCHK(hipMemcpyAsync(u, c->d_state, sizeof(double) * c->n_state,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FR_OK;
}

fr_status fr_rk4_step(fr_ctx* c, double dt, int nsteps) {
  if (!c) return FR_EINVAL;
  if (nsteps < 0 || !std::isfinite(dt)) return fail(c, FR_EINVAL, "bad step");
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  const int64_t N = c->n_state;
  // classical RK4: k1 = R(u), k2 = R(u + dt/2 k1), k3 = R(u + dt/2 k2),
  // k4 = R(u + dt k3), u += dt/6 (k1 + 2 k2 + 2 k3 + k4)
  if (c->ph.form == FR_FORM_FUSED) {
    // the stage update is fused into the interface kernel (no k buffer)
    for (int step = 0; step < nsteps; ++step)
      for (int st = 0; st < 4; ++st) {
        s = launch_rhs(c, nullptr, nullptr, 7, st, dt);
        if (s != FR_OK) return s;
      }
    return FR_OK;
  }
  double* ust = c->d_rk;
  double* k = c->d_rk + N;
  double* acc = c->d_rk + 2 * N;
  const double wa[4] = {dt / 6, dt / 3, dt / 3, dt / 6};
  const double wb[4] = {dt / 2, dt / 2, dt, 0.0};
  for (int step = 0; step < nsteps; ++step) {
    for (int st = 0; st < 4; ++st) {
      s = launch_rhs(c, st == 0 ? c->d_state : ust, k);
      if (s != FR_OK) return s;
      double* outu = st == 3 ? c->d_state : ust;
      HIPCHK(fr::rk_stage(N, c->d_state, k, acc, outu, wa[st], wb[st], st == 0 ? 1 : (st == 3 ? 2 : 0), c->st));
    }
  }
  return FR_OK;
}

fr_status fr_integrals(fr_ctx* c, double* out5) {
  if (!c || !out5) return FR_EINVAL;
  fr_status s = ensure_device(c);
  if (s != FR_OK) return s;
  std::vector<double> u(c->n_state);
  s = fr_get_state(c, u.data(), 0);
  if (s != FR_OK) return s;
  for (int v = 0; v < 5; ++v) out5[v] = 0.0;
  for (int t = 0; t < fr::NTYPES; ++t) {
    const fr::RefElem& r = c->ref[t];
    for (int64_t e = 0; e < c->M.nel[t]; ++e) {
      const double* ue = &u[c->off[t] + e * 5 * r.nu];
      // det J at every solution point (constant for affine elements)
      std::vector<double> dj(r.nu, c->M.detj[t][e]);
      if (c->M.curved && t < 2)
        for (int q = 0; q < r.nu; ++q) {
          double J[9];
          fr::jac_point(c->M, t, e, &r.upts[3 * q], J);
          dj[q] = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                  J[2] * (J[3] * J[7] - J[4] * J[6]);
        }
      for (int v = 0; v < 5; ++v) {
        double acc = 0.0;
        for (int q = 0; q < r.nu; ++q) acc += r.wu[q] * dj[q] * ue[v * r.nu + q];
        out5[v] += acc;
      }
    }
  }
  return FR_OK;
}

fr_status fr_fill_lds(void* hip_stream, float value) {
  return fr::lds_fill(value, (hipStream_t)hip_stream) == hipSuccess ? FR_OK : FR_EDEVICE;
}

fr_status fr_ref_operator(int etype, int p, const char* name, double* out, int64_t cap, int64_t* count) {
  if (!name || etype < 0 || etype >= fr::NTYPES) return FR_EINVAL;
  if (p < 1 || p > 4) return FR_EUNSUPPORTED;
  fr::RefElem r;
  try {
    fr::build_ref(etype, p, r);
  } catch (...) {
    return FR_EINVAL;
  }
  const std::vector<double>* v = nullptr;
  std::vector<double> tmp;
  std::string nm(name);
  if (nm == "upts") v = &r.upts;
  else if (nm == "fpts") v = &r.fpts;
  else if (nm == "qpts") v = &r.qpts;
  else if (nm == "qwts") v = &r.qwts;
  else if (nm == "M0") v = &r.M0;
  else if (nm == "M3") v = &r.M3;
  else if (nm == "M7") v = &r.M7;
  else if (nm == "M8") v = &r.M8;
  else if (nm == "wu") v = &r.wu;
  else if (nm == "APd") v = &r.APd;
  else if (nm == "Ku") v = &r.Ku;
  else if (nm == "K0" && etype >= 2) {
    // divergence of a flux held at the solution points (no anti-aliasing):
    // tetrahedra D_d - M3 n_d M0, pyramids Ku_d; 3 x N_u x N_u
    if (etype == 3) {
      tmp = r.Ku;
    } else {
      tmp.assign((size_t)3 * r.nu * r.nu, 0.0);
      for (int d = 0; d < 3; ++d)
        for (int s = 0; s < r.nu; ++s)
          for (int u = 0; u < r.nu; ++u) {
            long double acc = r.Dg[((size_t)d * r.nu + s) * r.nu + u];
            for (int f = 0; f < r.nf; ++f) {
              int face = 0;
              while (face + 1 < r.nfaces && f >= r.face_start[face + 1]) ++face;
              acc -= (long double)r.M3[(size_t)s * r.nf + f] * r.face_normal[3 * face + d] * r.M0[(size_t)f * r.nu + u];
            }
            tmp[((size_t)d * r.nu + s) * r.nu + u] = (double)acc;
          }
    }
    v = &tmp;
  }
  else if (nm == "Dxi" || nm == "Deta" || nm == "Dzeta") {
    int d = nm == "Dxi" ? 0 : (nm == "Deta" ? 1 : 2);
    tmp.assign(r.Dg.begin() + (size_t)d * r.nu * r.nu, r.Dg.begin() + (size_t)(d + 1) * r.nu * r.nu);
    v = &tmp;
  } else
    return FR_EINVAL;
  if (count) *count = (int64_t)v->size();
  if (!out) return FR_OK;
  if (cap < (int64_t)v->size()) return FR_EINVAL;
  std::memcpy(out, v->data(), sizeof(double) * v->size());
  return FR_OK;
}

fr_status fr_connectivity(const fr_ctx* c, int64_t* nbr, int8_t* is_left, int64_t* n_fpts) {
  if (!c) return FR_EINVAL;
  if (!c->mesh_ok) return FR_ESTATE;
  const fr::Mesh& M = c->M;
  // flat flux-point numbering: types in order, element, flux point
  int64_t base[fr::NTYPES] = {};
  for (int t = 1; t < fr::NTYPES; ++t) base[t] = base[t - 1] + M.nel[t - 1] * c->ref[t - 1].nf;
  int64_t total = base[fr::NTYPES - 1] + M.nel[fr::NTYPES - 1] * c->ref[fr::NTYPES - 1].nf;
  if (n_fpts) *n_fpts = total;
  if (!nbr) return FR_OK;
  auto type_of = [&](int64_t s) {
    int t = 0;
    for (int u = 1; u < fr::NTYPES; ++u)
      if (M.nel[u] > 0 && s >= M.slot_base[u]) t = u;
    return t;
  };
  for (int64_t s = 0; s < M.nslots; ++s) {
    int t = type_of(s);
    int64_t e = (s - M.slot_base[t]) / fr::kFacesOf[t];
    int f = int((s - M.slot_base[t]) % fr::kFacesOf[t]);
    int64_t o = M.nbr_slot[s];
    int to = type_of(o);
    int64_t eo = (o - M.slot_base[to]) / fr::kFacesOf[to];
    int fo = int((o - M.slot_base[to]) % fr::kFacesOf[to]);
    const fr::RefElem& r = c->ref[t];
    const fr::RefElem& ro = c->ref[to];
    const std::vector<int>& pm = M.perms[M.perm_id[s]];
    for (int q = 0; q < r.face_npts[f]; ++q) {
      int64_t i = base[t] + e * r.nf + r.face_start[f] + q;
      nbr[i] = base[to] + eo * ro.nf + ro.face_start[fo] + pm[q];
      if (is_left) is_left[i] = (int8_t)M.is_left[s];
    }
  }
  return FR_OK;
}

const char* fr_last_error(const fr_ctx* c) { return c ? c->err.c_str() : "null context"; }

void fr_destroy(fr_ctx* c) {
  if (!c) return;
  if (c->dev_ok || c->d_state) {
    (void)hipStreamSynchronize(c->st);
    void* bufs[] = {c->d_state, c->d_rk,   c->d_fgeo,     c->d_faces,
                    c->d_perms, c->d_pops, c->d_verts[0], c->d_verts[1]};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
    for (void* b : c->w.ptr)
      if (b) (void)hipFree(b);
    for (int t = 0; t < fr::NTYPES; ++t) {
      void* tb[] = {c->d_met[t], c->d_detj[t], c->d_dops[t]};
      for (void* b : tb)
        if (b) (void)hipFree(b);
    }
  }
  free_plain(c);
  delete c;
}

}  // extern "C"
