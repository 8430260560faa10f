// Serving pool (C ABI, host side): many independent periodic-box solves held
// on one GPU at once.  Requests queue in arrival order and are admitted while
// their device footprint fits a fixed byte budget and an active-slot limit;
// every fr_pool_step advances all admitted requests by one classical RK4 step
// with one launch per (element type, order, kernel) covering the elements of
// all of them (a per-workgroup table maps workgroups to (request, element)).
// Host work for new admissions (mesh and connectivity) runs while the GPU
// computes the step.  See include/fr.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fr.h"
#include "fr_host.h"
#include "fr_kernels.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over byte offsets [0, cap), coalescing on release.
class Arena {
 public:
  void reset(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = 0;
  }
  bool alloc(size_t n, size_t& off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used_ += n;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
    used_ -= n;
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// byte offsets of one request's arrays inside its arena block
struct Layout {
  int64_t nel[fr::NTYPES] = {}, nu[2] = {0, 0}, n_state = 0, nslots = 0, nfp = 0, npts = 0;
  size_t state = 0, ust = 0, acc = 0, Rp = 0, Uf = 0, Ub = 0, Vf = 0, faces = 0, fgeo = 0, perms = 0;
  size_t met[2] = {0, 0}, detj[2] = {0, 0}, total = 0;
};

Layout make_layout(const fr_request& q, int rs) {
  Layout L;
  fr::box_counts(q.nx, q.ny, q.nz, q.lo, q.hi, q.kind, L.nel);
  const int n = q.p + 1;
  L.nu[0] = (int64_t)n * n * n;
  L.nu[1] = (int64_t)n * n * (n + 1) / 2;
  L.nfp = (int64_t)n * n;
  L.n_state = 5 * (L.nel[0] * L.nu[0] + L.nel[1] * L.nu[1]);
  L.nslots = 6 * L.nel[0] + 5 * L.nel[1];
  // face points: six quadrilaterals per hexahedron, two triangles and three
  // quadrilaterals per prism
  L.npts = 6 * L.nfp * L.nel[0] + (n * (n + 1) + 3 * L.nfp) * L.nel[1];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.state = take(8 * L.n_state);
  L.ust = take(8 * L.n_state);
  L.acc = take(8 * L.n_state);
  L.Rp = take((size_t)rs * L.n_state);
  L.Uf = take((size_t)rs * 5 * L.npts);
  if (rs == 4) L.Ub = take(sizeof(float) * 5 * L.nslots);  // single precision: face bases
  L.Vf = take((size_t)rs * 4 * L.npts);
  L.faces = take(sizeof(fr::FaceRec) * L.nslots);
  L.fgeo = take((size_t)rs * 4 * L.nslots);
  L.perms = take((size_t)fr::MAX_PERMS * L.nfp);
  for (int t = 0; t < 2; ++t) {
    L.met[t] = take((size_t)rs * 10 * L.nel[t]);
    L.detj[t] = take(8 * L.nel[t]);
  }
  L.total = o;
  return L;
}

// Host arrays of one request, ready to upload: mesh connectivity, face and
// element geometry in the pool precision, and (for the Taylor-Green initial
// state) element origins and Jacobians.  Built off the critical path.
struct Prepared {
  std::string err;  // non-empty: the mesh could not be built
  int64_t nel[2] = {0, 0}, slot_base[2] = {0, 0}, po_base[2] = {0, 0}, nslots = 0, npts = 0;
  int nperm = 0;
  bool diag[2] = {false, false};
  std::vector<fr::FaceRec> faces;
  std::vector<unsigned char> fgeo, met[2];  // precision of the pool
  std::vector<uint8_t> perms;
  std::vector<double> detj[2], geo[2];  // geo: [E][12] origin, J (row-major)
};

template <typename T>
void to_prec(std::vector<unsigned char>& buf, const double* v, size_t n) {
  buf.resize(n * sizeof(T));
  T* d = reinterpret_cast<T*>(buf.data());
  for (size_t i = 0; i < n; ++i) d[i] = T(v[i]);
}

std::shared_ptr<Prepared> prepare(const fr_request& q, const fr::RefElem* refs[fr::NTYPES], int rs, bool saa) {
  auto out = std::make_shared<Prepared>();
  Prepared& R = *out;
  fr::Mesh M;
  try {
    R.err = fr::build_box_mesh(q.nx, q.ny, q.nz, q.lo, q.hi, q.p, q.kind, refs, M);
  } catch (const std::exception& ex) {
    R.err = ex.what();
  }
  if (!R.err.empty()) return out;
  const int64_t nfp = (int64_t)(q.p + 1) * (q.p + 1);
  if ((int64_t)M.perms.size() > fr::MAX_PERMS) {
    R.err = "too many face permutations";
    return out;
  }
  if (saa && !fr::prism_tri_faces_aligned(M)) {
    R.err = "surface-flux anti-aliasing needs aligned prism triangle faces";
    return out;
  }
  const int64_t S = M.nslots;
  R.nslots = S;
  R.npts = M.npts;
  R.faces.resize(S);
  std::vector<double> geo(4 * S);
  for (int64_t i = 0; i < S; ++i) {
    R.faces[i].nbr = (int32_t)M.nbr_slot[i];
    R.faces[i].npo = (int32_t)M.slot_po[M.nbr_slot[i]];
    R.faces[i].pad = 0;
    R.faces[i].info = (M.perm_id[i] << 1) | (M.is_left[i] ? 1 : 0);
    for (int d = 0; d < 3; ++d) geo[4 * i + d] = M.nrm[3 * i + d];
    geo[4 * i + 3] = M.mag[i];
  }
  if (rs == 4)
    to_prec<float>(R.fgeo, geo.data(), geo.size());
  else
    to_prec<double>(R.fgeo, geo.data(), geo.size());
  R.nperm = (int)M.perms.size();
  R.perms.assign(M.perms.size() * nfp, 0);
  for (size_t k = 0; k < M.perms.size(); ++k)
    for (size_t r = 0; r < M.perms[k].size(); ++r) R.perms[k * nfp + r] = (uint8_t)M.perms[k][r];
  for (int t = 0; t < 2; ++t) {
    const int64_t E = M.nel[t];
    R.nel[t] = E;
    R.slot_base[t] = M.slot_base[t];
    R.po_base[t] = E > 0 ? M.slot_po[M.slot_base[t]] : 0;
    std::vector<double> met(10 * E);
    bool d = true;
    for (int64_t e = 0; e < E; ++e) {
      for (int k = 0; k < 9; ++k) met[10 * e + k] = M.jinv[t][9 * e + k];
      met[10 * e + 9] = M.detj[t][e];
      const double* A = &M.jac[t][9 * e];
      d = d && A[1] == 0 && A[2] == 0 && A[3] == 0 && A[5] == 0 && A[6] == 0 && A[7] == 0;
    }
    R.diag[t] = d;
    if (rs == 4)
      to_prec<float>(R.met[t], met.data(), met.size());
    else
      to_prec<double>(R.met[t], met.data(), met.size());
    R.detj[t] = M.detj[t];
    if (!q.u_init) {
      R.geo[t].resize(12 * E);
      for (int64_t e = 0; e < E; ++e) {
        for (int k = 0; k < 3; ++k) R.geo[t][12 * e + k] = M.org[t][3 * e + k];
        for (int k = 0; k < 9; ++k) R.geo[t][12 * e + 3 + k] = M.jac[t][9 * e + k];
      }
    }
  }
  return out;
}

enum { Q_QUEUED = 0, Q_ACTIVE = 1, Q_DONE = 2, Q_FAILED = 3 };
// requests prepared ahead of admission by the worker thread
constexpr int kLookahead = 4;

struct Req {
  int64_t id = 0;
  fr_request q{};
  Layout L;
  int status = Q_QUEUED, steps_done = 0;
  bool inject_err = false;  // testing aid: its host set-up fails at admission
  size_t off = 0;
  char* base = nullptr;
  bool has[2] = {false, false}, diag[2] = {false, false};
  fr::Seg seg[2];
};

// per (element type, order): segment list and workgroup tables of the active set
struct Variant {
  int t = 0, p = 0;
  bool diag = true;
  std::vector<fr::Seg> segs;
  std::vector<fr::BlkRef> bt[3];
  size_t off_segs = 0, off_bt[3] = {0, 0, 0};  // byte offsets in the device table
};

}  // namespace

struct fr_pool {
  fr_physics ph;
  hipStream_t st = nullptr;
  std::string err;
  int64_t budget = 0;
  int max_active = 0;
  int rs = 8;
  char* d_arena = nullptr;
  Arena arena;
  int64_t next_id = 0;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;  // admission order
  bool dirty = true;
  std::vector<Variant> vars;
  char* d_tab = nullptr;
  size_t tab_cap = 0;
  std::vector<unsigned char> h_tab;
  // reference elements, operator factors and prism tables per order
  bool ref_ok[5] = {false, false, false, false, false};
  fr::RefElem ref[2][5];
  fr::HostOps hops[2][5];
  void* d_pops[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  fr::GasHost gas;
  // host staging kept alive until the stream has consumed it
  std::vector<std::vector<unsigned char>> staging;
  std::vector<std::shared_ptr<Prepared>> staged_preps;
  std::vector<int64_t> last_admitted, last_finished;
  // preparation worker: builds the host arrays of the next queued requests
  // while the GPU runs; mu guards prep_q, in_flight, ready, stop and inserts
  // into reqs
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<int64_t> prep_q;
  int64_t in_flight = -1;
  std::map<int64_t, std::shared_ptr<Prepared>> ready;
};

namespace {

fr_status pfail(fr_pool* P, fr_status s, const std::string& m) {
  if (P) P->err = m;
  return s;
}

#define PHIP(call)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return pfail(P, FR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

fr_status check_request(fr_pool* P, const fr_request* q) {
  if (!q) return pfail(P, FR_EINVAL, "null request");
  if (q->nx < 1 || q->ny < 1 || q->nz < 1 || !(q->hi > q->lo) || q->kind < 0 || q->kind >= fr::kNumKinds)
    return pfail(P, FR_EINVAL, "bad mesh size");
  if (fr::kind_dense(q->kind) || fr::kind_curved(q->kind))
    return pfail(P, FR_EUNSUPPORTED, "the pool serves affine hexahedra and prisms");
  if (q->p < 1 || q->p > 4) return pfail(P, FR_EUNSUPPORTED, "order must be 1..4");
  if (q->nsteps < 0 || !std::isfinite(q->dt)) return pfail(P, FR_EINVAL, "bad step");
  if (!q->u_init && !(q->tgv_p0 > 0.0)) return pfail(P, FR_EINVAL, "no initial state and tgv_p0 <= 0");
  const int64_t cells = (int64_t)q->nx * q->ny * q->nz;
  if (cells > (int64_t)1 << 26) return pfail(P, FR_EINVAL, "mesh too large");
  return FR_OK;
}

// host reference elements and operator factors of order p (submit time,
// before the worker may read them)
fr_status ensure_refs(fr_pool* P, int p) {
  if (P->ref_ok[p]) return FR_OK;
  try {
    fr::build_ref(0, p, P->ref[0][p]);
    fr::build_ref(1, p, P->ref[1][p]);
  } catch (const std::exception& ex) {
    return pfail(P, FR_EINVAL, ex.what());
  }
  for (int t = 0; t < 2; ++t) {
    const fr::RefElem& r = P->ref[t][p];
    fr::HostOps& h = P->hops[t][p];
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
  P->ref_ok[p] = true;
  return FR_OK;
}

// device copy of the prism operator table of order p (admission time)
fr_status ensure_device_ops(fr_pool* P, int p) {
  if (P->d_pops[p]) return FR_OK;
  const size_t nb = fr::prism_ops_bytes(p, P->ph.prec);
  P->staging.emplace_back(nb);
  fr::prism_ops_pack(P->ref[1][p], P->ph.prec, P->staging.back().data());
  PHIP(hipMalloc(&P->d_pops[p], nb));
  PHIP(hipMemcpyAsync(P->d_pops[p], P->staging.back().data(), nb, hipMemcpyHostToDevice, P->st));
  return FR_OK;
}

void worker_main(fr_pool* P) {
  std::unique_lock<std::mutex> lk(P->mu);
  for (;;) {
    P->cv.wait(lk, [P] { return P->stop || (!P->prep_q.empty() && (int)P->ready.size() < kLookahead); });
    if (P->stop) return;
    const int64_t id = P->prep_q.front();
    P->prep_q.pop_front();
    P->in_flight = id;
    const fr_request q = P->reqs.at(id)->q;
    const fr::RefElem* refs[fr::NTYPES] = {&P->ref[0][q.p], &P->ref[1][q.p], nullptr, nullptr};
    const int rs = P->rs;
    lk.unlock();
    std::shared_ptr<Prepared> r = prepare(q, refs, rs, P->ph.surface_aa != 0);
    lk.lock();
    P->ready[id] = std::move(r);
    P->in_flight = -1;
    P->cv.notify_all();
  }
}

// the prepared arrays of request id: from the worker if it has built (or is
// building) them, else built here
std::shared_ptr<Prepared> take_prepared(fr_pool* P, int64_t id) {
  std::unique_lock<std::mutex> lk(P->mu);
  for (;;) {
    auto it = P->ready.find(id);
    if (it != P->ready.end()) {
      std::shared_ptr<Prepared> r = std::move(it->second);
      P->ready.erase(it);
      P->cv.notify_all();
      return r;
    }
    if (P->in_flight == id) {
      P->cv.wait(lk);
      continue;
    }
    auto qi = std::find(P->prep_q.begin(), P->prep_q.end(), id);
    if (qi != P->prep_q.end()) P->prep_q.erase(qi);
    const fr_request q = P->reqs.at(id)->q;
    const fr::RefElem* refs[fr::NTYPES] = {&P->ref[0][q.p], &P->ref[1][q.p], nullptr, nullptr};
    const int rs = P->rs;
    lk.unlock();
    return prepare(q, refs, rs, P->ph.surface_aa != 0);
  }
}

// enqueue an upload of a prepared host array (kept alive until the sync)
fr_status upload_raw(fr_pool* P, void* dst, const void* src, size_t n) {
  if (n) PHIP(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, P->st));
  return FR_OK;
}

// enqueue the uploads and the initial state of an admitted request; it
// joins the active set at the next step
fr_status admit(fr_pool* P, Req& R) {
  const fr_request& q = R.q;
  fr_status s = ensure_device_ops(P, q.p);
  if (s != FR_OK) return s;
  std::shared_ptr<Prepared> pr = take_prepared(P, R.id);
  if (R.inject_err) return pfail(P, FR_EINVAL, "injected preparation error");
  if (!pr->err.empty()) return pfail(P, FR_EINVAL, pr->err);
  const Prepared& M = *pr;
  P->staged_preps.push_back(pr);
  const Layout& L = R.L;
  if (M.nel[0] != L.nel[0] || M.nel[1] != L.nel[1] || M.nslots != L.nslots || M.npts != L.npts)
    return pfail(P, FR_EINVAL, "mesh sizes differ from the footprint layout");
  char* b = R.base;
  s = upload_raw(P, b + L.faces, M.faces.data(), sizeof(fr::FaceRec) * M.faces.size());
  if (s == FR_OK) s = upload_raw(P, b + L.fgeo, M.fgeo.data(), M.fgeo.size());
  if (s == FR_OK) s = upload_raw(P, b + L.perms, M.perms.data(), M.perms.size());
  if (s != FR_OK) return s;
  int64_t off = 0;     // state offset of the type
  size_t tmp = L.ust;  // scratch for the initial-state geometry (ust is written before it is read)
  for (int t = 0; t < 2; ++t) {
    const int64_t E = M.nel[t];
    R.has[t] = E > 0;
    if (!E) continue;
    R.diag[t] = M.diag[t];
    s = upload_raw(P, b + L.met[t], M.met[t].data(), M.met[t].size());
    if (s == FR_OK) s = upload_raw(P, b + L.detj[t], M.detj[t].data(), 8 * M.detj[t].size());
    if (s != FR_OK) return s;
    fr::Seg& g = R.seg[t];
    g.U = (double*)(b + L.state) + off;
    g.ust = (double*)(b + L.ust) + off;
    g.acc = (double*)(b + L.acc) + off;
    g.du = nullptr;
    g.Uf = b + L.Uf;
    g.Ub = P->rs == 4 ? (float*)(b + L.Ub) : nullptr;
    g.Vf = b + L.Vf;
    g.Rp = b + L.Rp + (size_t)P->rs * off;
    g.faces = (const fr::FaceRec*)(b + L.faces);
    g.fgeo = b + L.fgeo;
    g.perms = (const uint8_t*)(b + L.perms);
    g.met = b + L.met[t];
    g.detj = (const double*)(b + L.detj[t]);
    g.dt = q.dt;
    g.E = (int32_t)E;
    g.slot_base = (int32_t)M.slot_base[t];
    g.po_base = (int32_t)M.po_base[t];
    g.nperm = M.nperm;
    if (!q.u_init) {
      // Taylor-Green state from element origins, Jacobians and reference points
      const fr::RefElem& r = P->ref[t][q.p];
      const size_t need = 8 * (M.geo[t].size() + r.upts.size());
      if (tmp + need > L.acc) return pfail(P, FR_EINVAL, "initial-state scratch too small");
      double* dg = (double*)(b + tmp);
      double* dr = dg + M.geo[t].size();
      s = upload_raw(P, dg, M.geo[t].data(), 8 * M.geo[t].size());
      if (s == FR_OK) s = upload_raw(P, dr, r.upts.data(), 8 * r.upts.size());
      if (s != FR_OK) return s;
      PHIP(fr::tgv_init(E, r.nu, dg, dr, P->ph.gamma, q.tgv_p0, g.U, P->st));
      tmp = align_up(tmp + need);
    }
    off += 5 * E * L.nu[t];
  }
  if (q.u_init) {
    PHIP(hipMemcpyAsync(b + L.state, q.u_init, 8 * L.n_state, hipMemcpyHostToDevice, P->st));
  }
  R.status = Q_ACTIVE;
  return FR_OK;
}

// rebuild the per-variant segment lists and workgroup tables of the active
// set and upload them (the stream is idle when this runs)
fr_status rebuild_tables(fr_pool* P) {
  P->vars.clear();
  std::map<int, size_t> index;  // t * 8 + p -> variant
  for (int64_t id : P->active) {
    const Req& R = *P->reqs.at(id);
    for (int t = 0; t < 2; ++t) {
      if (!R.has[t]) continue;
      const int key = t * 8 + R.q.p;
      auto it = index.find(key);
      if (it == index.end()) {
        it = index.emplace(key, P->vars.size()).first;
        P->vars.emplace_back();
        P->vars.back().t = t;
        P->vars.back().p = R.q.p;
      }
      Variant& V = P->vars[it->second];
      V.diag = V.diag && R.diag[t];
      const int32_t si = (int32_t)V.segs.size();
      V.segs.push_back(R.seg[t]);
      for (int k = 0; k < 3; ++k) {
        const bool saa = P->ph.surface_aa != 0;
        const int eb = t == 0 ? fr::hex_block_elems(R.q.p, P->ph.prec, k, P->ph.flux_aa != 0, saa)
                              : fr::prism_block_elems(R.q.p, P->ph.prec, k, saa);
        for (int32_t e0 = 0; e0 < R.seg[t].E; e0 += eb) V.bt[k].push_back({si, e0});
      }
    }
  }
  size_t o = 0;
  for (Variant& V : P->vars) {
    V.off_segs = o;
    o = align_up(o + sizeof(fr::Seg) * V.segs.size());
    for (int k = 0; k < 3; ++k) {
      V.off_bt[k] = o;
      o = align_up(o + sizeof(fr::BlkRef) * V.bt[k].size());
    }
  }
  if (o > P->tab_cap) {
    if (P->d_tab) PHIP(hipFree(P->d_tab));
    P->d_tab = nullptr;
    P->tab_cap = std::max(o, 2 * P->tab_cap);
    PHIP(hipMalloc(&P->d_tab, P->tab_cap));
  }
  P->h_tab.assign(o, 0);
  for (Variant& V : P->vars) {
    std::memcpy(P->h_tab.data() + V.off_segs, V.segs.data(), sizeof(fr::Seg) * V.segs.size());
    for (int k = 0; k < 3; ++k)
      std::memcpy(P->h_tab.data() + V.off_bt[k], V.bt[k].data(), sizeof(fr::BlkRef) * V.bt[k].size());
  }
  // h_tab stays untouched until the next rebuild, which follows a stream sync
  if (o) PHIP(hipMemcpyAsync(P->d_tab, P->h_tab.data(), o, hipMemcpyHostToDevice, P->st));
  P->dirty = false;
  return FR_OK;
}

// enqueue one RK4 step of every active request: per stage, each kernel of
// the right-hand side over every variant (disu of all types before any
// volume kernel, since mixed meshes exchange face data across types)
fr_status enqueue_step(fr_pool* P, int* launches) {
  int nl = 0;
  for (int st = 0; st < 4; ++st)
    for (int k = 0; k < 3; ++k)
      for (const Variant& V : P->vars) {
        fr::TypeArgs a;
        a.p = V.p;
        a.stage = 1 << k;
        a.diag = V.diag;
        a.from_ust = st > 0;
        a.rk = st;
        a.aa = P->ph.flux_aa != 0;
        a.saa = P->ph.surface_aa != 0;
        a.segs = (const fr::Seg*)(P->d_tab + V.off_segs);
        for (int j = 0; j < 3; ++j) {
          a.bt[j] = (const fr::BlkRef*)(P->d_tab + V.off_bt[j]);
          a.nblk[j] = (int)V.bt[j].size();
        }
        a.dops = P->d_pops[V.p];
        a.ops = &P->hops[V.t][V.p];
        a.gas = &P->gas;
        hipError_t e = V.t == 0 ? fr::hex_rhs(a, P->ph.prec, P->st) : fr::prism_rhs(a, P->ph.prec, P->st);
        if (e != hipSuccess) return pfail(P, FR_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        ++nl;
      }
  if (launches) *launches = nl;
  return FR_OK;
}

fr_status finish(fr_pool* P, Req& R) {
  if (R.q.u_out) {
    PHIP(hipMemcpyAsync(R.q.u_out, R.base + R.L.state, 8 * R.L.n_state, hipMemcpyDeviceToHost, P->st));
    PHIP(hipStreamSynchronize(P->st));
  }
  P->arena.release(R.off, R.L.total);
  R.base = nullptr;
  R.status = Q_DONE;
  P->active.erase(std::find(P->active.begin(), P->active.end(), R.id));
  P->last_finished.push_back(R.id);
  P->dirty = true;
  return FR_OK;
}

// the request at the head of the queue leaves it as failed: it never ran
// and holds no memory; it is reported among the finished ids of this round
void fail_head(fr_pool* P, Req& R, const std::string& why) {
  P->queue.pop_front();
  R.status = Q_FAILED;
  P->err = "request " + std::to_string(R.id) + ": " + why;
  P->last_finished.push_back(R.id);
}

// queued requests at the head whose host set-up has already failed leave
// the queue before any device work (host only; does not wait for the
// preparation worker: a request still being prepared is left to admission)
void screen_queue(fr_pool* P) {
  while (!P->queue.empty()) {
    Req& R = *P->reqs.at(P->queue.front());
    std::string why;
    {
      std::lock_guard<std::mutex> lk(P->mu);
      auto it = P->ready.find(R.id);
      if (it == P->ready.end()) return;
      why = R.inject_err ? std::string("injected preparation error") : it->second->err;
      if (why.empty()) return;
      P->ready.erase(it);
      P->cv.notify_all();
    }
    fail_head(P, R, why);
  }
}

}  // namespace

extern "C" {

fr_status fr_pool_create(const fr_physics* ph, void* stream, int64_t budget_bytes, int max_active, fr_pool** out) {
  if (!ph || !out) return FR_EINVAL;
  *out = nullptr;
  if (!(ph->gamma > 1.0) || !(ph->prandtl > 0.0) || !(ph->mu >= 0.0) || !(ph->ldg_tau >= 0.0) ||
      !std::isfinite(ph->ldg_beta) || !std::isfinite(ph->pref) || ph->prec < 0 || ph->prec > 1 ||
      ph->flux_aa < 0 || ph->flux_aa > 1 || ph->surface_aa < 0 || ph->surface_aa > 1)
    return FR_EINVAL;
  if (ph->form != FR_FORM_FUSED) return FR_EUNSUPPORTED;
  if (ph->surface_aa && !ph->flux_aa) return FR_EUNSUPPORTED;
  if (budget_bytes <= 0 || max_active < 1) return FR_EINVAL;
  fr_pool* P = new (std::nothrow) fr_pool();
  if (!P) return FR_ENOMEM;
  P->ph = *ph;
  P->st = (hipStream_t)stream;
  P->budget = budget_bytes;
  P->max_active = max_active;
  P->rs = ph->prec == FR_PREC_FP64 ? 8 : 4;
  P->gas = {ph->gamma, ph->prandtl, ph->mu, ph->pref, ph->ldg_beta, ph->ldg_tau, ph->rho_ref};
  *out = P;
  return FR_OK;
}

fr_status fr_pool_footprint(const fr_pool* P, const fr_request* q, int64_t* bytes, int64_t* n_state) {
  if (!P || !q) return FR_EINVAL;
  fr_status s = check_request(const_cast<fr_pool*>(P), q);
  if (s != FR_OK) return s;
  const Layout L = make_layout(*q, P->rs);
  if (bytes) *bytes = (int64_t)L.total;
  if (n_state) *n_state = L.n_state;
  return FR_OK;
}

fr_status fr_pool_submit(fr_pool* P, const fr_request* q, int64_t* id) {
  if (!P) return FR_EINVAL;
  fr_status s = check_request(P, q);
  if (s != FR_OK) return s;
  auto R = std::make_unique<Req>();
  R->q = *q;
  R->L = make_layout(*q, P->rs);
  if ((int64_t)R->L.total > P->budget) return pfail(P, FR_ENOMEM, "request larger than the pool budget");
  s = ensure_refs(P, q->p);
  if (s != FR_OK) return s;
  const int64_t rid = P->next_id++;
  R->id = rid;
  if (id) *id = rid;
  P->queue.push_back(rid);
  {
    std::lock_guard<std::mutex> lk(P->mu);
    P->reqs[rid] = std::move(R);
    P->prep_q.push_back(rid);
  }
  if (!P->worker.joinable()) P->worker = std::thread(worker_main, P);
  P->cv.notify_all();
  return FR_OK;
}

fr_status fr_pool_step(fr_pool* P, fr_pool_stats* stats) {
  if (!P) return FR_EINVAL;
  fr_pool_stats S;
  std::memset(&S, 0, sizeof(S));
  P->last_admitted.clear();
  P->last_finished.clear();
  screen_queue(P);
  if (!P->d_arena) {
    PHIP(hipMalloc(&P->d_arena, (size_t)P->budget));
    P->arena.reset((size_t)P->budget);
  }
  fr_status s = FR_OK;
  if (P->dirty) {
    s = rebuild_tables(P);
    if (s != FR_OK) return s;
  }
  // 1. one RK4 step of the active set (asynchronous)
  const std::vector<int64_t> stepped = P->active;
  if (!stepped.empty()) {
    s = enqueue_step(P, &S.n_launches);
    if (s != FR_OK) return s;
  }
  for (int64_t id : stepped) S.dof += P->reqs.at(id)->L.n_state;
  S.n_active = (int)stepped.size();
  // 2. admissions in arrival order while memory and slots allow; their host
  //    set-up overlaps the step on the GPU
  while (!P->queue.empty() && (int)P->active.size() < P->max_active) {
    Req& R = *P->reqs.at(P->queue.front());
    size_t off = 0;
    if (!P->arena.alloc(R.L.total, off)) break;
    R.off = off;
    R.base = P->d_arena + off;
    s = admit(P, R);
    if (s != FR_OK) {
      P->arena.release(off, R.L.total);
      R.base = nullptr;
      if (s != FR_EINVAL) return s;  // a device error: the pool is unusable
      // the request's own set-up failed: it leaves the queue, the round goes on
      fail_head(P, R, std::string(P->err));
      continue;
    }
    P->queue.pop_front();
    P->active.push_back(R.id);
    P->last_admitted.push_back(R.id);
    P->dirty = true;
    ++S.n_admitted;
  }
  PHIP(hipStreamSynchronize(P->st));
  P->staging.clear();
  P->staged_preps.clear();
  // 3. accounting and retirement
  for (int64_t id : stepped) {
    Req& R = *P->reqs.at(id);
    if (++R.steps_done >= R.q.nsteps) {
      s = finish(P, R);
      if (s != FR_OK) return s;
    }
  }
  for (int64_t id : P->last_admitted) {
    Req& R = *P->reqs.at(id);
    if (R.status == Q_ACTIVE && R.q.nsteps == 0) {
      s = finish(P, R);
      if (s != FR_OK) return s;
    }
  }
  S.n_finished = (int)P->last_finished.size();
  S.n_queued = (int)P->queue.size();
  S.bytes_in_use = (int64_t)P->arena.used();
  if (stats) *stats = S;
  return FR_OK;
}

fr_status fr_pool_events(const fr_pool* P, int64_t* admitted, int* n_admitted, int64_t* finished, int* n_finished,
                         int cap) {
  if (!P || cap < 0) return FR_EINVAL;
  const int na = (int)P->last_admitted.size(), nf = (int)P->last_finished.size();
  if (n_admitted) *n_admitted = na;
  if (n_finished) *n_finished = nf;
  if ((admitted && na > cap) || (finished && nf > cap)) return FR_EINVAL;
  if (admitted) std::copy(P->last_admitted.begin(), P->last_admitted.end(), admitted);
  if (finished) std::copy(P->last_finished.begin(), P->last_finished.end(), finished);
  return FR_OK;
}

fr_status fr_pool_inject_prepare_error(fr_pool* P, int64_t id) {
  if (!P) return FR_EINVAL;
  auto it = P->reqs.find(id);
  if (it == P->reqs.end() || it->second->status != Q_QUEUED) return pfail(P, FR_EINVAL, "no such queued request");
  std::lock_guard<std::mutex> lk(P->mu);
  it->second->inject_err = true;
  return FR_OK;
}

fr_status fr_pool_query(const fr_pool* P, int64_t id, int* status, int* steps_done) {
  if (!P) return FR_EINVAL;
  auto it = P->reqs.find(id);
  if (it == P->reqs.end()) return FR_EINVAL;
  if (status) *status = it->second->status;
  if (steps_done) *steps_done = it->second->steps_done;
  return FR_OK;
}

const char* fr_pool_last_error(const fr_pool* P) { return P ? P->err.c_str() : "null pool"; }

void fr_pool_destroy(fr_pool* P) {
  if (!P) return;
  if (P->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(P->mu);
      P->stop = true;
    }
    P->cv.notify_all();
    P->worker.join();
  }
  if (P->d_arena || P->d_tab) (void)hipStreamSynchronize(P->st);
  if (P->d_arena) (void)hipFree(P->d_arena);
  if (P->d_tab) (void)hipFree(P->d_tab);
  for (void* b : P->d_pops)
    if (b) (void)hipFree(b);
  delete P;
}

}  // extern "C"
