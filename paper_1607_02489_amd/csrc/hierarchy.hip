// Alg. 1 (setup_hierarchy without relaxation) as a native driver over the
// per-level calls, a batch form that builds many hierarchies concurrently
// and replays all of their numeric phases as one captured hipGraph, and the
// level-by-level device memory bookkeeping both need.
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

using namespace emin;

struct emin_hierarchy_s {
  Arena ar;                              // P and coarse values, reports
  emin_params_t prm{};
  std::vector<emin_pattern_t*> pats;     // one handle per transfer
  std::vector<emin_system_t> sys;        // input system of each level (level 0 borrowed)
  std::vector<double*> Pv, Pp, Ac, Bc;
  std::vector<emin_report_t*> rep;
  std::vector<emin_sizes_t> sizes;
  emin_system_t coarsest{};
  ~emin_hierarchy_s() {
    for (size_t l = pats.size(); l-- > 0;) emin_pattern_destroy(pats[l]);
  }
};

struct emin_batch_s {
  std::vector<emin_hierarchy_t*> hs;
  std::vector<emin_system_t> sys;
  emin_params_t prm{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;   // capture origin (the caller's stream may be the null stream)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  ~emin_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

emin_status coarse_of(emin_pattern_t* p, const double* Ac, const double* Bc, int dim,
                      emin_system_t* out) {
  emin_view_t a, b, x, q;
  emin_status st;
  if ((st = emin_pattern_view(p, EMIN_VIEW_AC, &a)) != EMIN_OK) return st;
  if ((st = emin_pattern_view(p, EMIN_VIEW_BC, &b)) != EMIN_OK) return st;
  if ((st = emin_pattern_view(p, EMIN_VIEW_XVC, &x)) != EMIN_OK) return st;
  if ((st = emin_pattern_view(p, EMIN_VIEW_P2VC, &q)) != EMIN_OK) return st;
  emin_system_t c{};
  c.dim = dim;
  c.Ahat = emin_csr_t{a.n, a.ncols, a.nnz, a.rowptr, a.col, Ac};
  c.Bdiv = emin_csr_t{b.n, b.ncols, b.nnz, b.rowptr, b.col, Bc};
  c.xv = static_cast<const double*>(x.data);
  c.p2v = static_cast<const int32_t*>(q.data);
  c.Wv = nullptr;
  c.Wp = nullptr;
  *out = c;
  return EMIN_OK;
}

int64_t dofs_of(const emin_system_t& s) { return (int64_t)s.dim * s.Ahat.nrows + s.Bdiv.nrows; }

emin_status resetup_levels(emin_hierarchy_t* h, hipStream_t s) {
  for (size_t l = 0; l < h->pats.size(); l++) {
    emin_status st = emin_setup(h->pats[l], &h->sys[l], &h->prm, h->Pv[l], h->Pp[l], s, h->rep[l]);
    if (st != EMIN_OK) return st;
    st = emin_rap(h->pats[l], &h->sys[l], h->Pv[l], h->Pp[l], h->Ac[l], h->Bc[l],
                  h->prm.precision, s);
    if (st != EMIN_OK) return st;
  }
  return EMIN_OK;
}

}  // namespace

extern "C" {

emin_status emin_hierarchy_build(const emin_system_t* sys, const emin_params_t* prm,
                                 int32_t nlevels, int64_t min_dofs, void* stream,
                                 emin_hierarchy_t** out) {
  if (!out || !sys || !prm || nlevels < 1) return EMIN_ERR_ARG;
  *out = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  emin_hierarchy_t* h = nullptr;
  try {
    h = new emin_hierarchy_s();
  } catch (...) {
    return EMIN_ERR_OOM;
  }
  h->prm = *prm;
  h->prm.flags &= ~(uint32_t)EMIN_FLAG_PATTERN_VALUES;   // re-setups take new values
  // each level's setup follows its pattern on the same values
  emin_params_t first = h->prm;
  first.flags |= EMIN_FLAG_PATTERN_VALUES;
  emin_system_t cur = *sys;
  emin_status st = EMIN_OK;
  try {
    for (int l = 0; l + 1 < nlevels; l++) {
      if (dofs_of(cur) <= min_dofs) break;
      emin_pattern_t* p = nullptr;
      if ((st = emin_pattern(&cur, prm, stream, &p)) != EMIN_OK) break;
      h->pats.push_back(p);
      emin_sizes_t z;
      emin_pattern_info(p, &z);
      h->sizes.push_back(z);
      h->sys.push_back(cur);
      h->Pv.push_back(h->ar.alloc<double>(z.nnz_Pv));
      h->Pp.push_back(h->ar.alloc<double>(z.nnz_Pp));
      h->Ac.push_back(h->ar.alloc<double>(z.nnz_Ac));
      h->Bc.push_back(h->ar.alloc<double>(z.nnz_Bc));
      h->rep.push_back(h->ar.alloc<emin_report_t>(1));
      if ((st = emin_setup(p, &cur, &first, h->Pv.back(), h->Pp.back(), stream,
                           h->rep.back())) != EMIN_OK)
        break;
      if ((st = emin_rap(p, &cur, h->Pv.back(), h->Pp.back(), h->Ac.back(), h->Bc.back(),
                         prm->precision, stream)) != EMIN_OK)
        break;
      if ((st = coarse_of(p, h->Ac.back(), h->Bc.back(), cur.dim, &cur)) != EMIN_OK) break;
    }
  } catch (const Error& e) {
    set_last_error(e.what());
    st = e.code;
  } catch (...) {
    set_last_error("emin_hierarchy_build: unexpected exception");
    st = EMIN_ERR_DEVICE;
  }
  if (st != EMIN_OK) {
    (void)hipStreamSynchronize(s);
    delete h;
    return st;
  }
  h->coarsest = cur;
  h->ar.used_on(s);
  *out = h;
  return EMIN_OK;
}

emin_status emin_hierarchy_resetup(emin_hierarchy_t* h, const emin_system_t* sys, void* stream) {
  if (!h || !sys) return EMIN_ERR_ARG;
  if (h->pats.empty()) return EMIN_OK;
  h->sys[0] = *sys;
  try {
    StreamUse use_ar(h->ar, reinterpret_cast<hipStream_t>(stream));
    return resetup_levels(h, reinterpret_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return EMIN_ERR_DEVICE;
  }
}

emin_status emin_hierarchy_info(const emin_hierarchy_t* h, int32_t* ntransfers,
                                emin_sizes_t* per_level, int32_t cap) {
  if (!h || !ntransfers) return EMIN_ERR_ARG;
  *ntransfers = (int32_t)h->pats.size();
  if (per_level)
    for (int32_t l = 0; l < cap && l < (int32_t)h->sizes.size(); l++) per_level[l] = h->sizes[l];
  return EMIN_OK;
}

emin_status emin_hierarchy_level(const emin_hierarchy_t* h, int32_t level, emin_pattern_t** pat,
                                 const double** Pv, const double** Pp, const double** Ac,
                                 const double** Bc, const emin_report_t** report) {
  if (!h || level < 0 || level >= (int32_t)h->pats.size()) return EMIN_ERR_ARG;
  if (pat) *pat = h->pats[level];
  if (Pv) *Pv = h->Pv[level];
  if (Pp) *Pp = h->Pp[level];
  if (Ac) *Ac = h->Ac[level];
  if (Bc) *Bc = h->Bc[level];
  if (report) *report = h->rep[level];
  return EMIN_OK;
}

int64_t emin_hierarchy_device_bytes(const emin_hierarchy_t* h) {
  if (!h) return 0;
  int64_t b = (int64_t)h->ar.bytes();
  for (const emin_pattern_t* p : h->pats) {
    emin_sizes_t z;
    if (emin_pattern_info(p, &z) == EMIN_OK) b += z.device_bytes;
  }
  return b;
}

void emin_hierarchy_destroy(emin_hierarchy_t* h) {
  if (!h) return;
  delete h;
}

emin_status emin_hierarchy_build_batch(const emin_system_t* const* systems, int32_t count,
                                       const emin_params_t* prm, int32_t nlevels,
                                       int64_t min_dofs, int32_t max_parallel,
                                       emin_hierarchy_t** out) {
  if (!systems || !prm || !out || count < 0 || max_parallel < 1) return EMIN_ERR_ARG;
  for (int32_t i = 0; i < count; i++) out[i] = nullptr;
  std::atomic<int32_t> next{0};
  std::atomic<int> first_err{EMIN_OK};
  std::mutex msg_mu;
  std::string first_msg;   // the first failing build's message (worker threads')
  auto work = [&]() {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      int ok = EMIN_OK;
      first_err.compare_exchange_strong(ok, EMIN_ERR_DEVICE);
      return;
    }
    while (true) {
      const int32_t i = next.fetch_add(1);
      if (i >= count) break;
      emin_status st = emin_hierarchy_build(systems[i], prm, nlevels, min_dofs, s, &out[i]);
      std::string why;
      if (st != EMIN_OK) {
        why = emin_last_error();
      } else {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
          st = EMIN_ERR_DEVICE;
          why = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
        }
      }
      if (st != EMIN_OK) {
        int ok = EMIN_OK;
        if (first_err.compare_exchange_strong(ok, st)) {
          std::lock_guard<std::mutex> g(msg_mu);
          first_msg = "system " + std::to_string(i) + ": " + why;
        }
      }
    }
    (void)hipStreamDestroy(s);
  };
  const int nt = max_parallel < count ? max_parallel : count;
  std::vector<std::thread> ts;
  for (int t = 0; t < nt; t++) ts.emplace_back(work);
  for (auto& t : ts) t.join();
  if (first_err.load() != EMIN_OK) {
    for (int32_t i = 0; i < count; i++) {
      emin_hierarchy_destroy(out[i]);
      out[i] = nullptr;
    }
    set_last_error(first_msg.c_str());
    return (emin_status)first_err.load();
  }
  return EMIN_OK;
}

emin_status emin_batch_create(emin_hierarchy_t* const* hs, const emin_system_t* const* systems,
                              int32_t count, void* stream, emin_batch_t** out) {
  if (!hs || !systems || !out || count < 1) return EMIN_ERR_ARG;
  *out = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  emin_batch_t* b = new emin_batch_s();
  emin_status st = EMIN_OK;
  try {
    for (int32_t i = 0; i < count; i++) {
      if (!hs[i]) throw Error(EMIN_ERR_ARG, "NULL hierarchy");
      b->hs.push_back(hs[i]);
      if (!hs[i]->pats.empty()) hs[i]->sys[0] = *systems[i];
    }
    // one eager pass first: lazily allocated buffers exist before capture
    for (emin_hierarchy_t* h : b->hs)
      if ((st = resetup_levels(h, s)) != EMIN_OK) throw Error(st, "eager re-setup");
    HIP_OK(hipStreamSynchronize(s));
    // capture: fork one branch per hierarchy off the origin stream, join back
    b->side.resize(count);
    b->ev.resize(count + 1);
    HIP_OK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    for (int32_t i = 0; i < count; i++) HIP_OK(hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking));
    for (auto& e : b->ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipStream_t c = b->cap;
    HIP_OK(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
    const char* where = "fork";
    bool ok = hipEventRecord(b->ev[count], c) == hipSuccess;
    for (int32_t i = 0; i < count && ok; i++) {
      where = "branch wait";
      ok = hipStreamWaitEvent(b->side[i], b->ev[count], 0) == hipSuccess;
      if (ok) { where = "branch work"; ok = resetup_levels(b->hs[i], b->side[i]) == EMIN_OK; }
      if (ok) { where = "branch record"; ok = hipEventRecord(b->ev[i], b->side[i]) == hipSuccess; }
      if (ok) { where = "join"; ok = hipStreamWaitEvent(c, b->ev[i], 0) == hipSuccess; }
    }
    hipError_t ec = hipStreamEndCapture(c, &b->graph);
    if (!ok) throw Error(EMIN_ERR_DEVICE, std::string("graph capture failed at ") + where);
    if (ec != hipSuccess)
      throw Error(EMIN_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  } catch (const Error& e) {
    set_last_error(e.what());
    delete b;
    return e.code;
  } catch (...) {
    delete b;
    return EMIN_ERR_DEVICE;
  }
  *out = b;
  return EMIN_OK;
}

emin_status emin_batch_run(emin_batch_t* b, void* stream) {
  if (!b || !b->exec) return EMIN_ERR_ARG;
  return hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? EMIN_OK
             : EMIN_ERR_DEVICE;
}

void emin_batch_destroy(emin_batch_t* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  delete b;
}

}  // extern "C"
