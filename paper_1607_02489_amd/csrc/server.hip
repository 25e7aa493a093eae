// Serving loop for setup requests (e.g. successive Picard linearisations):
// requests queue in arrival order and are admitted when a worker slot is
// free and their device-memory estimate fits the budget; each worker builds
// the hierarchy on its own stream, so admitted requests overlap on the GPU
// (Alg. 3 is one workgroup, the rest of the chip serves the other requests).
// Results stay on the device until released.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  int64_t id = 0;
  emin_system_t sys{};
  emin_params_t prm{};
  int32_t nlevels = 2;
  int64_t min_dofs = 0;
  int64_t estimate = 0, held = 0;
  Clock::time_point t_submit, t_start, t_done;
  emin_hierarchy_t* result = nullptr;
  emin_status status = EMIN_OK;
  bool done = false;
  bool started = false;
};

// device bytes one request is expected to hold: pattern handles, workspace
// and coarse values scale with the input's nonzeros (measured ratio with
// headroom), plus one arena chunk per level; the A^T A energy operator of
// the velocity block (EMIN_FLAG_ENERGY_ATA) has about three times the
// nonzeros of the symmetric one in 2-D and more in 3-D, so the velocity
// block's share is scaled by the operator's expected fill
int64_t estimate_bytes(const emin_system_t& s, const emin_params_t& prm, int32_t nlevels) {
  const int64_t fill = (prm.flags & EMIN_FLAG_ENERGY_ATA) ? (s.dim == 3 ? 6 : 3) : 1;
  const int64_t nz = fill * s.Ahat.nnz + s.Bdiv.nnz;
  return 64 * nz + 256 * (s.Ahat.nrows + s.Bdiv.nrows) + (int64_t)(nlevels + 1) * (64ll << 20);
}

}  // namespace

struct emin_server_s {
  int64_t budget = 0;
  int64_t in_use = 0;
  int32_t running = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<int64_t, Request*> reqs;
  int64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;

  void worker() {
    hipStream_t s = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    while (true) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return stop || (!queue.empty() && in_use + queue.front()->estimate <= budget);
        });
        if (stop) break;
        r = queue.front();
        queue.pop_front();
        r->started = true;
        in_use += r->estimate;
        r->held = r->estimate;
        running++;
      }
      r->t_start = Clock::now();
      emin_status st = have_stream ? EMIN_OK : EMIN_ERR_DEVICE;
      if (st == EMIN_OK)
        st = emin_hierarchy_build(&r->sys, &r->prm, r->nlevels, r->min_dofs, s, &r->result);
      if (st == EMIN_OK && hipStreamSynchronize(s) != hipSuccess) st = EMIN_ERR_DEVICE;
      const int64_t actual = st == EMIN_OK ? emin_hierarchy_device_bytes(r->result) : 0;
      {
        std::lock_guard<std::mutex> lk(mu);
        in_use += actual - r->held;
        r->held = actual;
        r->status = st;
        r->t_done = Clock::now();
        r->done = true;
        running--;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(s);
  }
};

extern "C" {

emin_status emin_server_create(int64_t budget_bytes, int32_t max_slots, emin_server_t** out) {
  if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > 64) return EMIN_ERR_ARG;
  emin_server_t* srv = new emin_server_s();
  srv->budget = budget_bytes;
  for (int32_t i = 0; i < max_slots; i++) srv->workers.emplace_back([srv] { srv->worker(); });
  *out = srv;
  return EMIN_OK;
}

emin_status emin_server_submit(emin_server_t* srv, const emin_system_t* sys,
                               const emin_params_t* prm, int32_t nlevels, int64_t min_dofs,
                               int64_t* ticket) {
  if (!srv || !sys || !prm || !ticket || nlevels < 1) return EMIN_ERR_ARG;
  Request* r = new Request();
  r->sys = *sys;
  r->prm = *prm;
  r->nlevels = nlevels;
  r->min_dofs = min_dofs;
  r->estimate = estimate_bytes(*sys, *prm, nlevels);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (r->estimate > srv->budget) {
      delete r;
      return EMIN_ERR_BUDGET;
    }
    r->id = srv->next_id++;
    srv->reqs[r->id] = r;
    srv->queue.push_back(r);
    *ticket = r->id;
  }
  srv->cv_work.notify_all();
  return EMIN_OK;
}

emin_status emin_server_poll(emin_server_t* srv, int64_t ticket, int32_t* done) {
  if (!srv || !done) return EMIN_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return EMIN_ERR_ARG;
  *done = it->second->done ? 1 : 0;
  return EMIN_OK;
}

emin_status emin_server_wait(emin_server_t* srv, int64_t ticket, emin_hierarchy_t** result,
                             double* queue_ms, double* run_ms) {
  if (!srv) return EMIN_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return EMIN_ERR_ARG;
  Request* r = it->second;
  srv->cv_done.wait(lk, [&] { return r->done; });
  if (result) *result = r->result;
  using ms = std::chrono::duration<double, std::milli>;
  if (queue_ms) *queue_ms = ms(r->t_start - r->t_submit).count();
  if (run_ms) *run_ms = ms(r->t_done - r->t_start).count();
  return r->status;
}

emin_status emin_server_cancel(emin_server_t* srv, int64_t ticket, int32_t* cancelled) {
  if (!srv) return EMIN_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return EMIN_ERR_ARG;
    Request* r = it->second;
    bool hit = false;
    if (!r->started) {
      for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
        if (*q == r) {
          srv->queue.erase(q);
          hit = true;
          break;
        }
    }
    if (hit) {
      r->status = EMIN_ERR_CANCELLED;
      r->t_start = r->t_done = Clock::now();
      r->done = true;
    }
    if (cancelled) *cancelled = hit ? 1 : 0;
  }
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();   // the next queued request may fit now
  return EMIN_OK;
}

emin_status emin_server_release(emin_server_t* srv, int64_t ticket) {
  if (!srv) return EMIN_ERR_ARG;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || !it->second->done) return EMIN_ERR_ARG;
    r = it->second;
    srv->reqs.erase(it);
    srv->in_use -= r->held;
  }
  emin_hierarchy_destroy(r->result);
  delete r;
  srv->cv_work.notify_all();
  return EMIN_OK;
}

emin_status emin_server_stats(emin_server_t* srv, int64_t* in_use, int32_t* queued,
                              int32_t* running) {
  if (!srv) return EMIN_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (in_use) *in_use = srv->in_use;
  if (queued) *queued = (int32_t)srv->queue.size();
  if (running) *running = srv->running;
  return EMIN_OK;
}

void emin_server_destroy(emin_server_t* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  for (auto& kv : srv->reqs) {
    emin_hierarchy_destroy(kv.second->result);
    delete kv.second;
  }
  delete srv;
}

}  // extern "C"
