// Request loop with continuous batching (vecchia_server_*, vecchia_submit/poll).
//
// The log-CDF requests come from repeated likelihood evaluations (one Gaussian
// CDF per temporal replicate and per scale-mixture node, Section 4, eqs.
// (9)-(11)), with mixed D and m. At creation the server reserves one device
// arena of hbm_budget_bytes and max_slots execution slots, each with its own
// stream. submit() lays the request out (no GPU work) and queues it. A
// scheduler thread admits queued requests in arrival order whenever a slot is
// free and the request's workspace fits in the arena, enqueues its kernels on
// the slot's stream at once (so admitted requests overlap on the device), and
// retires requests whose completion event has fired. A request's result depends
// only on its own inputs: shifts are keyed by plan-order term indices and every
// reduction has a fixed order.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "arena.h"
#include "runtime.h"

using namespace vecchia;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  vecchia_plan_s* plan = nullptr;
  const double* x = nullptr;
  double scale = 1.0;
  vecchia_cov cov{};
  bool has_cov = false;
  vecchia_qmc q{};
  std::unique_ptr<Batch> batch;
  size_t bytes = 0;
  size_t arena_off = 0;
  Clock::time_point t_submit;
  double latency = 0.0;
  double logF = 0.0, se = 0.0;
  int64_t bad = -1;
  vecchia_status status = VECCHIA_OK;
  std::string msg;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  double* d_out = nullptr;       // {log F, SE}
  double* h_res = nullptr;       // pinned {log F, SE, bad term (as int64 bits)}
  InstDesc* h_stage = nullptr;   // pinned descriptor staging
  Request* req = nullptr;
};

}  // namespace

struct vecchia_server_s {
  int device = 0;
  size_t budget = 0;
  char* d_arena = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slots;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  int running = 0;

  void loop();
  bool retire_done();     // under mu
  void admit();           // under mu
};

bool vecchia_server_s::retire_done() {
  bool any = false;
  for (Slot& sl : slots) {
    if (!sl.req) continue;
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) continue;
    Request* r = sl.req;
    if (q != hipSuccess) {
      r->status = VECCHIA_E_HIP;
      r->msg = std::string("request failed on the device: ") + hipGetErrorString(q);
    } else {
      r->logF = sl.h_res[0];
      r->se = sl.h_res[1];
      int64_t bad;
      std::memcpy(&bad, &sl.h_res[2], sizeof(bad));
      if (bad != INT64_MAX) {
        r->bad = bad;
        r->status = VECCHIA_E_NOT_PD;
        r->msg = "covariance block of plan term " + std::to_string(bad) + " is not positive definite";
      }
    }
    r->latency = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
    r->done = true;
    arena->release(r->arena_off, r->bytes);
    r->batch.reset();
    r->plan->inflight.fetch_sub(1);
    sl.req = nullptr;
    --running;
    any = true;
  }
  return any;
}

void vecchia_server_s::admit() {
  while (!pending.empty()) {
    Slot* free_slot = nullptr;
    for (Slot& sl : slots)
      if (!sl.req) { free_slot = &sl; break; }
    if (!free_slot) return;
    Request* r = pending.front();
    size_t off = 0;
    if (!arena->alloc(r->bytes, &off)) return;   // wait for memory; keep arrival order
    pending.pop_front();
    r->arena_off = off;
    r->batch->bind_external(d_arena + off, free_slot->h_stage);
    const uint64_t seed = r->q.seed;
    vecchia_status st = r->batch->run(r->x, &r->scale, r->has_cov ? &r->cov : nullptr, free_slot->d_out,
                                      nullptr, &seed, free_slot->stream);
    hipError_t e = hipSuccess;
    if (st == VECCHIA_OK) {
      e = hipMemcpyAsync(free_slot->h_res, free_slot->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost,
                         free_slot->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&free_slot->h_res[2], r->batch->device_bad_terms(), sizeof(int64_t),
                           hipMemcpyDeviceToHost, free_slot->stream);
      if (e == hipSuccess) e = hipEventRecord(free_slot->ev, free_slot->stream);
    }
    if (st != VECCHIA_OK || e != hipSuccess) {
      r->status = st != VECCHIA_OK ? st : VECCHIA_E_HIP;
      r->msg = st != VECCHIA_OK ? std::string(vecchia_last_error()) : hipGetErrorString(e);
      r->done = true;
      r->latency = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
      arena->release(off, r->bytes);
      r->batch.reset();
      r->plan->inflight.fetch_sub(1);
      continue;
    }
    free_slot->req = r;
    ++running;
  }
}

void vecchia_server_s::loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    retire_done();
    admit();
    if (stop && pending.empty() && running == 0) break;
    if (running == 0 && pending.empty()) {
      cv.wait(lk);
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

extern "C" {

vecchia_status vecchia_server_create(size_t hbm_budget_bytes, int32_t max_slots, vecchia_server_t* out) {
  if (!out) return set_error(VECCHIA_E_INVALID, "null pointer");
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64)
    return set_error(VECCHIA_E_INVALID, "budget must be > 0 and max_slots in 1..64");
  auto* S = new (std::nothrow) vecchia_server_s();
  if (!S) return set_error(VECCHIA_E_NOMEM, "host allocation");
  hipGetDevice(&S->device);
  S->budget = (hbm_budget_bytes + 255) / 256 * 256;
  hipError_t e = hipMalloc(&S->d_arena, S->budget);
  if (e != hipSuccess) {
    delete S;
    return hip_error(e, "server arena");
  }
  S->arena.reset(new Arena(S->budget));
  S->slots.resize(max_slots);
  for (Slot& sl : S->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&sl.d_out, 2 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_res), 4 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_stage), sizeof(InstDesc), hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    vecchia_status st = hip_error(e, "server slots");
    for (Slot& sl : S->slots) {
      if (sl.stream) hipStreamDestroy(sl.stream);
      if (sl.ev) hipEventDestroy(sl.ev);
      hipFree(sl.d_out);
      if (sl.h_res) hipHostFree(sl.h_res);
      if (sl.h_stage) hipHostFree(sl.h_stage);
    }
    hipFree(S->d_arena);
    delete S;
    return st;
  }
  S->worker = std::thread([S] { S->loop(); });
  *out = S;
  return VECCHIA_OK;
}

vecchia_status vecchia_submit(vecchia_server_t server, vecchia_plan_t plan, const double* x_dev, double scale,
                              const vecchia_cov* cov_override, const vecchia_qmc* q, uint64_t* ticket) {
  if (!server || !plan || !q || !ticket || !x_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  if (!(std::isfinite(scale) && scale > 0)) return set_error(VECCHIA_E_INVALID, "scale must be finite and > 0");
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != server->device || plan->device != server->device)
    return set_error(VECCHIA_E_INVALID, "plan, server and current device differ");
  std::string why;
  if (!valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (cov_override) {
    if (!valid_cov(*cov_override, &why)) return set_error(VECCHIA_E_INVALID, why);
    if (!plan->matrix && (cov_override->family != plan->cov.family ||
                          (cov_override->family == VECCHIA_COV_MATERN && cov_override->nu != plan->cov.nu)))
      return set_error(VECCHIA_E_INVALID, "covariance override must keep the plan's family and nu");
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return set_error(VECCHIA_E_NOMEM, "host allocation");
  r->plan = plan;
  r->x = x_dev;
  r->scale = scale;
  r->has_cov = cov_override != nullptr;
  if (cov_override) r->cov = *cov_override;
  r->q = *q;
  vecchia_status st = Batch::create({plan}, {*q}, &r->batch);
  if (st != VECCHIA_OK) return st;
  r->bytes = r->batch->workspace_bytes();
  if (r->bytes > server->budget)
    return set_error(VECCHIA_E_NOMEM, "request needs " + std::to_string(r->bytes) + " bytes, budget is " +
                                          std::to_string(server->budget));
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(server->mu);
    if (server->stop) return set_error(VECCHIA_E_INVALID, "server is shutting down");
    r->ticket = server->next_ticket++;
    *ticket = r->ticket;
    plan->inflight.fetch_add(1);
    server->pending.push_back(r.get());
    server->reqs.emplace(r->ticket, std::move(r));
  }
  server->cv.notify_one();
  return VECCHIA_OK;
}

vecchia_status vecchia_poll(vecchia_server_t server, uint64_t ticket, double* logF, double* se, int32_t* done,
                            double* latency_s) {
  if (!server || !done) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::lock_guard<std::mutex> lk(server->mu);
  auto it = server->reqs.find(ticket);
  if (it == server->reqs.end()) {
    *done = 0;
    return set_error(VECCHIA_E_INVALID, "unknown ticket " + std::to_string(ticket));
  }
  Request* r = it->second.get();
  if (!r->done) {
    *done = 0;
    return VECCHIA_OK;
  }
  *done = 1;
  if (logF) *logF = r->logF;
  if (se) *se = r->se;
  if (latency_s) *latency_s = r->latency;
  const vecchia_status st = r->status;
  const std::string msg = r->msg;
  server->reqs.erase(it);
  if (st != VECCHIA_OK) return set_error(st, msg);
  return VECCHIA_OK;
}

vecchia_status vecchia_server_destroy(vecchia_server_t server) {
  if (!server) return set_error(VECCHIA_E_INVALID, "null server");
  {
    std::lock_guard<std::mutex> lk(server->mu);
    server->stop = true;
  }
  server->cv.notify_one();
  if (server->worker.joinable()) server->worker.join();
  for (Slot& sl : server->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.ev) hipEventDestroy(sl.ev);
    hipFree(sl.d_out);
    if (sl.h_res) hipHostFree(sl.h_res);
    if (sl.h_stage) hipHostFree(sl.h_stage);
  }
  hipFree(server->d_arena);
  delete server;
  return VECCHIA_OK;
}

}  // extern "C"
