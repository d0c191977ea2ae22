// Request loop with continuous batching (vecchia_server_*, vecchia_submit/poll).
//
// The log-CDF requests come from repeated likelihood evaluations (one Gaussian
// CDF per temporal replicate and per scale-mixture node, Section 4, eqs.
// (9)-(11)), with mixed D and m. At creation the server reserves one device
// arena of hbm_budget_bytes and max_slots execution slots, each a stream with
// two side streams. submit() validates and sizes the request (no GPU work) and
// queues it. A scheduler thread forms groups: whenever a slot is free it takes
// the queued requests in arrival order, as many as fit in the arena, up to
// kMaxGroup requests and kGroupSteps SOV steps (one request at least), and runs
// them as one batch: one set-up launch, one QMC launch per conditioning-set size
// over every request of the group, one finalize. Groups on different slots
// overlap on the device; finished groups are retired by event query. A
// request's result depends only on its own inputs (shifts are keyed by
// plan-order term indices and every reduction has a fixed order), so it is the
// same alone, in any group and in any mix.
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

constexpr int kMaxGroup = 64;            // requests per group
constexpr double kGroupSteps = 6e10;     // SOV steps per group (about 60 ms of the device), unless one request has more

struct Request {
  uint64_t ticket = 0;
  vecchia_plan_s* plan = nullptr;
  const double* x = nullptr;
  double scale = 1.0;
  vecchia_cov cov{};
  bool has_cov = false;
  vecchia_qmc q{};
  size_t bytes = 0;        // workspace of the request alone (an upper bound of its share in a group)
  double steps = 0.0;      // SOV steps of the request
  Clock::time_point t_submit;
  double latency = 0.0;
  double logF = 0.0, se = 0.0;
  int64_t bad = -1;
  vecchia_status status = VECCHIA_OK;
  std::string msg;
  bool done = false;
};

// Requests admitted together: one batch, one arena block.
struct Group {
  std::vector<Request*> reqs;
  std::unique_ptr<Batch> batch;
  size_t off = 0, bytes = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev = nullptr;
  double* d_out = nullptr;       // kMaxGroup x {log F, SE}
  double* h_res = nullptr;       // pinned: kMaxGroup x {log F, SE}, then kMaxGroup bad terms (int64)
  InstDesc* h_stage = nullptr;   // pinned descriptor staging, kMaxGroup entries
  std::unique_ptr<Group> grp;
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
  void finish(Request* r, vecchia_status st, const std::string& msg);
};

void vecchia_server_s::finish(Request* r, vecchia_status st, const std::string& msg) {
  r->status = st;
  r->msg = msg;
  r->latency = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
  r->done = true;
  r->plan->inflight.fetch_sub(1);
}

bool vecchia_server_s::retire_done() {
  bool any = false;
  for (Slot& sl : slots) {
    if (!sl.grp) continue;
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) continue;
    Group& g = *sl.grp;
    const int n = (int)g.reqs.size();
    for (int j = 0; j < n; ++j) {
      Request* r = g.reqs[j];
      if (q != hipSuccess) {
        finish(r, VECCHIA_E_HIP, std::string("request failed on the device: ") + hipGetErrorString(q));
        continue;
      }
      r->logF = sl.h_res[2 * j];
      r->se = sl.h_res[2 * j + 1];
      int64_t bad;
      std::memcpy(&bad, &sl.h_res[2 * kMaxGroup + j], sizeof(bad));
      if (bad != INT64_MAX) {
        r->bad = bad;
        finish(r, VECCHIA_E_NOT_PD, "covariance block of plan term " + std::to_string(bad) + " is not positive definite");
      } else {
        finish(r, VECCHIA_OK, "");
      }
    }
    arena->release(g.off, g.bytes);
    sl.grp.reset();
    --running;
    any = true;
  }
  return any;
}

void vecchia_server_s::admit() {
  while (!pending.empty()) {
    Slot* sl = nullptr;
    for (Slot& c : slots)
      if (!c.grp) { sl = &c; break; }
    if (!sl) return;
    // a prefix of the queue: arrival order is kept
    size_t n = 0;
    size_t est = 0;
    double steps = 0.0;
    const size_t room = arena->largest_free();
    for (Request* r : pending) {
      if (n == (size_t)kMaxGroup) break;
      if (n > 0 && (steps + r->steps > kGroupSteps || est + r->bytes > room)) break;
      est += r->bytes;
      steps += r->steps;
      ++n;
    }
    std::unique_ptr<Group> g;
    size_t off = 0;
    while (n > 0) {
      std::vector<vecchia_plan_s*> plans;
      std::vector<vecchia_qmc> qmcs;
      for (size_t j = 0; j < n; ++j) {
        plans.push_back(pending[j]->plan);
        qmcs.push_back(pending[j]->q);
      }
      std::unique_ptr<Batch> b;
      if (Batch::create(plans, qmcs, &b) != VECCHIA_OK) {
        // requests were validated one by one at submit; a group fails only on
        // a batch-wide limit, so the first request runs alone
        if (n > 1) { n = 1; continue; }
        Request* r = pending.front();
        pending.pop_front();
        finish(r, VECCHIA_E_INVALID, vecchia_last_error());
        break;
      }
      if (arena->alloc(b->workspace_bytes(), &off)) {
        g.reset(new Group());
        g->bytes = b->workspace_bytes();
        g->off = off;
        g->batch = std::move(b);
        break;
      }
      if (n == 1) return;   // wait for memory
      n = n / 2;            // the group's own layout did not fit: a shorter prefix
    }
    if (!g) continue;
    g->reqs.assign(pending.begin(), pending.begin() + n);
    pending.erase(pending.begin(), pending.begin() + n);
    std::vector<const double*> xs(n);
    std::vector<double> scales(n);
    std::vector<vecchia_cov> covs(n);
    std::vector<uint64_t> seeds(n);
    for (size_t j = 0; j < n; ++j) {
      Request* r = g->reqs[j];
      xs[j] = r->x;
      scales[j] = r->scale;
      covs[j] = r->has_cov ? r->cov : r->plan->cov;
      seeds[j] = r->q.seed;
    }
    Batch* b = g->batch.get();
    b->bind_external(d_arena + g->off, sl->h_stage, sl->side[0], sl->side[1]);
    b->set_x_ptrs(xs);
    vecchia_status st = b->run(xs[0], scales.data(), covs.data(), sl->d_out, nullptr, seeds.data(), sl->stream);
    hipError_t e = hipSuccess;
    if (st == VECCHIA_OK) {
      e = hipMemcpyAsync(sl->h_res, sl->d_out, 2 * n * sizeof(double), hipMemcpyDeviceToHost, sl->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&sl->h_res[2 * kMaxGroup], b->device_bad_terms(), n * sizeof(int64_t),
                           hipMemcpyDeviceToHost, sl->stream);
      if (e == hipSuccess) e = hipEventRecord(sl->ev, sl->stream);
    }
    if (st != VECCHIA_OK || e != hipSuccess) {
      const std::string msg = st != VECCHIA_OK ? std::string(vecchia_last_error()) : hipGetErrorString(e);
      for (Request* r : g->reqs) finish(r, st != VECCHIA_OK ? st : VECCHIA_E_HIP, msg);
      hipStreamSynchronize(sl->stream);   // nothing enqueued may still read the block
      arena->release(g->off, g->bytes);
      continue;
    }
    sl->grp = std::move(g);
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
    for (auto& sd : sl.side)
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&sd, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&sl.d_out, 2 * kMaxGroup * sizeof(double));
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_res), 3 * kMaxGroup * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_stage), kMaxGroup * sizeof(InstDesc), hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    vecchia_status st = hip_error(e, "server slots");
    for (Slot& sl : S->slots) {
      if (sl.stream) hipStreamDestroy(sl.stream);
      for (auto& sd : sl.side)
        if (sd) hipStreamDestroy(sd);
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
  std::unique_ptr<Batch> alone;
  vecchia_status st = Batch::create({plan}, {*q}, &alone);
  if (st != VECCHIA_OK) return st;
  r->bytes = alone->workspace_bytes();
  {
    double k = 0.0;
    for (int32_t v : plan->sov_dims()) k += v;
    r->steps = k * (double)q->n_points * q->n_shifts * (q->flags == VECCHIA_QMC_INDEPENDENT ? 2 : 1);
  }
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
    for (auto& sd : sl.side)
      if (sd) {
        hipStreamSynchronize(sd);
        hipStreamDestroy(sd);
      }
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
