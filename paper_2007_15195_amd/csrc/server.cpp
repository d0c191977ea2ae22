// Request loop with continuous batching (vecchia_server_*, vecchia_submit/poll).
//
// The log-CDF requests come from repeated likelihood evaluations (one Gaussian
// CDF per temporal replicate and per scale-mixture node, Section 4, eqs.
// (9)-(11)), with mixed D and m. At creation the server reserves one device
// arena of hbm_budget_bytes and max_slots execution slots, each a stream with
// two side streams. submit() validates and sizes the request (no GPU work) and
// queues it. The scheduler of scheduler.h forms groups on its worker thread:
// whenever a slot is free it takes the queued requests in arrival order, as
// many as fit in the arena, up to 64 requests and 6e10 SOV steps (one request
// at least). The device executor below runs a group as one batch: one set-up
// launch, one QMC launch per conditioning-set size over every request of the
// group, one finalize. Groups on different slots overlap on the device;
// finished groups are retired by event query. A request's result depends only
// on its own inputs (shifts are keyed by plan-order term indices and every
// reduction has a fixed order), so it is the same alone, in any group and in
// any mix.
#include <cmath>
#include <cstring>

#include "scheduler.h"

#include "arena.h"
#include "runtime.h"

using namespace vecchia;

namespace {

constexpr int kMaxGroup = 64;   // requests per group (the slots' staging is sized for it)

struct Request : SchedItem {
  vecchia_plan_s* plan = nullptr;
  const double* x = nullptr;
  double scale = 1.0;
  vecchia_cov cov{};
  bool has_cov = false;
  vecchia_qmc q{};
};

Request* req(SchedItem* it) { return static_cast<Request*>(it); }

// Requests admitted together: one batch, one arena block.
struct Group {
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

// Runs groups on the device. Called only from the scheduler's worker thread,
// under its lock.
class DeviceExecutor : public Executor {
 public:
  int device = 0;
  size_t budget = 0;
  char* d_arena = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slot;

  int slots() const override { return (int)slot.size(); }
  size_t largest_free() const override { return arena->largest_free(); }
  void on_worker_start() override { hipSetDevice(device); }
  int start(int s, SchedItem* const* items, int n) override;
  bool finished(int s, SchedItem* const* items, int n) override;

 private:
  static void settle(Request* r, vecchia_status st, const std::string& msg) {
    r->status = st;
    r->msg = msg;
    r->plan->inflight.fetch_sub(1);
  }
};

int DeviceExecutor::start(int s, SchedItem* const* items, int n) {
  Slot& sl = slot[s];
  std::unique_ptr<Batch> b;
  size_t off = 0;
  int k = n < kMaxGroup ? n : kMaxGroup;
  while (k > 0) {
    std::vector<vecchia_plan_s*> plans;
    std::vector<vecchia_qmc> qmcs;
    for (int j = 0; j < k; ++j) {
      plans.push_back(req(items[j])->plan);
      qmcs.push_back(req(items[j])->q);
    }
    if (Batch::create(plans, qmcs, &b) != VECCHIA_OK) {
      // requests were validated one by one at submit; a group fails only on
      // a batch-wide limit, so the first request runs alone
      if (k > 1) { k = 1; continue; }
      settle(req(items[0]), VECCHIA_E_INVALID, vecchia_last_error());
      return -1;
    }
    if (arena->alloc(b->workspace_bytes(), &off)) break;
    if (k == 1) return 0;   // wait for memory
    k = k / 2;              // the group's own layout did not fit: a shorter prefix
  }
  std::vector<const double*> xs(k);
  std::vector<double> scales(k);
  std::vector<vecchia_cov> covs(k);
  std::vector<uint64_t> seeds(k);
  for (int j = 0; j < k; ++j) {
    Request* r = req(items[j]);
    xs[j] = r->x;
    scales[j] = r->scale;
    covs[j] = r->has_cov ? r->cov : r->plan->cov;
    seeds[j] = r->q.seed;
  }
  b->bind_external(d_arena + off, sl.h_stage, sl.side[0], sl.side[1]);
  b->set_x_ptrs(xs);
  vecchia_status st = b->run(xs[0], scales.data(), covs.data(), sl.d_out, nullptr, seeds.data(), sl.stream);
  hipError_t e = hipSuccess;
  if (st == VECCHIA_OK) {
    e = hipMemcpyAsync(sl.h_res, sl.d_out, 2 * (size_t)k * sizeof(double), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&sl.h_res[2 * kMaxGroup], b->device_bad_terms(), (size_t)k * sizeof(int64_t),
                         hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.ev, sl.stream);
  }
  if (st != VECCHIA_OK || e != hipSuccess) {
    const std::string msg = st != VECCHIA_OK ? std::string(vecchia_last_error()) : hipGetErrorString(e);
    for (int j = 0; j < k; ++j) settle(req(items[j]), st != VECCHIA_OK ? st : VECCHIA_E_HIP, msg);
    hipStreamSynchronize(sl.stream);   // nothing enqueued may still read the block
    arena->release(off, b->workspace_bytes());
    return -k;
  }
  sl.grp.reset(new Group());
  sl.grp->bytes = b->workspace_bytes();
  sl.grp->off = off;
  sl.grp->batch = std::move(b);
  return k;
}

bool DeviceExecutor::finished(int s, SchedItem* const* items, int n) {
  Slot& sl = slot[s];
  const hipError_t q = hipEventQuery(sl.ev);
  if (q == hipErrorNotReady) return false;
  for (int j = 0; j < n; ++j) {
    Request* r = req(items[j]);
    if (q != hipSuccess) {
      settle(r, VECCHIA_E_HIP, std::string("request failed on the device: ") + hipGetErrorString(q));
      continue;
    }
    r->logF = sl.h_res[2 * j];
    r->se = sl.h_res[2 * j + 1];
    int64_t bad;
    std::memcpy(&bad, &sl.h_res[2 * kMaxGroup + j], sizeof(bad));
    if (bad != INT64_MAX) {
      r->bad = bad;
      settle(r, VECCHIA_E_NOT_PD, "covariance block of plan term " + std::to_string(bad) + " is not positive definite");
    } else {
      settle(r, VECCHIA_OK, "");
    }
  }
  arena->release(sl.grp->off, sl.grp->bytes);
  sl.grp.reset();
  return true;
}

}  // namespace

struct vecchia_server_s {
  DeviceExecutor ex;
  std::unique_ptr<Scheduler> sched;
};

extern "C" {

static void free_slots(DeviceExecutor& ex) {
  for (Slot& sl : ex.slot) {
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
  hipFree(ex.d_arena);
}

vecchia_status vecchia_server_create(size_t hbm_budget_bytes, int32_t max_slots, vecchia_server_t* out) {
  if (!out) return set_error(VECCHIA_E_INVALID, "null pointer");
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64)
    return set_error(VECCHIA_E_INVALID, "budget must be > 0 and max_slots in 1..64");
  auto* S = new (std::nothrow) vecchia_server_s();
  if (!S) return set_error(VECCHIA_E_NOMEM, "host allocation");
  DeviceExecutor& ex = S->ex;
  hipGetDevice(&ex.device);
  ex.budget = (hbm_budget_bytes + 255) / 256 * 256;
  hipError_t e = hipMalloc(&ex.d_arena, ex.budget);
  if (e != hipSuccess) {
    delete S;
    return hip_error(e, "server arena");
  }
  ex.arena.reset(new Arena(ex.budget));
  ex.slot.resize(max_slots);
  for (Slot& sl : ex.slot) {
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
    free_slots(ex);
    delete S;
    return st;
  }
  GroupLimits lim;
  lim.max_group = kMaxGroup;
  lim.max_steps = 6e10;   // about 60 ms of the device
  S->sched.reset(new Scheduler(&ex, lim));
  S->sched->start_worker();
  *out = S;
  return VECCHIA_OK;
}

vecchia_status vecchia_submit(vecchia_server_t server, vecchia_plan_t plan, const double* x_dev, double scale,
                              const vecchia_cov* cov_override, const vecchia_qmc* q, uint64_t* ticket) {
  if (!server || !plan || !q || !ticket || !x_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  if (!(std::isfinite(scale) && scale > 0)) return set_error(VECCHIA_E_INVALID, "scale must be finite and > 0");
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != server->ex.device || plan->device != server->ex.device)
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
  if (r->bytes > server->ex.budget)
    return set_error(VECCHIA_E_NOMEM, "request needs " + std::to_string(r->bytes) + " bytes, budget is " +
                                          std::to_string(server->ex.budget));
  plan->inflight.fetch_add(1);
  std::unique_ptr<SchedItem> item(r.release());
  if (!server->sched->submit(item, ticket)) {
    plan->inflight.fetch_sub(1);
    return set_error(VECCHIA_E_INVALID, "server is shutting down");
  }
  return VECCHIA_OK;
}

vecchia_status vecchia_poll(vecchia_server_t server, uint64_t ticket, double* logF, double* se, int32_t* done,
                            double* latency_s) {
  if (!server || !done) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::unique_ptr<SchedItem> r;
  const Scheduler::PollResult pr = server->sched->poll(ticket, &r);
  if (pr == Scheduler::kUnknown) {
    *done = 0;
    return set_error(VECCHIA_E_INVALID, "unknown ticket " + std::to_string(ticket));
  }
  if (pr == Scheduler::kPending) {
    *done = 0;
    return VECCHIA_OK;
  }
  *done = 1;
  if (logF) *logF = r->logF;
  if (se) *se = r->se;
  if (latency_s) *latency_s = r->latency;
  if (r->status != VECCHIA_OK) return set_error((vecchia_status)r->status, r->msg);
  return VECCHIA_OK;
}

vecchia_status vecchia_server_destroy(vecchia_server_t server) {
  if (!server) return set_error(VECCHIA_E_INVALID, "null server");
  server->sched->shutdown();   // queued and in-flight requests drain first
  server->sched.reset();
  free_slots(server->ex);
  delete server;
  return VECCHIA_OK;
}

}  // extern "C"
