// Request scheduling of the serving loop, independent of the device.
//
// The serving loop answers the repeated log-CDF evaluations of Section 4 (one
// Gaussian CDF per temporal replicate and per scale-mixture node, eqs.
// (9)-(11)). This header holds its host-side policy: a FIFO of requests, a
// worker thread that forms groups from the FIFO's prefix and hands them to an
// Executor, and the ticket table that submit / poll share. It has no HIP
// dependency, so the same code runs against the device executor of server.cpp
// and against a simulated executor under ThreadSanitizer on the host.
//
// Threading: submit(), poll() and shutdown() may be called from any thread.
// The worker thread is the only caller of the Executor; it calls it with the
// scheduler's mutex held, so an Executor needs no locking of its own for state
// that only those calls touch.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace vecchia {

// One queued request. The executor subclasses it with what it needs to run the
// request; the scheduler owns it from submit until poll hands it back.
struct SchedItem {
  virtual ~SchedItem() = default;
  uint64_t ticket = 0;
  size_t bytes = 0;       // device workspace of the request alone (an upper bound of its share in a group)
  double steps = 0.0;     // SOV steps: the request's device work
  std::chrono::steady_clock::time_point t_submit;
  // results, written by the executor (or by the scheduler on shutdown paths)
  double logF = 0.0, se = 0.0;
  int64_t bad = -1;
  int status = 0;         // a vecchia_status value; 0 is OK
  std::string msg;
  double latency = 0.0;   // submit to completion, seconds
  bool done = false;
};

struct GroupLimits {
  int max_group = 64;        // requests per group
  double max_steps = 6e10;   // SOV steps per group, unless its first request alone has more
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual int slots() const = 0;
  // Largest block of device workspace that one group could take now.
  virtual size_t largest_free() const = 0;
  // Start items[0 .. n) as one group on the free slot `slot`. Returns k > 0:
  // items[0 .. k) run as the slot's group (k < n: only a shorter prefix fits);
  // 0: nothing fits now, retry after a group retires; -k < 0: items[0 .. k)
  // failed to start (the executor has set their status and message) and leave
  // the queue, and the slot stays free.
  virtual int start(int slot, SchedItem* const* items, int n) = 0;
  // Non-blocking. True once the group on `slot` has finished; the executor has
  // then written every item's results and status and released its resources.
  virtual bool finished(int slot, SchedItem* const* items, int n) = 0;
  // First call on the worker thread (for example, to make a device current).
  virtual void on_worker_start() {}
};

class Scheduler {
 public:
  Scheduler(Executor* ex, GroupLimits lim) : ex_(ex), lim_(lim), on_slot_(ex->slots()) {}
  ~Scheduler() { shutdown(); }
  Scheduler(const Scheduler&) = delete;
  Scheduler& operator=(const Scheduler&) = delete;

  void start_worker() { worker_ = std::thread([this] { loop(); }); }

  // Queues the item and assigns its ticket. False (item untouched) once
  // shutdown has begun.
  bool submit(std::unique_ptr<SchedItem>& item, uint64_t* ticket) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) return false;
      item->ticket = next_ticket_++;
      item->t_submit = std::chrono::steady_clock::now();
      *ticket = item->ticket;
      pending_.push_back(item.get());
      items_.emplace(item->ticket, std::move(item));
    }
    cv_.notify_one();
    return true;
  }

  enum PollResult { kUnknown = 0, kPending = 1, kDone = 2 };
  // kDone hands the finished item back (its ticket is then released).
  PollResult poll(uint64_t ticket, std::unique_ptr<SchedItem>* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = items_.find(ticket);
    if (it == items_.end()) return kUnknown;
    if (!it->second->done) return kPending;
    *out = std::move(it->second);
    items_.erase(it);
    return kDone;
  }

  // Stops admissions of new requests, runs every queued and in-flight request
  // to completion, and joins the worker. Idempotent.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_one();
    if (worker_.joinable()) worker_.join();
  }

 private:
  void complete(SchedItem* r) {
    r->latency = std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_submit).count();
    r->done = true;
  }

  bool retire() {
    bool any = false;
    for (int s = 0; s < (int)on_slot_.size(); ++s) {
      std::vector<SchedItem*>& g = on_slot_[s];
      if (g.empty() || !ex_->finished(s, g.data(), (int)g.size())) continue;
      for (SchedItem* r : g) complete(r);
      g.clear();
      --running_;
      any = true;
    }
    return any;
  }

  void admit() {
    while (!pending_.empty()) {
      int slot = -1;
      for (int s = 0; s < (int)on_slot_.size(); ++s)
        if (on_slot_[s].empty()) { slot = s; break; }
      if (slot < 0) return;
      // a prefix of the queue, so arrival order is kept
      const size_t room = ex_->largest_free();
      int n = 0;
      size_t bytes = 0;
      double steps = 0.0;
      for (SchedItem* r : pending_) {
        if (n == lim_.max_group) break;
        if (n > 0 && (steps + r->steps > lim_.max_steps || bytes + r->bytes > room)) break;
        bytes += r->bytes;
        steps += r->steps;
        ++n;
      }
      std::vector<SchedItem*> head(pending_.begin(), pending_.begin() + n);
      const int k = ex_->start(slot, head.data(), n);
      if (k == 0) return;   // wait for a group to retire
      const int used = k > 0 ? k : -k;
      pending_.erase(pending_.begin(), pending_.begin() + used);
      if (k > 0) {
        on_slot_[slot].assign(head.begin(), head.begin() + used);
        ++running_;
      } else {
        for (int j = 0; j < used; ++j) complete(head[j]);
      }
    }
  }

  void loop() {
    ex_->on_worker_start();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      retire();
      admit();
      if (stop_ && pending_.empty() && running_ == 0) break;
      if (running_ == 0 && pending_.empty()) {
        cv_.wait(lk);
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
  }

  Executor* ex_;
  GroupLimits lim_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::thread worker_;
  std::deque<SchedItem*> pending_;
  std::unordered_map<uint64_t, std::unique_ptr<SchedItem>> items_;
  std::vector<std::vector<SchedItem*>> on_slot_;
  bool stop_ = false;
  uint64_t next_ticket_ = 1;
  int running_ = 0;
};

}  // namespace vecchia
