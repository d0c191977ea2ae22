// Host check of the serving loop's scheduler (scheduler.h) against a simulated
// device, built with ThreadSanitizer (and, separately, AddressSanitizer and
// UBSan) by the CPU test suite.
//
// The simulated executor runs each slot's group on a "device" thread that
// publishes the group's results after a short random delay, as the real
// executor's event query does. Several client threads submit and poll at once,
// and one more polls random tickets. The check holds the scheduler to its
// contract:
//   - a group is a prefix of the queue: the tickets it starts are consecutive
//     and follow the last started ticket (arrival order is kept);
//   - a group has at most max_group requests, and more than max_steps SOV steps
//     only when it is a single request; its bytes fit the arena;
//   - every ticket completes once, with its own result, or with the injected
//     start failure when it heads a group;
//   - submit after shutdown is refused; shutdown drains queued requests.
// Prints "ok".
#include <atomic>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "arena.h"
#include "scheduler.h"

using namespace vecchia;

namespace {

constexpr int kSlots = 6;
constexpr size_t kBudget = 1 << 20;
constexpr int kMaxGroup = 16;
constexpr double kMaxSteps = 1000.0;

struct Item : SchedItem {
  uint64_t payload = 0;
};

double value_of(uint64_t p) { return (double)(p % 100003) * 0.5 + 1.0; }
double se_of(uint64_t p) { return (double)(p % 97) * 1e-3; }
bool fails_at_start(uint64_t p) { return p % 61 == 0; }

std::atomic<int> g_errors{0};

void fail(const char* what, unsigned long long a = 0, unsigned long long b = 0) {
  if (g_errors.fetch_add(1) < 20) std::printf("FAIL %s (%llu, %llu)\n", what, a, b);
}

class FakeExecutor : public Executor {
 public:
  FakeExecutor() : arena_(kBudget), slot_(kSlots) { device_ = std::thread([this] { device_loop(); }); }
  ~FakeExecutor() override {
    quit_.store(true);
    device_.join();
  }
  int slots() const override { return kSlots; }
  size_t largest_free() const override { return arena_.largest_free(); }

  int start(int s, SchedItem* const* items, int n) override {
    Slot& sl = slot_[s];
    if (sl.state.load(std::memory_order_relaxed) != kIdle) fail("start on a busy slot", s);
    if (n < 1 || n > kMaxGroup) fail("group size", n);
    double steps = 0.0;
    size_t bytes = 0;
    for (int j = 0; j < n; ++j) {
      if (items[j]->ticket != next_ticket_ + j) fail("not a queue prefix", items[j]->ticket, next_ticket_ + j);
      steps += items[j]->steps;
      bytes += items[j]->bytes;
    }
    if (n > 1 && steps > kMaxSteps) fail("group over the step limit", n);
    if (n > 1 && bytes > arena_.largest_free()) fail("group over the free block", bytes);
    Item* head = static_cast<Item*>(items[0]);
    if (fails_at_start(head->payload)) {
      head->status = 1;
      head->msg = "injected";
      next_ticket_ += 1;
      ++started_;
      return -1;
    }
    // sometimes only a shorter prefix fits, as when a group's own layout is larger
    int k = (n > 1 && head->ticket % 5 == 0) ? n / 2 : n;
    size_t off = 0;
    for (;;) {
      size_t b = 0;
      for (int j = 0; j < k; ++j) b += items[j]->bytes;
      if (arena_.alloc(b, &off)) {
        sl.off = off;
        sl.bytes = b;
        break;
      }
      if (k == 1) return 0;
      k /= 2;
    }
    sl.payload.assign(k, 0);
    for (int j = 0; j < k; ++j) sl.payload[j] = static_cast<Item*>(items[j])->payload;
    sl.n = k;
    sl.delay_us = 20 + (int)(head->payload % 300);
    sl.state.store(kRunning, std::memory_order_release);   // hands the group to the device thread
    next_ticket_ += k;
    started_ += k;
    return k;
  }

  bool finished(int s, SchedItem* const* items, int n) override {
    Slot& sl = slot_[s];
    if (sl.state.load(std::memory_order_acquire) != kDone) return false;
    if (n != sl.n) fail("retired group size", n, sl.n);
    for (int j = 0; j < n; ++j) {
      items[j]->logF = sl.out[2 * j];
      items[j]->se = sl.out[2 * j + 1];
      items[j]->status = 0;
    }
    arena_.release(sl.off, sl.bytes);
    sl.state.store(kIdle, std::memory_order_relaxed);
    return true;
  }

  long started() const { return started_; }

 private:
  enum { kIdle = 0, kRunning = 1, kDone = 2 };
  struct Slot {
    std::atomic<int> state{kIdle};
    int n = 0;
    int delay_us = 0;
    size_t off = 0, bytes = 0;
    std::vector<uint64_t> payload;   // written by the worker before kRunning
    std::vector<double> out;         // written by the device thread before kDone
  };

  void device_loop() {
    while (!quit_.load()) {
      bool any = false;
      for (Slot& sl : slot_) {
        if (sl.state.load(std::memory_order_acquire) != kRunning) continue;
        std::this_thread::sleep_for(std::chrono::microseconds(sl.delay_us));
        sl.out.assign(2 * sl.n, 0.0);
        for (int j = 0; j < sl.n; ++j) {
          sl.out[2 * j] = value_of(sl.payload[j]);
          sl.out[2 * j + 1] = se_of(sl.payload[j]);
        }
        sl.state.store(kDone, std::memory_order_release);
        any = true;
      }
      if (!any) std::this_thread::yield();
    }
  }

  Arena arena_;
  std::vector<Slot> slot_;
  std::thread device_;
  std::atomic<bool> quit_{false};
  uint64_t next_ticket_ = 1;   // touched only on the worker thread
  long started_ = 0;
};

struct Sent {
  uint64_t ticket;
  uint64_t payload;
};

void check_result(const Sent& s, const SchedItem& r) {
  if (!r.done) fail("handed back before done", s.ticket);
  if (r.ticket != s.ticket) fail("ticket mismatch", r.ticket, s.ticket);
  if (r.status == 0) {
    if (r.logF != value_of(s.payload) || r.se != se_of(s.payload)) fail("wrong result", s.ticket);
  } else if (!(r.status == 1 && r.msg == "injected" && fails_at_start(s.payload))) {
    fail("unexpected failure", s.ticket, r.status);
  }
  if (!(r.latency >= 0.0)) fail("latency", s.ticket);
}

void client(Scheduler* sch, int id, int count, std::atomic<long>* completed) {
  std::mt19937_64 rng(77 + id);
  std::vector<Sent> sent;
  for (int i = 0; i < count; ++i) {
    std::unique_ptr<SchedItem> it(new Item());
    Item* p = static_cast<Item*>(it.get());
    p->payload = rng();
    p->bytes = 1 + rng() % (kBudget / 10);
    p->steps = (rng() % 50 == 0) ? 5000.0 : (double)(1 + rng() % 200);   // a few above the group limit
    uint64_t t = 0;
    const uint64_t payload = p->payload;
    if (!sch->submit(it, &t)) {
      fail("submit refused while open", id);
      return;
    }
    sent.push_back({t, payload});
    if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
  }
  size_t left = sent.size();
  std::vector<char> got(sent.size(), 0);
  while (left) {
    for (size_t i = 0; i < sent.size(); ++i) {
      if (got[i]) continue;
      std::unique_ptr<SchedItem> r;
      const Scheduler::PollResult pr = sch->poll(sent[i].ticket, &r);
      if (pr == Scheduler::kUnknown) {
        fail("ticket lost", sent[i].ticket);
        got[i] = 1;
        --left;
      } else if (pr == Scheduler::kDone) {
        check_result(sent[i], *r);
        got[i] = 1;
        --left;
        completed->fetch_add(1);
        std::unique_ptr<SchedItem> again;
        if (sch->poll(sent[i].ticket, &again) != Scheduler::kUnknown) fail("ticket handed back twice", sent[i].ticket);
      }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace

int main() {
  // many clients at once
  {
    FakeExecutor ex;
    GroupLimits lim;
    lim.max_group = kMaxGroup;
    lim.max_steps = kMaxSteps;
    Scheduler sch(&ex, lim);
    sch.start_worker();
    std::atomic<long> completed{0};
    std::atomic<bool> stop_prober{false};
    std::thread prober([&] {
      std::mt19937_64 rng(5);
      while (!stop_prober.load()) {
        std::unique_ptr<SchedItem> r;
        // tickets far beyond any issued one: always unknown
        if (sch.poll(1000000 + rng() % 1000, &r) != Scheduler::kUnknown) fail("unknown ticket answered");
        std::this_thread::sleep_for(std::chrono::microseconds(30));
      }
    });
    const int kClients = 4, kEach = 1500;
    std::vector<std::thread> cl;
    for (int c = 0; c < kClients; ++c) cl.emplace_back(client, &sch, c, kEach, &completed);
    for (auto& t : cl) t.join();
    stop_prober.store(true);
    prober.join();
    if (completed.load() != (long)kClients * kEach) fail("completed count", completed.load());
    sch.shutdown();
    if (ex.started() != (long)kClients * kEach) fail("started count", ex.started());
    std::unique_ptr<SchedItem> it(new Item());
    uint64_t t = 0;
    if (sch.submit(it, &t)) fail("submit accepted after shutdown");
  }
  // shutdown drains what is queued
  {
    FakeExecutor ex;
    GroupLimits lim;
    lim.max_group = kMaxGroup;
    lim.max_steps = kMaxSteps;
    Scheduler sch(&ex, lim);
    sch.start_worker();
    std::vector<Sent> sent;
    for (int i = 0; i < 300; ++i) {
      std::unique_ptr<SchedItem> it(new Item());
      Item* p = static_cast<Item*>(it.get());
      p->payload = 1000 + 7 * (uint64_t)i;
      p->bytes = 1 + (size_t)i * 97 % (kBudget / 4);
      p->steps = 10.0;
      const uint64_t payload = p->payload;
      uint64_t t = 0;
      if (!sch.submit(it, &t)) fail("submit refused");
      sent.push_back({t, payload});
    }
    sch.shutdown();
    for (const Sent& s : sent) {
      std::unique_ptr<SchedItem> r;
      if (sch.poll(s.ticket, &r) != Scheduler::kDone) {
        fail("not drained by shutdown", s.ticket);
        continue;
      }
      check_result(s, *r);
    }
  }
  if (g_errors.load()) return 1;
  std::printf("ok\n");
  return 0;
}
