// Host check of the serving loop's first-fit arena (arena.h) against a
// brute-force model over 256-byte units: random allocations and releases; every
// allocation must be the lowest fitting free run of the model, no two live
// allocations may overlap, and releasing everything must leave one free range.
// Built with AddressSanitizer and UBSan by the CPU test suite. Prints "ok".
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "arena.h"

int main() {
  for (int trial = 0; trial < 40; ++trial) {
    const size_t units = 64 + (size_t)trial * 37;
    const size_t size = units * 256;
    vecchia::Arena a(size);
    std::vector<int> used(units, 0);   // the model: 1 = allocated
    struct Live { size_t off, n; };
    std::vector<Live> live;
    std::mt19937_64 rng(1234 + trial);
    for (int step = 0; step < 4000; ++step) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const size_t bytes = 1 + rng() % (size / 6);
        const size_t need = (bytes + 255) / 256;
        // the model's lowest free run of `need` units
        size_t want = SIZE_MAX, run = 0;
        for (size_t u = 0; u < units; ++u) {
          run = used[u] ? 0 : run + 1;
          if (run == need) { want = u + 1 - need; break; }
        }
        size_t off = 0;
        const bool ok = a.alloc(bytes, &off);
        if (ok != (want != SIZE_MAX)) { std::printf("fit mismatch trial %d step %d\n", trial, step); return 1; }
        if (!ok) continue;
        if (off != want * 256) { std::printf("not first fit: %zu vs %zu\n", off, want * 256); return 1; }
        for (size_t u = off / 256; u < off / 256 + need; ++u) {
          if (used[u]) { std::printf("overlap\n"); return 1; }
          used[u] = 1;
        }
        live.push_back({off, bytes});
      } else {
        const size_t k = rng() % live.size();
        const Live l = live[k];
        live[k] = live.back();
        live.pop_back();
        a.release(l.off, l.n);
        for (size_t u = l.off / 256; u < l.off / 256 + (l.n + 255) / 256; ++u) used[u] = 0;
      }
    }
    for (const Live& l : live) a.release(l.off, l.n);
    if (a.free.size() != 1 || a.free.begin()->first != 0 || a.free.begin()->second != size) {
      std::printf("not coalesced: %zu ranges\n", a.free.size());
      return 1;
    }
  }
  std::printf("ok\n");
  return 0;
}
