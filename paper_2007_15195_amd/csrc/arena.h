// First-fit device-memory arena of the serving loop (host bookkeeping only):
// offsets into one reserved block, in 256-byte units, with neighbouring free
// ranges merged on release. Not thread-safe: the server calls it under its lock.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace vecchia {

struct Arena {
  std::map<size_t, size_t> free;   // offset -> length
  explicit Arena(size_t size) { free[0] = size; }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) / 256 * 256;
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free.erase(it);
        if (rest) free[at] = rest;
        return true;
      }
    }
    return false;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free) m = kv.second > m ? kv.second : m;
    return m;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) / 256 * 256;
    auto it = free.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace vecchia
