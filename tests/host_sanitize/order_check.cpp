// Host driver for the library's orderings, built by the CPU test suite with
// AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only).
// stdin: D, then D lines "x y"; stdout: the COORD permutation, then the MAXMIN
// permutation, one line each.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "host_order.h"

int main() {
  long long D = 0;
  if (std::scanf("%lld", &D) != 1 || D < 1) return 2;
  std::vector<double> locs(2 * D);
  for (long long i = 0; i < 2 * D; ++i)
    if (std::scanf("%lf", &locs[i]) != 1) return 2;
  std::vector<int64_t> perm(D);
  vecchia::order_coord(locs.data(), D, perm.data());
  for (long long i = 0; i < D; ++i) std::printf("%lld%c", (long long)perm[i], i + 1 < D ? ' ' : '\n');
  vecchia::order_maxmin(locs.data(), D, perm.data());
  for (long long i = 0; i < D; ++i) std::printf("%lld%c", (long long)perm[i], i + 1 < D ? ' ' : '\n');
  return 0;
}
