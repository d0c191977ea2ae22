// Host build of the FP64 normal quantile (device_math_f64.h) for the CPU
// tests: reads q values (one per line, as 17-digit decimals) and prints
// ninv64(q) with 17 significant digits.
#include <cmath>
#include <cstdio>

#define __host__
#define __device__
#define __forceinline__ inline
#include "device_math_f64.h"

int main() {
  double q;
  while (std::scanf("%lf", &q) == 1) std::printf("%.17g\n", vecchia::ninv64(q));
  return 0;
}
