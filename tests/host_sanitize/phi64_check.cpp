// Host build of the FP64 normal CDF (device_math_f64.h) for the CPU tests:
// reads t values (one per line) and prints phi64(t) with 17 significant digits.
#include <cmath>
#include <cstdio>

#define __host__
#define __device__
#define __forceinline__ inline
#include "device_math_f64.h"

int main() {
  double t;
  while (std::scanf("%lf", &t) == 1) std::printf("%.17g\n", vecchia::phi64(t));
  return 0;
}
