// Host build of the FP64 exponential the normal CDF uses (device_math_f64.h)
// for the CPU tests: reads x values (one per line, as 17-digit decimals) and
// prints exp64(x) with 17 significant digits.
#include <cmath>
#include <cstdio>

#define __host__
#define __device__
#define __forceinline__ inline
#include "device_math_f64.h"

int main() {
  double x;
  while (std::scanf("%lf", &x) == 1) std::printf("%.17g\n", vecchia::exp64(x));
  return 0;
}
