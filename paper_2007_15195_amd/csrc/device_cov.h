// Stationary isotropic covariance of the Gaussian process (device side): the
// exponential model of the paper's simulations and application (Sections 3 and
// 4.1) and the Matern family with nu in {1/2, 3/2, 5/2}, parameterised as
//   K(h) = sigma2 2^(1-nu) / Gamma(nu) (sqrt(2 nu) h / rho)^nu K_nu(sqrt(2 nu) h / rho),
// whose half-integer cases have the closed forms below.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/vecchia.h"

namespace vecchia {

__device__ __forceinline__ double cov_kernel(double h, int family, double nu, double s2, double rho) {
#pragma clang fp contract(off)
  if (family == VECCHIA_COV_EXPONENTIAL || nu == 0.5) return s2 * exp(-h / rho);
  if (nu == 1.5) {
    const double a = 1.7320508075688772 * h / rho;   // sqrt(3) h / rho
    return s2 * (1.0 + a) * exp(-a);
  }
  const double a = 2.23606797749979 * h / rho;       // sqrt(5) h / rho
  return s2 * (1.0 + a + a * a / 3.0) * exp(-a);
}

}  // namespace vecchia
