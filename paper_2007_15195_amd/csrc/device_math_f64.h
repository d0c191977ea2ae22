// FP64 normal CDF and quantile for the FP64 SOV loops (the plain parity path,
// the terms an FP32 evaluation hands over, and the full-dimension comparator).
//
// Phi(t): with a = |t|, Phi(-a) = R(a) exp(-a^2/2), R the scaled tail
// Phi(-a) exp(a^2/2), a fitted ratio of degrees (9, 10) with positive
// coefficients over [0, 38.5] (relative error of the fit 5.1e-17). a^2 is split
// exactly (h + l with an FMA) so that exp(-a^2/2) keeps its relative accuracy
// for large a; Phi(t) = 1 - Phi(-a) for t >= 0; beyond a = 38.5 the lower tail
// is below the smallest subnormal and rounds to 0.
//
// z = Phi^{-1}(q), q in (0, 1), in three pieces on p = min(q, 1 - q) (1 - q is
// exact for q >= 1/2 in binary floating point):
//   |q - 1/2| <= 0.425:  z = r P(x) / Q(x), r = q - 1/2, x = 0.425^2 - r^2;
//   otherwise s = sqrt(-log p) and |z| = P(s - s0) / Q(s - s0), with s0 =
//   sqrt(-log 0.075) for s <= 5 and s0 = 5 beyond, z taking the sign of r.
// The rationals (fp64_math_coeffs.h, fitted by fit_fp64_math.py) have
// coefficients of one sign, so Horner's rule evaluates them without
// cancellation; the fits' relative error is below 2.1e-16 and the evaluated
// function stays within a few units in the last place of the exact quantile
// over p from 1/2 down to the smallest subnormal; q = 0 and 1 give -inf and
// +inf, anything outside [0, 1] NaN.
//
// exp(x), x in [-745, 0] (exp64, the CDF's Gaussian factor): x = k ln 2 + r,
// |r| <= ln 2 / 2, exp(r) = 1 + r + r^2 g(r) with g fitted in r + 0.3466 >= 0
// (positive coefficients), scaled by 2^k
// (a subnormal result below 2^-1022); no range checks, as the CDF's argument
// is bounded.
//
// Quotients of the rationals (div64): their denominators are at least 1 and
// their numerators moderate, so a reciprocal refined by two Newton steps and
// one residual correction replaces the IEEE division's scaling and fix-up
// steps, within about one unit in the last place.
//
// log p (log64): p = m 2^e with m in [sqrt(1/2), sqrt(2)); with f = m - 1
// (exact) and s = f / (2 + f), log m = 2 atanh(s) = f - s f + s R, where
// R = z P(z), z = s^2, is the series' remainder (P fitted), and f - s f is
// taken as f - (f^2/2 - s f^2/2) so that the small terms carry the rounding;
// e ln 2 is added in two parts, the first exact. About a third of the
// instructions of a correctly rounded logarithm, within about one unit in the
// last place.
#pragma once

#include "fp64_math_coeffs.h"

namespace vecchia {

template <int N>
__host__ __device__ __forceinline__ double horner64(const double (&c)[N], double x) {
  double v = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) v = __builtin_fma(v, x, c[i]);
  return v;
}

// The same at x >= 0 (up to rounding), evaluated at |x|. On gfx950 an FMA
// whose operand carries a source modifier keeps the three-operand form, with
// each coefficient in a pair of scalar registers; without one the compiler
// prefers the two-operand form and copies every coefficient into vector
// registers first (two extra vector instructions per coefficient).
template <int N>
__host__ __device__ __forceinline__ double horner64_pos(const double (&c)[N], double x) {
  return horner64(c, __builtin_fabs(x));
}

// n / d for d >= 1 and a moderate n.
__host__ __device__ __forceinline__ double div64(double n, double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(d);   // about half the bits
#else
  double r = 1.0 / d;
#endif
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  const double y = n * r;
  return __builtin_fma(__builtin_fma(-d, y, n), r, y);
}

// exp(x) for x in [-745, 0].
__host__ __device__ __forceinline__ double exp64(double x) {
  const double k = __builtin_rint(x * 1.44269504088896340736);   // x / ln 2, to the nearest integer
  const double r = __builtin_fma(-k, kLn2Lo, __builtin_fma(-k, kLn2Hi, x));
  const double e = 1.0 + __builtin_fma(r * r, horner64_pos(kExpG, r + kExpShift), r);
  return __builtin_ldexp(e, (int)k);
}

__host__ __device__ inline double phi64(double t) {
  const double a = __builtin_fabs(t);
  double lower = 0.0;   // Phi(-a)
  if (a <= 38.5) {
    const double R = div64(horner64(kPhiRP, a), horner64(kPhiRQ, a));
    const double h = a * a;
    const double l = __builtin_fma(a, a, -h);   // h + l = a^2 exactly
    lower = R * (exp64(-0.5 * h) * (1.0 - 0.5 * l));
  } else if (!(a > 38.5)) {
    return t;   // NaN
  }
  return t < 0.0 ? lower : 1.0 - lower;
}

// Natural logarithm of a positive finite x (subnormal included).
__host__ __device__ __forceinline__ double log64(double x) {
  int e;
  double m = __builtin_frexp(x, &e);   // x = m 2^e, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double f = m - 1.0;
  const double s = div64(f, 2.0 + f);
  const double z = s * s;
  const double R = z * horner64_pos(kLogP, z);
  const double hf = 0.5 * f * f;
  const double de = (double)e;
  return de * kLn2Hi + (f - (hf - (s * (hf + R) + de * kLn2Lo)));
}

__host__ __device__ inline double ninv64(double q) {
  const double r = q - 0.5;
  if (__builtin_fabs(r) <= 0.425) {
    const double x = __builtin_fma(-r, r, 0.180625);
    return r * div64(horner64_pos(kNinvCentralP, x), horner64_pos(kNinvCentralQ, x));
  }
  // outside (0, 1) p is negative or NaN (NaN results) or 0 (infinite results)
  const double p = r < 0.0 ? q : 1.0 - q;
  if (!(p > 0.0)) return p == 0.0 ? (r < 0.0 ? -HUGE_VAL : HUGE_VAL) : __builtin_nan("");
  const double s = sqrt(-log64(p));
  double z;
  if (s <= 5.0) {
    const double x = s - kNinvS1;
    z = div64(horner64_pos(kNinvTail1P, x), horner64_pos(kNinvTail1Q, x));
  } else {
    const double x = s - 5.0;
    z = div64(horner64_pos(kNinvTail2P, x), horner64_pos(kNinvTail2Q, x));
  }
  return r < 0.0 ? -z : z;
}

}  // namespace vecchia
