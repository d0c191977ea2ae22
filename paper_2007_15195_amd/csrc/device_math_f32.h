// Single-precision normal CDF and quantile pieces for the SOV loop.
//
// Every factor e = Phi(t) is carried in a base-2 log split, e = em * 2^en (en an
// integer held in a float, 0 when t > 0), together with ec = 1 - e, so neither
// deep lower tails (e below the FP32 range) nor factors close to 1 lose digits.
//
// Phi(t): with a = |t|, the smaller tail is Phi(-a) = exp(-a^2/2) R(a), where
// R(a) = erfcx(a / sqrt 2) / 2 is a (3,4) rational fitted by fit_fp32_math.py
// (relative error < 1.4e-6 in FP32 on [0, 40]); exp(-a^2/2) is taken as
// 2^fl * 2^(f - fl) with f = -a^2 log2(e) / 2 and fl = floor(f).
//
// Phi^{-1}: for q in (0, 1/2], z = -Phi^{-1}(q) is a (5,4) rational in
// x = sqrt(-2 log q) - sqrt(2 log 2) (relative error < 2.7e-6 in FP32), from
// log2(q) = log2(q's mantissa) + q's exponent.
// Hardware v_log_f32 / v_exp_f32 (base 2), v_sqrt_f32, v_rcp_f32, v_ldexp_f32
// are used directly.
#pragma once
#include <hip/hip_runtime.h>

#include "fp32_math_coeffs.h"

namespace vecchia {

constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// z = -Phi^{-1}(q) >= 0 given log2(q), q <= 1/2.
__device__ __forceinline__ float ninv_tail_from_log2(float lq2) {
  const float s = fast_sqrt(lq2 * (-2.0f * kLn2));
  const float x = s - kS0;
  float p = kZP[5];
#pragma unroll
  for (int c = 4; c >= 0; --c) p = fmaf(p, x, kZP[c]);
  float q = kZQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, x, kZQ[c]);
  return p * fast_rcp(q);
}

struct Factor {
  float em;   // mantissa part of e = Phi(t)
  float en;   // exponent part (integer valued), 0 when t > 0
  float ec;   // 1 - e
  bool neg;   // t <= 0
};

__device__ __forceinline__ Factor phi_f32(float t) {
  const float a = fabsf(t);
  const float f = (a * a) * (-0.5f * kLog2e);
  const float fl = floorf(f);
  const float E = fast_exp2(f - fl);                 // in [1, 2)
  float p = kRP[3];
#pragma unroll
  for (int c = 2; c >= 0; --c) p = fmaf(p, a, kRP[c]);
  float q = kRQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, a, kRQ[c]);
  const float m = E * (p * fast_rcp(q));            // Phi(-a) = m * 2^fl
  const float P = __builtin_amdgcn_ldexpf(m, (int)fl);
  const float omP = 1.0f - P;
  Factor o;
  o.neg = t <= 0.0f;
  o.em = o.neg ? m : omP;
  o.en = o.neg ? fl : 0.0f;
  o.ec = o.neg ? omP : P;
  return o;
}

}  // namespace vecchia
