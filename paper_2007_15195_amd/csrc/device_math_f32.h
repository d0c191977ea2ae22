// Single-precision normal CDF pieces for the SOV loop, in log space.
//
// Phi(t): with a = |t|, the smaller tail is Phi(-a) = exp(-a^2/2) R(a), where
// R(a) = erfcx(a / sqrt 2) / 2 is approximated by a (4,5) rational fitted by
// fit_fp32_math.py (relative error < 5e-7 in FP32 on [0, 40]). Returned together:
// e = Phi(t), ec = 1 - Phi(t) (each accurate as the smaller tail) and
// le = log Phi(t) (from log R - a^2/2 when t <= 0, log(1 - Phi(-t)) otherwise).
//
// Phi^{-1}: for q in (0, 1/2], z = -Phi^{-1}(q) is a (6,5) rational in
// x = sqrt(-2 log q) - sqrt(2 log 2) (relative error < 4e-7 in FP32). The caller
// passes the smaller tail q of u and its sign, so 1 - u never loses digits.
// Hardware v_log_f32 / v_exp_f32 (base 2), v_sqrt_f32 and v_rcp_f32 are used.
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
  const float s = fast_sqrt(-2.0f * kLn2 * lq2);
  const float x = fmaxf(s - kS0, 0.0f);
  float p = kZP[6];
#pragma unroll
  for (int c = 5; c >= 0; --c) p = fmaf(p, x, kZP[c]);
  float q = kZQ[5];
#pragma unroll
  for (int c = 4; c >= 0; --c) q = fmaf(q, x, kZQ[c]);
  return p * fast_rcp(q);
}

struct PhiOut {
  float e, ec, le;
};

__device__ __forceinline__ PhiOut phi_f32(float t) {
  const float a = fabsf(t);
  const float a2 = a * a;
  const float E = fast_exp2(a2 * (-0.5f * kLog2e));
  float p = kRP[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) p = fmaf(p, a, kRP[c]);
  float q = kRQ[5];
#pragma unroll
  for (int c = 4; c >= 0; --c) q = fmaf(q, a, kRQ[c]);
  const float R = p * fast_rcp(q);
  const float P = E * R;                 // Phi(-a)
  const bool neg = t <= 0.0f;
  const float omP = 1.0f - P;
  PhiOut o;
  o.e = neg ? P : omP;
  o.ec = neg ? omP : P;
  const float L2 = fast_log2(neg ? R : omP);
  o.le = neg ? fmaf(L2, kLn2, -0.5f * a2) : L2 * kLn2;
  return o;
}

}  // namespace vecchia
