// Single-precision normal CDF and quantile pieces for the SOV loop.
//
// Every factor e = Phi(t) is carried in a base-2 log split, e = em * 2^en (en an
// integer held in a float), with its complement: a factor below the FP32 range
// keeps its exponent in en, and a factor close to 1 is used through 1 - e.
//
// Phi(t): with a = |t|, the smaller tail is Phi(-a) = exp(-a^2/2) R(a), where
// R(a) = erfcx(a / sqrt 2) / 2 is a (3,4) rational fitted by fit_fp32_math.py
// (relative error < 1.4e-6 in FP32 on [0, 40]); exp(-a^2/2) = 2^f with
// f = -a^2 log2(e) / 2. A lower-tail factor with f < -60 (t < -9.1) keeps
// 2^floor(f) as its exponent (a wave-uniform branch taken only when some lane
// needs it), so every mantissa stays >= 2^-65 and w * e stays a normal number.
//
// Phi^{-1}: for q in (0, 1/2], z = -Phi^{-1}(q) is a (5,4) rational in
// x = sqrt(-log2 q) - 1 (relative error < 2.7e-6 in FP32), with
// log2(q) = log2(q's mantissa) + q's exponent.
// Hardware v_log_f32 / v_exp_f32 (base 2), v_sqrt_f32 and v_rcp_f32 are used
// directly.
#pragma once
#include <hip/hip_runtime.h>

#include "fp32_math_coeffs.h"

namespace vecchia {

constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// z = -Phi^{-1}(q) >= 0 given log2(q), q <= 1/2.
__device__ __forceinline__ float ninv_tail_from_log2(float lq2) {
  const float x = fast_sqrt(-lq2) - 1.0f;
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
  float en;   // exponent part (integer valued); nonzero only for t below -13.2
  float m;    // Phi(-|t|) (its mantissa when en != 0): 1 - e when t > 0
  bool neg;   // t <= 0
};

__device__ __forceinline__ Factor phi_f32(float t) {
  const float a = fabsf(t);
  const float f = (a * a) * (-0.5f * kLog2e);
  float p = kRP[3];
#pragma unroll
  for (int c = 2; c >= 0; --c) p = fmaf(p, a, kRP[c]);
  float q = kRQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, a, kRQ[c]);
  const float R = p * fast_rcp(q);
  Factor o;
  o.neg = t <= 0.0f;
  o.en = 0.0f;
  o.m = fast_exp2(f) * R;                       // Phi(-a)
  o.em = o.neg ? o.m : 1.0f - o.m;
  const bool deep = o.neg && f < -60.0f;
  if (__builtin_expect(__any(deep), 0)) {       // wave-uniform, rare
    if (deep) {
      const float fl = floorf(f);
      o.em = fast_exp2(f - fl) * R;
      o.en = fl;
    }
  }
  return o;
}

}  // namespace vecchia
