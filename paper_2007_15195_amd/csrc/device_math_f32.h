// Single-precision normal CDF and quantile pieces for the SOV loop.
//
// The loop works with v = kappa t, kappa = sqrt(log2(e) / 2) (its rows are
// scaled by kappa), so that exp(-t^2/2) = 2^(-v^2).
//
// Phi: with a = |t|, the smaller tail is Phi(-a) = 2^(-v^2) R, where
// R = erfcx(a / sqrt 2) / 2 is a (3,4) rational in |v| fitted by
// fit_fp32_math.py (relative error < 1.4e-6 in FP32 for a in [0, 40]).
//
// Phi^{-1}: for q in (0, 1/2], z = -Phi^{-1}(q) is a (5,4) rational in
// s = sqrt(-log2 q) (relative error < 3.1e-6 in FP32 for s <= 34); where
// log2 q carries an exponent kept outside the FP32 number, a second rational
// covers s in [34, 1100].
//
// Hardware v_log_f32 / v_exp_f32 (base 2), v_sqrt_f32 and v_rcp_f32 are used
// directly; every argument they see is a normal FP32 number or zero.
#pragma once
#include <hip/hip_runtime.h>

#include "fp32_math_coeffs.h"

namespace vecchia {

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// z = -Phi^{-1}(q) >= 0 given log2(q), q <= 1/2.
__device__ __forceinline__ float ninv_tail_from_log2(float lq2) {
  const float s = fast_sqrt(-lq2);
  float p = kZP[5];
#pragma unroll
  for (int c = 4; c >= 0; --c) p = fmaf(p, s, kZP[c]);
  float q = kZQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, s, kZQ[c]);
  return p * fast_rcp(q);
}

// The split path's quantile: log2 q carries the exponent kept outside the FP32
// number and reaches -2^20 - 126 (s up to 1025). Up to s = 34 the main rational
// applies; beyond it a (3,2) rational fitted on s in [34, 1100] (relative error
// < 3.3e-7 in FP32) replaces the main one's extrapolation.
__device__ __forceinline__ float ninv_tail_from_log2_split(float lq2) {
  const float s = fast_sqrt(-lq2);
  float p = kZP[5];
#pragma unroll
  for (int c = 4; c >= 0; --c) p = fmaf(p, s, kZP[c]);
  float q = kZQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, s, kZQ[c]);
  float pw = kZPW[3];
#pragma unroll
  for (int c = 2; c >= 0; --c) pw = fmaf(pw, s, kZPW[c]);
  float qw = kZQW[2];
#pragma unroll
  for (int c = 1; c >= 0; --c) qw = fmaf(qw, s, kZQW[c]);
  return s > 34.0f ? pw * fast_rcp(qw) : p * fast_rcp(q);
}

// Phi(t) from v = kappa t, as e = em (exact unless em is split further by the
// caller) with the smaller tail m = Phi(-|t|) = 2^f R, f = -v^2.
struct PhiParts {
  float em;   // Phi(t)
  float m;    // Phi(-|t|)
  float f;    // -v^2
  float R;    // erfcx(|t| / sqrt 2) / 2
  bool neg;   // t <= 0
};

__device__ __forceinline__ PhiParts phi_f32(float v) {
  const float a = fabsf(v);
  PhiParts o;
  o.f = -(v * v);
  float p = kRP[3];
#pragma unroll
  for (int c = 2; c >= 0; --c) p = fmaf(p, a, kRP[c]);
  float q = kRQ[4];
#pragma unroll
  for (int c = 3; c >= 0; --c) q = fmaf(q, a, kRQ[c]);
  o.R = p * fast_rcp(q);
  o.m = fast_exp2(o.f) * o.R;
  o.neg = v <= 0.0f;
  o.em = o.neg ? o.m : 1.0f - o.m;
  return o;
}

}  // namespace vecchia
