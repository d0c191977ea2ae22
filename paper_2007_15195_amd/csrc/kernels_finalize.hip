// finalize_logsum: steps a6-a7 (Section 2.2, eq. (6); Section 3.1).
//
// One block per instance. For every term: k = 0 gives the exact log Phi(b_0/L_00)
// with SE 0; otherwise the R shift sums give
//     log-term = log(sum_r num_r) - log(sum_r den_r)
// (with the FP32 loop, log1p(-sum cnum / sum den) when that tail is the smaller,
// which keeps digits for terms close to 1), and the delta-method standard error
//     se^2 = R/(R-1) sum_r (num_r / sum num - den_r / sum den)^2
// (NaN for R = 1). The instance's log F is the sum of its log-terms and its SE
// the root of the summed se^2, both reduced in a fixed order.
#include "vecchia_internal.h"

namespace vecchia {
namespace {

__global__ __launch_bounds__(kFinalizeThreads) void finalize_logsum(
    const InstDesc* __restrict__ insts, const Aux64* __restrict__ aux64,
    const double* __restrict__ sums) {
  __shared__ double red_lt[kFinalizeThreads];
  __shared__ double red_se[kFinalizeThreads];
  const InstDesc& I = insts[blockIdx.x];
  const int R = I.n_shifts;
  const bool f32 = I.precision == VECCHIA_FP32_LOOP;
  double part_lt = 0.0, part_se = 0.0;
  for (int64_t i = threadIdx.x; i < I.D; i += kFinalizeThreads) {
    const int64_t t = I.term_base + i;
    double lt, se2;
    if (I.kcnt[i] == 0) {
      lt = aux64[t].lt0;
      se2 = 0.0;
    } else {
      const double* s = sums + 3 * (I.sums_base + i * R);
      double sn = 0.0, sd = 0.0, sc = 0.0;
      for (int r = 0; r < R; ++r) {
        sn += s[3 * r];
        sd += s[3 * r + 1];
        sc += s[3 * r + 2];
      }
      if (f32 && sc < sn)
        lt = log1p(-sc / sd);
      else
        lt = log(sn) - log(sd);
      if (R > 1) {
        double acc = 0.0;
        for (int r = 0; r < R; ++r) {
          const double d = s[3 * r] / sn - s[3 * r + 1] / sd;
          acc += d * d;
        }
        se2 = acc * (double)R / (double)(R - 1);
      } else {
        se2 = __builtin_nan("");
      }
    }
    part_lt += lt;
    part_se += se2;
    if (I.terms_out) {
      const int64_t u = I.perm[i];
      I.terms_out[2 * u] = lt;
      I.terms_out[2 * u + 1] = sqrt(se2);
    }
  }
  red_lt[threadIdx.x] = part_lt;
  red_se[threadIdx.x] = part_se;
  __syncthreads();
  for (int o = kFinalizeThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red_lt[threadIdx.x] += red_lt[threadIdx.x + o];
      red_se[threadIdx.x] += red_se[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    I.out[0] = red_lt[0];
    I.out[1] = sqrt(red_se[0]);
  }
}

}  // namespace

hipError_t launch_finalize(const InstDesc* d_insts, int n_inst, const Aux64* aux64,
                           const double* sums, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_logsum, dim3((unsigned)n_inst), dim3(kFinalizeThreads), 0, s, d_insts,
                     aux64, sums);
  return hipGetLastError();
}

}  // namespace vecchia
