// Steps a6-a7 (Section 2.2, eq. (6); Section 3.1) in two kernels.
//
// term_finalize: one wave per term (all instances of a launch). A term with no
// SOV dimension (k = 0; in a censored plan also a density term or a censored
// term whose neighbours are all uncensored), or one that term_setup found to be
// 0 (a -inf limit), takes the exact value term_setup wrote, with SE 0;
// otherwise the wave's lanes take the shifts (lane r sums shift r's chunks in
// order), fixed butterflies give the totals, and
//     log-term = log(sum_r num_r) - log(sum_r den_r)
// (with the FP32 loop, log1p(-sum cnum / sum den) when that tail is the smaller,
// which keeps digits for terms close to 1), and the delta-method standard error
//     se^2 = R/(R-1) sum_r (num_r / sum num - den_r / sum den)^2   (NaN for R = 1).
// With independent points (passes = 2) the denominators come from the second
// lattice's sums and se^2 = R/(R-1) sum_r [(num_r / sum num - 1/R)^2 + (den_r / sum den - 1/R)^2].
// Results go to a per-term array and, when asked for, to the user-order output.
// In an FP32 evaluation a term whose SE exceeds kRedoSe is not written by this
// pass: it goes to the re-run list, whose FP64 pass term_finalize_redo finalizes.
//
// instance_logsum: one block per instance sums its terms' log-terms and se^2 in
// a fixed order (per-thread strided partial sums, then a fixed tree), so the
// result does not depend on anything but the instance.
#include "vecchia_internal.h"

namespace vecchia {
namespace {

__device__ __forceinline__ int find_inst(const int64_t* __restrict__ bases, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bases[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kFinalizeWaves = 4;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Finalize of global term t by the calling wave. allow_redo: the first pass of
// an FP32 evaluation, which hands a term whose FP32 estimate is heavy-tailed
// (SE above kRedoSe) to the FP64 re-run list instead of writing it.
__device__ __forceinline__ void finalize_term(const InstDesc* __restrict__ insts, int n_inst,
                                              const int64_t* __restrict__ term_bases,
                                              const Aux64* __restrict__ aux64, const double* __restrict__ sums,
                                              double2* __restrict__ term_res, int64_t t, bool allow_redo) {
  const int lane = threadIdx.x & 63;
  const int ii = find_inst(term_bases, n_inst, t);
  const InstDesc& I = insts[ii];
  const int64_t i = t - term_bases[ii];
  const int R = I.n_shifts;
  double lt, se2;
  bool fp32_sums = false;
  if (I.sovk[i] == 0 || aux64[t].e0 < 0.0) {   // exact, or a term that is 0 (e0 = -1)
    lt = aux64[t].lt0;
    se2 = 0.0;
  } else {
    const int C = I.n_chunks;
    const bool indep = I.passes == 2;
    // numerators from the term's lattice; denominators from the same sums, or
    // from the second lattice's R x C sums that follow them
    const double* s = sums + 3 * (I.sums_base + i * I.passes * R * (int64_t)C);
    const double* sdn = s + (indep ? 3 * (int64_t)R * C : 0);
    double pn = 0.0, pd = 0.0, pc = 0.0;
    for (int r = lane; r < R; r += 64) {
      for (int c = 0; c < C; ++c) {
        pn += s[3 * (r * C + c)];
        pd += sdn[3 * (r * C + c) + 1];
        pc += s[3 * (r * C + c) + 2];
      }
    }
    const double sn = wave_sum(pn), sd = wave_sum(pd), sc = wave_sum(pc);
    // the log1p form needs the FP32 loop's complement sums (not kept by the FP64
    // items of a handed-over term)
    fp32_sums = I.precision == VECCHIA_FP32_LOOP && I.promote[t] == 0;
    if (fp32_sums && !indep && sc < sn)
      lt = log1p(-sc / sd);
    else
      lt = log(sn) - log(sd);
    if (R > 1) {
      double acc = 0.0;
      for (int r = lane; r < R; r += 64) {
        double nr = 0.0, dr = 0.0;
        for (int c = 0; c < C; ++c) {
          nr += s[3 * (r * C + c)];
          dr += sdn[3 * (r * C + c) + 1];
        }
        if (indep) {
          // independent estimates: their relative variances add
          const double a = nr / sn - 1.0 / R, b = dr / sd - 1.0 / R;
          acc += a * a + b * b;
        } else {
          const double d = nr / sn - dr / sd;
          acc += d * d;
        }
      }
      se2 = wave_sum(acc) * (double)R / (double)(R - 1);
    } else {
      se2 = __builtin_nan("");
    }
  }
  if (allow_redo && fp32_sums && se2 > kRedoSe * kRedoSe && __builtin_isfinite(lt) && __builtin_isfinite(se2)) {
    // heavy-tailed: the few samples that carry the estimate also carry the FP32
    // loop's rounding; the term runs again in FP64 and its pass writes it
    if (lane == 0) {
      I.promote[t] = 2;
      const unsigned long long slot = atomicAdd(reinterpret_cast<unsigned long long*>(&I.pctr[2]), 1ULL);
      if ((int64_t)slot < I.plist_cap) I.plist[I.plist_cap + slot] = (int32_t)t;
    }
    return;
  }
  if (lane == 0) {
    term_res[t] = make_double2(lt, se2);
    if (I.terms_out) {
      const int64_t u = I.bvars ? i : I.perm[i];   // block plans: group order
      I.terms_out[2 * u] = lt;
      I.terms_out[2 * u + 1] = sqrt(se2);
    }
  }
}

__global__ __launch_bounds__(64 * kFinalizeWaves) void term_finalize(
    const InstDesc* __restrict__ insts, int n_inst, const int64_t* __restrict__ term_bases,
    int64_t total_terms, const Aux64* __restrict__ aux64, const double* __restrict__ sums,
    double2* __restrict__ term_res, int64_t term_base, int allow_redo) {
  const int64_t t = term_base + (int64_t)blockIdx.x * kFinalizeWaves + (threadIdx.x >> 6);
  if (t >= total_terms) return;   // t is the same on every lane of a wave
  finalize_term(insts, n_inst, term_bases, aux64, sums, term_res, t, allow_redo != 0);
}

// The re-run list's terms after their FP64 pass, one per wave in turn.
__global__ __launch_bounds__(64 * kFinalizeWaves) void term_finalize_redo(
    const InstDesc* __restrict__ insts, int n_inst, const int64_t* __restrict__ term_bases,
    const Aux64* __restrict__ aux64, const double* __restrict__ sums, double2* __restrict__ term_res,
    const int32_t* __restrict__ list, const int64_t* __restrict__ count, int64_t cap) {
  const int64_t n = min(*count, cap);
  const int64_t waves = (int64_t)gridDim.x * kFinalizeWaves;
  for (int64_t e = (int64_t)blockIdx.x * kFinalizeWaves + (threadIdx.x >> 6); e < n; e += waves)
    finalize_term(insts, n_inst, term_bases, aux64, sums, term_res, (int64_t)list[e], false);
}

__global__ __launch_bounds__(kFinalizeThreads) void instance_logsum(const InstDesc* __restrict__ insts,
                                                                     const double2* __restrict__ term_res,
                                                                     int64_t inst_base) {
  __shared__ double red_lt[kFinalizeThreads];
  __shared__ double red_se[kFinalizeThreads];
  const InstDesc& I = insts[inst_base + (int64_t)blockIdx.x];
  const double2* r = term_res + I.term_base;
  double part_lt = 0.0, part_se = 0.0;
  for (int64_t i = threadIdx.x; i < I.n_terms; i += kFinalizeThreads) {
    const double2 v = r[i];
    part_lt += v.x;
    part_se += v.y;
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

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Scale-mixture combination of one mixture (one wave, node k on lane k; fixed
// butterflies): out = {log sum_k exp(logw_k + lf_k), sqrt(sum_k (c_k / G)^2 se_k^2)}.
__device__ void combine_wave(const double* __restrict__ node_out, double logw, int n,
                             double* __restrict__ out, double* __restrict__ nodes_out) {
  const int lane = threadIdx.x;
  const bool on = lane < n;
  const double lf = on ? node_out[2 * lane] : 0.0;
  const double se = on ? node_out[2 * lane + 1] : 0.0;
  const double c = on ? logw + lf : -HUGE_VAL;
  const double mx = wave_max(on ? c : -HUGE_VAL);
  double logG;
  if (mx == -HUGE_VAL) {
    logG = -HUGE_VAL;    // every node's Phi_D underflowed to 0
  } else {
    const double sum = wave_sum(on ? exp(c - mx) : 0.0);
    logG = mx + log(sum);
  }
  const double frac = (on && logG > -HUGE_VAL) ? exp(c - logG) : 0.0;   // G = 0 is exact: SE 0
  const double var = wave_sum(on ? (frac * se) * (frac * se) : 0.0);
  if (lane == 0) {
    out[0] = logG;
    out[1] = sqrt(var);
  }
  if (nodes_out && on) {
    nodes_out[2 * lane] = lf;
    nodes_out[2 * lane + 1] = se;
  }
}

__global__ __launch_bounds__(64) void mixture_combine(const double* __restrict__ node_out, MixWeights mw,
                                                      double* __restrict__ out, double* __restrict__ nodes_out) {
  const int lane = threadIdx.x;
  combine_wave(node_out, lane < mw.n ? mw.logw[lane] : 0.0, mw.n, out, nodes_out);
}

// Many mixtures (one wave each): mixture t's n nodes at node_out + 2 n t, its log
// weights at logw + n t, its result at out + 2 t.
__global__ __launch_bounds__(64) void mixture_combine_many(const double* __restrict__ node_out,
                                                           const double* __restrict__ logw, int n,
                                                           double* __restrict__ out) {
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x;
  combine_wave(node_out + 2 * n * t, lane < n ? logw[n * t + lane] : 0.0, n, out + 2 * t, nullptr);
}

// Sum over mixtures in a fixed order: total = {sum_t log G_t, sqrt(sum_t se_t^2)}.
__global__ __launch_bounds__(kFinalizeThreads) void mixture_total(const double* __restrict__ out, int64_t n,
                                                                   double* __restrict__ total) {
  __shared__ double red_lg[kFinalizeThreads];
  __shared__ double red_se[kFinalizeThreads];
  double lg = 0.0, se = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += kFinalizeThreads) {
    lg += out[2 * t];
    se += out[2 * t + 1] * out[2 * t + 1];
  }
  red_lg[threadIdx.x] = lg;
  red_se[threadIdx.x] = se;
  __syncthreads();
  for (int o = kFinalizeThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red_lg[threadIdx.x] += red_lg[threadIdx.x + o];
      red_se[threadIdx.x] += red_se[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    total[0] = red_lg[0];
    total[1] = sqrt(red_se[0]);
  }
}

}  // namespace

hipError_t launch_mixture_combine(const double* node_out, const MixWeights& mw, double* out, double* nodes_out,
                                  hipStream_t s) {
  if (mw.n < 1 || mw.n > kMaxMixNodes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mixture_combine, dim3(1), dim3(64), 0, s, node_out, mw, out, nodes_out);
  return hipGetLastError();
}

hipError_t launch_mixture_combine_many(const double* node_out, const double* logw, int n_nodes, int64_t n_mix,
                                       double* out, double* total, hipStream_t s) {
  if (n_nodes < 1 || n_nodes > kMaxMixNodes || n_mix < 1 || n_mix > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mixture_combine_many, dim3((unsigned)n_mix), dim3(64), 0, s, node_out, logw, n_nodes, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && total) {
    hipLaunchKernelGGL(mixture_total, dim3(1), dim3(kFinalizeThreads), 0, s, out, n_mix, total);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_finalize_terms(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                                 int64_t total_terms, const Aux64* aux64, const double* sums,
                                 double2* term_res, bool allow_redo, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  constexpr int64_t kPer = kMaxLaunchThreads / 64;   // terms (one wave each) per launch
  for (int64_t b = 0; b < total_terms; b += kPer) {
    const int64_t n = total_terms - b < kPer ? total_terms - b : kPer;
    const unsigned blocks = (unsigned)((n + kFinalizeWaves - 1) / kFinalizeWaves);
    hipLaunchKernelGGL(term_finalize, dim3(blocks), dim3(64 * kFinalizeWaves), 0, s, d_insts, n_inst,
                       d_term_bases, total_terms, aux64, sums, term_res, b, allow_redo ? 1 : 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_finalize_redo(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                                const Aux64* aux64, const double* sums, double2* term_res,
                                const int32_t* list, const int64_t* count, int64_t cap, hipStream_t s) {
  if (n_inst <= 0 || cap <= 0) return hipSuccess;
  const int64_t blocks = (cap + kFinalizeWaves - 1) / kFinalizeWaves;
  hipLaunchKernelGGL(term_finalize_redo, dim3((unsigned)(blocks < 256 ? blocks : 256)), dim3(64 * kFinalizeWaves), 0,
                     s, d_insts, n_inst, d_term_bases, aux64, sums, term_res, list, count, cap);
  return hipGetLastError();
}

hipError_t launch_logsum(const InstDesc* d_insts, int n_inst, const double2* term_res, hipStream_t s) {
  constexpr int64_t kPerInst = kMaxLaunchThreads / kFinalizeThreads;   // instances (one block each) per launch
  for (int64_t b = 0; b < n_inst; b += kPerInst) {
    const unsigned n = (unsigned)(n_inst - b < kPerInst ? n_inst - b : kPerInst);
    hipLaunchKernelGGL(instance_logsum, dim3(n), dim3(kFinalizeThreads), 0, s, d_insts, term_res, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vecchia
