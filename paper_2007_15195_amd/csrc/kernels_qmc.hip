// QMC kernels: steps a4-a5 of every Vecchia term (Section 2.2, eq. (6); Genz's
// separation of variables with a randomized lattice rule).
//
// Work item = (term, shift): one wave evaluates all N lattice points of one
// random shift of one term, lattice points across the 64 lanes (lane l takes
// p = l+1, l+65, ...). K = the term's conditioning-set size is a template
// parameter so the chain is fully unrolled and y[] stays in registers. Per
// chain (variables 0..K, the term's own component last):
//     e_0 = Phi(b'_0)                         (constant, from term_setup)
//     y_{a-1} = Phi^{-1}(w_{a-1} e_{a-1})      a = 1..K
//     t_a = b'_a - sum_{c<a} L'_ac y_c,   e_a = Phi(t_a)
//     den = prod_{a<K} e_a,   num = den * e_K
// and the wave writes the point sums {sum num, sum den, sum den*(1-e_K)} of its
// shift. Sums use a fixed butterfly, so a shift's result does not depend on
// where or with what else it runs.
//
// FP64 kernel: the plain parity path (HIP's normcdf / normcdfinv).
// FP32 kernel: the chain in single precision in log space: the product is
// carried as sum log e_a, u's smaller tail is formed as u or (1-w) + w(1-e), and
// log u falls back to log w + log e when u underflows; the per-chain product is
// rebuilt exactly as 2^n * 2^f in FP64 and accumulated in FP64.
#include "device_math_f32.h"
#include "lattice.h"
#include "vecchia_internal.h"

namespace vecchia {
namespace {

__device__ __forceinline__ int find_range(const RangeDesc* __restrict__ r, int n, int64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].item_begin <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct ItemInfo {
  const InstDesc* I;
  int64_t i;      // plan index of the term
  int64_t t;      // global term index
  int r;          // shift
};

__device__ __forceinline__ ItemInfo decode_item(const InstDesc* __restrict__ insts,
                                                const RangeDesc* __restrict__ ranges, int n_ranges,
                                                int64_t g) {
  const int ri = find_range(ranges, n_ranges, g);
  const RangeDesc R = ranges[ri];
  const int64_t local = g - R.item_begin;
  ItemInfo it;
  it.I = insts + R.inst;
  it.i = R.term_begin + local / R.n_shifts;
  it.r = (int)(local - (local / R.n_shifts) * R.n_shifts);
  it.t = it.I->term_base + it.i;
  return it;
}

// Out-of-line double-precision normal CDF and quantile (HIP device library),
// so the unrolled chain does not inline several copies of them.
__device__ __noinline__ double ncdf64(double t) { return normcdf(t); }
__device__ __noinline__ double ncdfinv64(double u) { return normcdfinv(u); }

template <int K>
__global__ __launch_bounds__(64 * kQmcWaves) __attribute__((amdgpu_waves_per_eu(4))) void qmc_f64(const InstDesc* __restrict__ insts,
                                                          const RangeDesc* __restrict__ ranges,
                                                          int n_ranges, int64_t n_items,
                                                          const Aux64* __restrict__ aux64,
                                                          const uint64_t* __restrict__ Zg,
                                                          double* __restrict__ sums) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g = (int64_t)blockIdx.x * kQmcWaves + wave;
  if (g >= n_items) return;
  const ItemInfo it = decode_item(insts, ranges, n_ranges, g);
  const InstDesc& I = *it.I;
  const double* __restrict__ prep = reinterpret_cast<const double*>(I.prep) + it.i * I.prep_stride;
  const double e0 = aux64[it.t].e0;
  const int N = I.n_points;

  uint64_t U[K], step[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t S = lattice_shift(I.seed, it.i, it.r, j);
    U[j] = (uint64_t)(lane + 1) * Zg[j] + S;
    step[j] = Zg[j] << 6;
  }
  double acc_num = 0.0, acc_den = 0.0;
  for (int p0 = 1; p0 <= N; p0 += 64) {
    const bool live = p0 + lane <= N;
    double y[K];
    double e = e0, prod = e0;
    bool alive = e0 > 0.0;
#pragma unroll
    for (int a = 1; a <= K; ++a) {
      const double w = lattice_coord_f64(U[a - 1]);
      U[a - 1] += step[a - 1];
      const double u = fmax(w * e, 2.2250738585072014e-308);
      y[a - 1] = alive ? ncdfinv64(u) : 0.0;
      const double* row = prep + a * (a + 1) / 2;
      double acc = row[a];
#pragma unroll
      for (int c = 0; c < a; ++c) acc -= row[c] * y[c];
      e = alive ? ncdf64(acc) : 0.0;
      alive = alive && e > 0.0;
      if (a < K) prod *= e;
    }
    if (live) {
      acc_den += prod;
      acc_num += prod * e;
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  if (lane == 0) {
    double* o = sums + 3 * (I.sums_base + it.i * I.n_shifts + it.r);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = -1.0;
  }
}

__device__ __forceinline__ double exp_to_f64(float l) {
  // exp(l) for l <= 0 as 2^n * 2^f in double, l log2(e) = n + f, f in [0, 1).
  const float q2 = l * kLog2e;
  const float fl = floorf(q2);
  const float v = fast_exp2(q2 - fl);
  return ldexp((double)v, (int)fl);
}

template <int K>
__global__ __launch_bounds__(64 * kQmcWaves) void qmc_f32(const InstDesc* __restrict__ insts,
                                                          const RangeDesc* __restrict__ ranges,
                                                          int n_ranges, int64_t n_items,
                                                          const Aux32* __restrict__ aux32,
                                                          const uint64_t* __restrict__ Zg,
                                                          double* __restrict__ sums) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g = (int64_t)blockIdx.x * kQmcWaves + wave;
  if (g >= n_items) return;
  const ItemInfo it = decode_item(insts, ranges, n_ranges, g);
  const InstDesc& I = *it.I;
  const float* __restrict__ prep = reinterpret_cast<const float*>(I.prep) + it.i * I.prep_stride;
  const Aux32 ax = aux32[it.t];
  const int N = I.n_points;

  uint32_t Uh[K], Ul[K], sh[K], sl[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t S = lattice_shift(I.seed, it.i, it.r, j);
    const uint64_t u = (uint64_t)(lane + 1) * Zg[j] + S;
    const uint64_t st = Zg[j] << 6;
    Uh[j] = (uint32_t)(u >> 32);
    Ul[j] = (uint32_t)u;
    sh[j] = (uint32_t)(st >> 32);
    sl[j] = (uint32_t)st;
  }
  double acc_num = 0.0, acc_den = 0.0, acc_cnum = 0.0;
  for (int p0 = 1; p0 <= N; p0 += 64) {
    const bool live = p0 + lane <= N;
    float y[K];
    float e = ax.e0, ec = ax.ec0, le = ax.le0;
    float lsum = 0.0f;
#pragma unroll
    for (int a = 1; a <= K; ++a) {
      const uint32_t cell = lattice_cell_f32(Uh[a - 1], Ul[a - 1]);
      {
        const uint64_t u = ((uint64_t)Uh[a - 1] << 32 | Ul[a - 1]) + ((uint64_t)sh[a - 1] << 32 | sl[a - 1]);
        Uh[a - 1] = (uint32_t)(u >> 32);
        Ul[a - 1] = (uint32_t)u;
      }
      const float w = (float)(2u * cell + 1u) * 0x1p-24f;
      const float wc = 1.0f - w;
      const float u = w * e;
      const bool lower = u <= 0.5f;
      const float q = lower ? u : fmaf(w, ec, wc);
      float lq2 = fast_log2(q);
      if (q < 1e-30f) lq2 = fast_log2(w) + le * kLog2e;
      const float z = ninv_tail_from_log2(lq2);
      y[a - 1] = lower ? -z : z;
      const float* row = prep + a * (a + 1) / 2;
      float acc = row[a];
#pragma unroll
      for (int c = 0; c < a; ++c) acc = fmaf(-row[c], y[c], acc);
      const PhiOut ph = phi_f32(acc);
      e = ph.e;
      ec = ph.ec;
      le = ph.le;
      if (a < K) lsum += le;
    }
    if (live) {
      const double den = exp_to_f64(lsum);
      acc_den += den;
      acc_num = fma(den, (double)e, acc_num);
      acc_cnum = fma(den, (double)ec, acc_cnum);
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  acc_cnum = wave_sum(acc_cnum);
  if (lane == 0) {
    double* o = sums + 3 * (I.sums_base + it.i * I.n_shifts + it.r);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = acc_cnum;
  }
}

template <int K>
hipError_t qmc_dispatch(int precision, const InstDesc* insts, const RangeDesc* ranges, int n_ranges,
                        int64_t n_items, const Aux64* aux64, const Aux32* aux32, const uint64_t* Z,
                        double* sums, hipStream_t s) {
  const int64_t blocks = (n_items + kQmcWaves - 1) / kQmcWaves;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (precision == VECCHIA_FP32_LOOP)
    hipLaunchKernelGGL(qmc_f32<K>, dim3((unsigned)blocks), dim3(64 * kQmcWaves), 0, s, insts,
                       ranges, n_ranges, n_items, aux32, Z, sums);
  else
    hipLaunchKernelGGL(qmc_f64<K>, dim3((unsigned)blocks), dim3(64 * kQmcWaves), 0, s, insts,
                       ranges, n_ranges, n_items, aux64, Z, sums);
  return hipGetLastError();
}

template <int... Ks>
hipError_t qmc_switch(int K, int precision, const InstDesc* insts, const RangeDesc* ranges,
                      int n_ranges, int64_t n_items, const Aux64* aux64, const Aux32* aux32,
                      const uint64_t* Z, double* sums, hipStream_t s,
                      std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks + 1 ? (err = qmc_dispatch<Ks + 1>(precision, insts, ranges, n_ranges, n_items, aux64,
                                              aux32, Z, sums, s), 0) : 0), ...);
  return err;
}

}  // namespace

hipError_t launch_qmc(int K, int precision, const InstDesc* d_insts, const RangeDesc* d_ranges,
                      int n_ranges, int64_t n_items, const Aux64* aux64, const Aux32* aux32,
                      const uint64_t* d_Z, double* sums, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (K < 1 || K > kMaxM) return hipErrorInvalidValue;
  return qmc_switch(K, precision, d_insts, d_ranges, n_ranges, n_items, aux64, aux32, d_Z, sums, s,
                    std::make_integer_sequence<int, kMaxM>{});
}

}  // namespace vecchia
