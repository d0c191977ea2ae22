// QMC kernels: steps a4-a5 of every Vecchia term (Section 2.2, eq. (6); Genz's
// separation of variables with a randomized lattice rule).
//
// Work item = (term, shift, chunk): one wave evaluates one chunk of the N
// lattice points of one random shift of one term, points across the 64 lanes.
// A launch covers the terms of one conditioning-set size K, a template
// parameter, so the chain is fully unrolled and y[] stays in registers. Per chain (variables 0..K, the term's own component last):
//     e_0 = Phi(b'_0)                         (constant, from term_setup)
//     y_{a-1} = Phi^{-1}(w_{a-1} e_{a-1})      a = 1..K
//     t_a = b'_a - sum_{c<a} L'_ac y_c,   e_a = Phi(t_a)
//     den = prod_{a<K} e_a,   num = den * e_K
// (the constant e_0 cancels from the ratio and is left out of the FP32
// products). Joint block terms (Section 3.2; the BLOCK variants) keep every
// factor in the product instead and take the denominator at the term's split s:
//     den = prod_{a<s} e_a (1 for s = 0),   num = prod_{a<=K} e_a,
// with 1 - prod_{a>=s} e_a carried as its own recurrence for the FP32 log1p form.
// The wave writes {sum num, sum den, sum den*(1-e_K)} of its chunk,
// summed over lanes by a fixed butterfly, so an item's result does not depend on
// where or with what else it runs.
//
// FP64 chain: the plain parity path (the normal CDF and quantile of device_math_f64.h).
// FP32 chain: single precision with every factor e carried as a base-2 log
// split em * 2^en; the products keep a separate exponent, so they cannot
// underflow, and are rebuilt exactly in FP64 for the accumulation.
#include "device_math_f32.h"
#include "device_math_f64.h"
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

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// true when the predicate holds on some active lane (the ballot's mask is a
// scalar, so the result is wave-uniform)
__device__ __forceinline__ bool any_lane(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

// The work item of this block. Consecutive blocks go to the chip's 8 XCDs in
// turn (block b to XCD b mod 8), each with its own L2; the blocks of one XCD
// take one contiguous range of the launch's items instead, so that the items
// of one term (consecutive) share an L2 for the term's rows and for the lines
// of their partial sums. A bijection of [0, gridDim.x) for any grid size; the
// results do not depend on it.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ int64_t block_item(int64_t item_base) {
  const unsigned b = blockIdx.x, n = gridDim.x;
  const unsigned x = b % kXcds, j = b / kXcds, q = n / kXcds, r = n % kXcds;
  return item_base + (int64_t)(x * q + (x < r ? x : r) + j);
}

struct Item {
  const InstDesc* I;
  int64_t i;      // plan index of the term
  int64_t t;      // global term index
  int r;          // pass * n_shifts + shift: the item's slot among the term's shifts
  int sr;         // shift
  bool second;    // pass 1: the term's second lattice (independent-points estimator)
  int c;          // chunk
  int K;
};

__device__ __forceinline__ Item decode_item(const InstDesc* __restrict__ insts,
                                            const RangeDesc* __restrict__ ranges, int n_ranges,
                                            int64_t g) {
  const int ri = uniform(find_range(ranges, n_ranges, g));
  const RangeDesc& R = ranges[ri];
  const int local = uniform((int)(g - R.item_begin));      // < 2^31 per range
  const int ipt = R.items_per_term;
  const int term_off = uniform(local / ipt);
  const int rem = local - term_off * ipt;
  Item it;
  it.I = insts + R.inst;
  it.i = R.term_begin + term_off;
  it.r = uniform(rem / R.n_chunks);
  it.c = uniform(rem - it.r * R.n_chunks);
  const int ns = uniform(it.I->n_shifts);
  it.second = it.r >= ns;
  it.sr = it.second ? it.r - ns : it.r;
  it.K = uniform(R.K);
  it.t = it.I->term_base + it.i;
  return it;
}

// The term's scaled rows are staged in LDS once per work item (one wave per
// block) and read from there in every step: broadcast reads at LDS latency
// instead of L1/L2 round trips. Measured on gfx950 this is neutral for small K
// and up to 1.3x (FP32) / 2.4x (FP64) faster for large K, whose rows no longer
// fit the vector L1 beside the other resident waves.
__device__ __forceinline__ double* item_out(const InstDesc& I, const Item& it, double* sums) {
  return sums + 3 * (I.sums_base + (it.i * I.passes * I.n_shifts + it.r) * (int64_t)I.n_chunks + it.c);
}

// Out-of-line double-precision normal CDF and quantile (device_math_f64.h), so
// the unrolled chain does not inline several copies of them.
__device__ __noinline__ double ncdf64(double t) { return phi64(t); }
__device__ __noinline__ double ncdfinv64(double u) { return ninv64(u); }

template <int K, bool BLOCK>
__device__ __forceinline__ void item_f64(const Item& it, const Aux64* __restrict__ aux64,
                                         const uint64_t* __restrict__ Zg, double* __restrict__ sums) {
  const InstDesc& I = *it.I;
  const int lane = threadIdx.x & 63;
  const int sp = BLOCK ? uniform(I.split[it.i]) : K;   // denominator: the first sp factors
  const double* __restrict__ prep = reinterpret_cast<const double*>(I.prep) + it.i * I.prep_stride;
  const double e0 = aux64[it.t].e0;
  const int p_begin = 1 + it.c * I.chunk_points;
  const int p_last = min(I.n_points, p_begin + I.chunk_points - 1);
  // the lane's chain starts at point p_begin + lane and strides 64 (U_j += 64 Z_j)
  uint64_t U[K];
#pragma unroll
  for (int j = 0; j < K; ++j)
    U[j] = (uint64_t)(p_begin + lane) * Zg[j] + lattice_shift(I.seed, it.i, it.sr, j, it.second);
  constexpr int kRowElems = (K + 1) * (K + 2) / 2;   // rows 0..K of the term's block
  __shared__ double srow[kRowElems];
  for (int e = lane; e < kRowElems; e += 64) srow[e] = prep[e];
  __syncthreads();
  double acc_num = 0.0, acc_den = 0.0;
  for (int p0 = p_begin; p0 <= p_last; p0 += 64) {
    __asm__ volatile("" ::: "memory");   // re-read the term's rows each iteration
    const bool live = p0 + lane <= p_last;
    double y[K];
    double e = e0, prod = e0;
    double head = 1.0;   // BLOCK: prod_{a<sp} e_a
    bool alive = e0 > 0.0;
#pragma unroll
    for (int a = 1; a <= K; ++a) {
      if (BLOCK && a == sp) head = prod;
      const double w = lattice_coord_f64(U[a - 1]);
      U[a - 1] += Zg[a - 1] << 6;
      const double u = fmax(w * e, 2.2250738585072014e-308);
      y[a - 1] = alive ? ncdfinv64(u) : 0.0;
      const double* row = srow + a * (a + 1) / 2;
      double acc = row[a];
#pragma unroll
      for (int c = 0; c < a; ++c) acc -= row[c] * y[c];
      e = alive ? ncdf64(acc) : 0.0;
      alive = alive && e > 0.0;
      if (BLOCK || a < K) prod *= e;
    }
    if (live) {
      // no contraction here: a fused prod * e_{K-1} + acc_den would add the
      // unrounded product to den while num takes the rounded one
#pragma clang fp contract(off)
      if (BLOCK) {
        acc_den += head;
        acc_num += prod;
      } else {
        acc_den += prod;
        acc_num += prod * e;
      }
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  if (lane == 0) {
    double* o = item_out(I, it, sums);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = -1.0;
  }
}

constexpr float kDeepV = 7.74596669f;   // sqrt(60)


// FP32 chain of one lane. Factors are e = em * 2^en, with en = 0 except for
// lower-tail factors below 2^-60 (t < -9.1), which keep 2^floor(-v^2) in en so
// that em stays in [R, 2R). A wave-uniform flag `split` records that some
// lane's current factor has en != 0; without it the step carries no exponent
// arithmetic at all, and the wave takes the exponent branches only in the rare
// steps that need them. The product of e_1..e_{K-1} is qm * 2^qe (qe an
// integer), renormalised when some lane's qm falls below 2^-50; every factor
// is >= 2^-65, so qm never leaves the normal range.
template <int K, bool BLOCK>
__device__ __forceinline__ void item_f32(const Item& it, const Aux32* __restrict__ aux32,
                                         const uint64_t* __restrict__ Zg, double* __restrict__ sums) {
  const InstDesc& I = *it.I;
  if (uniform(I.promote[it.t]) != 0) return;   // this term runs in FP64 (qmc_promoted)
  const int lane = threadIdx.x & 63;
  const int sp = BLOCK ? uniform(I.split[it.i]) : K;   // denominator: the first sp factors
  const float* __restrict__ prep = reinterpret_cast<const float*>(I.prep) + it.i * I.prep_stride;
  const Aux32 ax = aux32[it.t];
  const bool split0 = uniform(ax.en0 != 0.0f) != 0;
  const int p_begin = 1 + it.c * I.chunk_points;
  const int p_last = min(I.n_points, p_begin + I.chunk_points - 1);
  // the lane's chain starts at point p_begin + lane and strides 64: U_j += 64 Z_j
  // per iteration, with Z_j re-read (scalar load) in the loop so the K steps do
  // not occupy 2K SGPRs across it
  uint64_t U[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t S = lattice_shift(I.seed, it.i, it.sr, j, it.second);
    U[j] = (uint64_t)(p_begin + lane) * Zg[j] + S;
  }
  constexpr int kRowElems = (K + 1) * (K + 2) / 2;   // rows 0..K of the term's block
  __shared__ float srow[kRowElems];
  for (int e = lane; e < kRowElems; e += 64) srow[e] = prep[e];
  __syncthreads();
  double acc_num = 0.0, acc_den = 0.0, acc_cnum = 0.0;
  for (int p0 = p_begin; p0 <= p_last; p0 += 64) {
    // compiler-only barrier: the term's rows are re-read from LDS in every
    // iteration instead of being held in K(K+3)/2 registers across the loop
    __asm__ volatile("" ::: "memory");
    float y[K];
    float em = ax.em0, en = ax.en0, m = ax.ec0;   // e_0 and 1 - e_0 (the latter used when t_0 > 0)
    bool neg = ax.neg0 != 0.0f;
    bool split = split0;
    float qm = 1.0f;
    int qe = 0;
    float dm = 1.0f;   // BLOCK: prod_{a<sp} e_a = dm 2^de
    int de = 0;
    float cc = 0.0f;   // BLOCK: 1 - prod_{sp<=a} e_a so far
    if (BLOCK) {
      // every factor is in the products, e_0 included
      qe = (int)ax.en0 + __builtin_amdgcn_frexp_expf(ax.em0);
      qm = __builtin_amdgcn_frexp_mantf(ax.em0);
      if (sp == 0) cc = ax.ec0;
    }
#pragma unroll
    for (int a = 1; a <= K; ++a) {
      if (BLOCK && a == sp) {
        dm = qm;
        de = qe;
      }
      const int ro = a * (a + 1) / 2;
      const CoordF32 wp = lattice_coord_f32((uint32_t)(U[a - 1] >> 32));
      U[a - 1] += Zg[a - 1] << 6;
      // y = Phi^{-1}(u), u = w e; u <= 1/2 whenever the previous t <= 0, and
      // otherwise 1 - u = (1 - w) + w (1 - e) keeps its digits
      const float um = wp.w * em;
      const bool lower = neg || um <= 0.5f;
      const float qt = lower ? um : fmaf(wp.w, m, wp.wc);
      const float lq = fast_log2(qt);
      float z = ninv_tail_from_log2(lq);
      if (__builtin_expect(split, 0)) {   // some lane's e carries 2^en
        z = ninv_tail_from_log2_split(lq + en);
        en = 0.0f;
        split = false;
      }
      y[a - 1] = lower ? -z : z;
      float v = srow[ro + a];
#pragma unroll
      for (int c = 0; c < a; ++c) v = fmaf(-srow[ro + c], y[c], v);
      const PhiParts ph = phi_f32(v);
      em = ph.em;
      m = ph.m;
      neg = ph.neg;
      // deep: Phi(t) < 2^-60, i.e. v < -sqrt(60); the compare's lane mask is
      // taken directly (LLVM predicate 4 = ordered less-than)
      if (__builtin_expect(__builtin_amdgcn_fcmpf(v, -kDeepV, 4) != 0, 0)) {
        if (v < -kDeepV) {
          // exponent kept outside the float (bounded so that qe cannot overflow)
          const float fl = floorf(fmaxf(ph.f, -1048576.0f));
          em = fast_exp2(fmaxf(ph.f, -1048576.0f) - fl) * ph.R;
          en = fl;
          if (BLOCK || a < K) qe += (int)fl;
        }
        split = true;
      }
      if (BLOCK && a >= sp) {
        const float eca = neg ? 1.0f - ldexpf(em, (int)en) : m;
        cc = fmaf(eca, 1.0f - cc, cc);
      }
      if (BLOCK || a < K) {
        qm *= em;
        const bool low = qm < 0x1p-50f;
        if (__builtin_expect(any_lane(low), 0)) {
          if (low) {
            qe += __builtin_amdgcn_frexp_expf(qm);
            qm = __builtin_amdgcn_frexp_mantf(qm);
          }
        }
      }
    }
    // den = prod_{a<K} e_a, num = den e_K, cnum = den (1 - e_K); lanes past the
    // chunk's last point contribute zero
    const bool in_chunk = p0 + lane <= p_last;
    if (BLOCK) {
      const double den = ldexp((double)(in_chunk ? dm : 0.0f), de);
      acc_den += den;
      acc_num += ldexp((double)(in_chunk ? qm : 0.0f), qe);
      acc_cnum = fma(den, (double)cc, acc_cnum);
    } else {
      const float qml = in_chunk ? qm : 0.0f;
      const int enk = (int)en;
      const double den = ldexp((double)qml, qe);
      const double num = ldexp(den * (double)em, enk);
      const float ec = neg ? 1.0f - ldexpf(em, enk) : m;
      acc_den += den;
      acc_num += num;
      acc_cnum = fma(den, (double)ec, acc_cnum);
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  acc_cnum = wave_sum(acc_cnum);
  if (lane == 0) {
    double* o = item_out(I, it, sums);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = acc_cnum;
  }
}

// ---------------------------------------------------------------------------
// Chains of kMaxUnrolledK + 1 .. kMaxM steps (terms of 33..64 variables): the
// same recursions with a runtime K, not unrolled. Each lane's y live in LDS
// (column `lane` of ys, so the lanes' accesses never share a bank), the rows
// and the K shifts are staged in LDS once per work item, and U_j = p Z_j + S_j
// is formed from the point index in each step. One wave per block.
constexpr int kGenRowElems = (kMaxM + 1) * (kMaxM + 2) / 2;

__device__ __forceinline__ void item_f32_gen(const Item& it, const Aux32* __restrict__ aux32,
                                             const uint64_t* __restrict__ Zg, double* __restrict__ sums) {
  __shared__ float srow[kGenRowElems];
  __shared__ float ys[kMaxM][64];
  __shared__ uint64_t sh[kMaxM];
  const InstDesc& I = *it.I;
  if (uniform(I.promote[it.t]) != 0) return;   // this term runs in FP64 (qmc_promoted)
  const int lane = threadIdx.x & 63;
  const int K = it.K;
  const bool block = I.split != nullptr;
  const int sp = block ? uniform(I.split[it.i]) : K;
  const float* __restrict__ prep = reinterpret_cast<const float*>(I.prep) + it.i * I.prep_stride;
  const Aux32 ax = aux32[it.t];
  const bool split0 = uniform(ax.en0 != 0.0f) != 0;
  const int p_begin = 1 + it.c * I.chunk_points;
  const int p_last = min(I.n_points, p_begin + I.chunk_points - 1);
  const int rows = (K + 1) * (K + 2) / 2;
  for (int e = lane; e < rows; e += 64) srow[e] = prep[e];
  for (int j = lane; j < K; j += 64) sh[j] = lattice_shift(I.seed, it.i, it.sr, j, it.second);
  __syncthreads();
  double acc_num = 0.0, acc_den = 0.0, acc_cnum = 0.0;
  for (int p0 = p_begin; p0 <= p_last; p0 += 64) {
    const uint64_t pt = (uint64_t)(p0 + lane);
    float em = ax.em0, en = ax.en0, m = ax.ec0;
    bool neg = ax.neg0 != 0.0f;
    bool split = split0;
    float qm = 1.0f;
    int qe = 0;
    float dm = 1.0f;
    int de = 0;
    float cc = 0.0f;
    if (block) {
      qe = (int)ax.en0 + __builtin_amdgcn_frexp_expf(ax.em0);
      qm = __builtin_amdgcn_frexp_mantf(ax.em0);
      if (sp == 0) cc = ax.ec0;
    }
#pragma unroll 1
    for (int a = 1; a <= K; ++a) {
      if (block && a == sp) {
        dm = qm;
        de = qe;
      }
      const int ro = a * (a + 1) / 2;
      const CoordF32 wp = lattice_coord_f32((uint32_t)((pt * Zg[a - 1] + sh[a - 1]) >> 32));
      const float um = wp.w * em;
      const bool lower = neg || um <= 0.5f;
      const float qt = lower ? um : fmaf(wp.w, m, wp.wc);
      const float lq = fast_log2(qt);
      float z = ninv_tail_from_log2(lq);
      if (__builtin_expect(split, 0)) {
        z = ninv_tail_from_log2_split(lq + en);
        en = 0.0f;
        split = false;
      }
      ys[a - 1][lane] = lower ? -z : z;
      float v = srow[ro + a];
      int c = 0;
      for (; c + 4 <= a; c += 4) {
        v = fmaf(-srow[ro + c], ys[c][lane], v);
        v = fmaf(-srow[ro + c + 1], ys[c + 1][lane], v);
        v = fmaf(-srow[ro + c + 2], ys[c + 2][lane], v);
        v = fmaf(-srow[ro + c + 3], ys[c + 3][lane], v);
      }
      for (; c < a; ++c) v = fmaf(-srow[ro + c], ys[c][lane], v);
      const PhiParts ph = phi_f32(v);
      em = ph.em;
      m = ph.m;
      neg = ph.neg;
      if (__builtin_expect(__builtin_amdgcn_fcmpf(v, -kDeepV, 4) != 0, 0)) {
        if (v < -kDeepV) {
          const float fl = floorf(fmaxf(ph.f, -1048576.0f));
          em = fast_exp2(fmaxf(ph.f, -1048576.0f) - fl) * ph.R;
          en = fl;
          if (block || a < K) qe += (int)fl;
        }
        split = true;
      }
      if (block && a >= sp) {
        const float eca = neg ? 1.0f - ldexpf(em, (int)en) : m;
        cc = fmaf(eca, 1.0f - cc, cc);
      }
      if (block || a < K) {
        qm *= em;
        const bool low = qm < 0x1p-50f;
        if (__builtin_expect(any_lane(low), 0)) {
          if (low) {
            qe += __builtin_amdgcn_frexp_expf(qm);
            qm = __builtin_amdgcn_frexp_mantf(qm);
          }
        }
      }
    }
    const bool in_chunk = p0 + lane <= p_last;
    if (block) {
      const double den = ldexp((double)(in_chunk ? dm : 0.0f), de);
      acc_den += den;
      acc_num += ldexp((double)(in_chunk ? qm : 0.0f), qe);
      acc_cnum = fma(den, (double)cc, acc_cnum);
    } else {
      const float qml = in_chunk ? qm : 0.0f;
      const int enk = (int)en;
      const double den = ldexp((double)qml, qe);
      const double num = ldexp(den * (double)em, enk);
      const float ec = neg ? 1.0f - ldexpf(em, enk) : m;
      acc_den += den;
      acc_num += num;
      acc_cnum = fma(den, (double)ec, acc_cnum);
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  acc_cnum = wave_sum(acc_cnum);
  if (lane == 0) {
    double* o = item_out(I, it, sums);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = acc_cnum;
  }
}

// prep: the term's FP64 rows (the instance's own, or a promoted term's slot)
__device__ __forceinline__ void item_f64_gen(const Item& it, const Aux64* __restrict__ aux64,
                                             const uint64_t* __restrict__ Zg, double* __restrict__ sums,
                                             const double* __restrict__ prep) {
  __shared__ double srow[kGenRowElems];
  __shared__ double ys[kMaxM][64];
  __shared__ uint64_t sh[kMaxM];
  const InstDesc& I = *it.I;
  const int lane = threadIdx.x & 63;
  const int K = it.K;
  const bool block = I.split != nullptr;
  const int sp = block ? uniform(I.split[it.i]) : K;
  const double e0 = aux64[it.t].e0;
  const int p_begin = 1 + it.c * I.chunk_points;
  const int p_last = min(I.n_points, p_begin + I.chunk_points - 1);
  const int rows = (K + 1) * (K + 2) / 2;
  for (int e = lane; e < rows; e += 64) srow[e] = prep[e];
  for (int j = lane; j < K; j += 64) sh[j] = lattice_shift(I.seed, it.i, it.sr, j, it.second);
  __syncthreads();
  double acc_num = 0.0, acc_den = 0.0;
  for (int p0 = p_begin; p0 <= p_last; p0 += 64) {
    const uint64_t pt = (uint64_t)(p0 + lane);
    const bool live = p0 + lane <= p_last;
    double e = e0, prod = e0, head = 1.0;
    bool alive = e0 > 0.0;
#pragma unroll 1
    for (int a = 1; a <= K; ++a) {
      if (block && a == sp) head = prod;
      const double w = lattice_coord_f64(pt * Zg[a - 1] + sh[a - 1]);
      const double u = fmax(w * e, 2.2250738585072014e-308);
      ys[a - 1][lane] = alive ? ncdfinv64(u) : 0.0;
      const double* row = srow + a * (a + 1) / 2;
      double acc = row[a];
      for (int c = 0; c < a; ++c) acc -= row[c] * ys[c][lane];
      e = alive ? ncdf64(acc) : 0.0;
      alive = alive && e > 0.0;
      if (block || a < K) prod *= e;
    }
    if (live) {
#pragma clang fp contract(off)
      if (block) {
        acc_den += head;
        acc_num += prod;
      } else {
        acc_den += prod;
        acc_num += prod * e;
      }
    }
  }
  acc_num = wave_sum(acc_num);
  acc_den = wave_sum(acc_den);
  if (lane == 0) {
    double* o = item_out(I, it, sums);
    o[0] = acc_num;
    o[1] = acc_den;
    o[2] = -1.0;
  }
}

__global__ __launch_bounds__(64) void qmc_gen_f32(const InstDesc* __restrict__ insts,
                                                  const RangeDesc* __restrict__ ranges, int n_ranges,
                                                  const Aux32* __restrict__ aux32, const uint64_t* __restrict__ Zg,
                                                  double* __restrict__ sums, int64_t item_base) {
  const Item it = decode_item(insts, ranges, n_ranges, block_item(item_base));
  item_f32_gen(it, aux32, Zg, sums);
}

__global__ __launch_bounds__(64) void qmc_gen_f64(const InstDesc* __restrict__ insts,
                                                  const RangeDesc* __restrict__ ranges, int n_ranges,
                                                  const Aux64* __restrict__ aux64, const uint64_t* __restrict__ Zg,
                                                  double* __restrict__ sums, int64_t item_base) {
  const Item it = decode_item(insts, ranges, n_ranges, block_item(item_base));
  item_f64_gen(it, aux64, Zg, sums, reinterpret_cast<const double*>(it.I->prep) + it.i * it.I->prep_stride);
}

__device__ __forceinline__ int find_inst_q(const int64_t* __restrict__ bases, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bases[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Handed-over terms of FP32 instances, in FP64: each wave takes the next
// (list entry, item) pair from the work counter ctr[1] until the count x
// ipt_max pairs are used up; pairs past a term's own item count are skipped.
// Every wave leaves once the counter passes the end, so the grid always drains.
__global__ __launch_bounds__(64) void qmc_promoted(const InstDesc* __restrict__ insts, int n_inst,
                                                   const int64_t* __restrict__ term_bases,
                                                   const Aux64* __restrict__ aux64, const uint64_t* __restrict__ Zg,
                                                   double* __restrict__ sums, const int32_t* __restrict__ list,
                                                   int64_t* __restrict__ ctr, int64_t cap, int ipt_max) {
  const int lane = threadIdx.x;
  const int64_t count = min(ctr[0], cap);
  if (count == 0) return;   // nothing handed over: no wave touches the work counter
  const int64_t total = count * (int64_t)ipt_max;
  for (;;) {
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[1]), 1ULL);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
    const int64_t v = (int64_t)(((uint64_t)hi << 32) | lo);
    if (v >= total) break;
    const int64_t e = v / ipt_max;
    const int j = (int)(v - e * ipt_max);
    const int64_t t = uniform(list[e]);
    const int ii = uniform(find_inst_q(term_bases, n_inst, t));
    const InstDesc& I = insts[ii];
    const int ns = uniform(I.n_shifts), nc = uniform(I.n_chunks);
    if (j >= uniform(I.passes) * ns * nc) continue;
    Item it;
    it.I = &I;
    it.i = t - term_bases[ii];
    it.t = t;
    it.r = j / nc;
    it.c = j - it.r * nc;
    it.second = it.r >= ns;
    it.sr = it.second ? it.r - ns : it.r;
    it.K = uniform(I.sovk[it.i]);
    item_f64_gen(it, aux64, Zg, sums, prep_f64(I, it.i));
  }
}

hipError_t qmc_gen_dispatch(int precision, const InstDesc* insts, const RangeDesc* ranges, int n_ranges,
                            int64_t n_items, const Aux64* aux64, const Aux32* aux32, const uint64_t* Z,
                            double* sums, hipStream_t s) {
  if (n_items > 0x7fffffffLL) return hipErrorInvalidValue;
  constexpr int64_t kPer = kMaxLaunchThreads / 64;   // items (one wave each) per launch
  for (int64_t b = 0; b < n_items; b += kPer) {
    const unsigned n = (unsigned)(n_items - b < kPer ? n_items - b : kPer);
    if (precision == VECCHIA_FP32_LOOP)
      hipLaunchKernelGGL(qmc_gen_f32, dim3(n), dim3(64), 0, s, insts, ranges, n_ranges, aux32, Z, sums, b);
    else
      hipLaunchKernelGGL(qmc_gen_f64, dim3(n), dim3(64), 0, s, insts, ranges, n_ranges, aux64, Z, sums, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Minimum waves per SIMD requested per chain size K: the largest value at which
// the unrolled chain still compiles without spilling (measured on gfx950; the
// hint only caps registers, so chains that fit more waves keep them).
constexpr int f32_min_waves(int K) { return K <= 30 ? 4 : K <= 40 ? 3 : 2; }
constexpr int f64_min_waves(int K) { return K <= 11 ? 4 : K <= 18 ? 3 : 2; }

template <int K, bool BLOCK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(f64_min_waves(K)))) void qmc_f64(
    const InstDesc* __restrict__ insts, const RangeDesc* __restrict__ ranges, int n_ranges,
    const Aux64* __restrict__ aux64, const uint64_t* __restrict__ Zg, double* __restrict__ sums,
    int64_t item_base) {
  const Item it = decode_item(insts, ranges, n_ranges, block_item(item_base));
  item_f64<K, BLOCK>(it, aux64, Zg, sums);
}


template <int K, bool BLOCK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(f32_min_waves(K)))) void qmc_f32(
    const InstDesc* __restrict__ insts,
                                              const RangeDesc* __restrict__ ranges, int n_ranges,
                                              const Aux32* __restrict__ aux32,
                                              const uint64_t* __restrict__ Zg, double* __restrict__ sums,
                                              int64_t item_base) {
  const Item it = decode_item(insts, ranges, n_ranges, block_item(item_base));
  item_f32<K, BLOCK>(it, aux32, Zg, sums);
}

template <int K, bool BLOCK>
hipError_t qmc_dispatch(int precision, const InstDesc* insts, const RangeDesc* ranges, int n_ranges,
                        int64_t n_items, const Aux64* aux64, const Aux32* aux32, const uint64_t* Z,
                        double* sums, hipStream_t s) {
  if (n_items > 0x7fffffffLL) return hipErrorInvalidValue;
  constexpr int64_t kPer = kMaxLaunchThreads / 64;   // items (one wave each) per launch
  for (int64_t b = 0; b < n_items; b += kPer) {
    const unsigned n = (unsigned)(n_items - b < kPer ? n_items - b : kPer);
    if (precision == VECCHIA_FP32_LOOP)
      hipLaunchKernelGGL((qmc_f32<K, BLOCK>), dim3(n), dim3(64), 0, s, insts, ranges, n_ranges, aux32, Z, sums, b);
    else
      hipLaunchKernelGGL((qmc_f64<K, BLOCK>), dim3(n), dim3(64), 0, s, insts, ranges, n_ranges, aux64, Z, sums, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool BLOCK, int... Ks>
hipError_t qmc_switch(int K, int precision, const InstDesc* insts, const RangeDesc* ranges,
                      int n_ranges, int64_t n_items, const Aux64* aux64, const Aux32* aux32,
                      const uint64_t* Z, double* sums, hipStream_t s, std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks + 1 ? (err = qmc_dispatch<Ks + 1, BLOCK>(precision, insts, ranges, n_ranges, n_items, aux64,
                                                     aux32, Z, sums, s), 0) : 0), ...);
  return err;
}

// FP32 plain chains of 32..63 steps: unrolled like the shorter ones
template <int... Ks>
hipError_t qmc_switch_f32_long(int K, const InstDesc* insts, const RangeDesc* ranges, int n_ranges,
                               int64_t n_items, const Aux64* aux64, const Aux32* aux32, const uint64_t* Z,
                               double* sums, hipStream_t s, std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks + kMaxUnrolledK + 1
        ? (err = qmc_dispatch<Ks + kMaxUnrolledK + 1, false>(VECCHIA_FP32_LOOP, insts, ranges, n_ranges, n_items,
                                                              aux64, aux32, Z, sums, s), 0)
        : 0), ...);
  return err;
}

}  // namespace

hipError_t launch_qmc_promoted(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases, const Aux64* aux64,
                               const uint64_t* d_Z, double* sums, const int32_t* list, int64_t* ctr, int64_t cap,
                               int ipt_max, hipStream_t s) {
  if (cap <= 0 || ipt_max <= 0) return hipSuccess;
  const int64_t pairs = cap * (int64_t)ipt_max;
  const unsigned grid = (unsigned)(pairs < 2048 ? pairs : 2048);
  hipLaunchKernelGGL(qmc_promoted, dim3(grid), dim3(64), 0, s, d_insts, n_inst, d_term_bases, aux64, d_Z, sums,
                     list, ctr, cap, ipt_max);
  return hipGetLastError();
}

hipError_t launch_qmc(int K, int precision, bool block, const InstDesc* d_insts, const RangeDesc* d_ranges,
                      int n_ranges, int64_t n_items, const Aux64* aux64, const Aux32* aux32,
                      const uint64_t* d_Z, double* sums, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (K < 1 || K > kMaxM) return hipErrorInvalidValue;
  if (K > kMaxUnrolledK && precision == VECCHIA_FP32_LOOP && !block)
    return qmc_switch_f32_long(K, d_insts, d_ranges, n_ranges, n_items, aux64, aux32, d_Z, sums, s,
                               std::make_integer_sequence<int, kMaxM - kMaxUnrolledK>{});
  if (K > kMaxUnrolledK)
    return qmc_gen_dispatch(precision, d_insts, d_ranges, n_ranges, n_items, aux64, aux32, d_Z, sums, s);
  if (block)
    return qmc_switch<true>(K, precision, d_insts, d_ranges, n_ranges, n_items, aux64, aux32, d_Z, sums, s,
                            std::make_integer_sequence<int, kMaxUnrolledK>{});
  return qmc_switch<false>(K, precision, d_insts, d_ranges, n_ranges, n_items, aux64, aux32, d_Z, sums, s,
                           std::make_integer_sequence<int, kMaxUnrolledK>{});
}

}  // namespace vecchia
