// term_setup: steps a2-a3 of every Vecchia term (Section 2.2, eq. (6)).
//
// One wave per term, with LDS blocks sized for the batch's largest term (16, 32
// or 64 variables). The term's variables are its conditioning set N_i (in the
// plan's (d^2, index) order) followed by i itself. The wave gathers their
// locations and thresholds b = x / scale, builds the covariance block C in LDS
// (FP64), factors C = L L^T in place (left-looking, one lane per row) and writes
// the rows the SOV chain needs, scaled by the diagonal:
//     row a (a = 0..K):  L_a0/L_aa, ..., L_a,a-1/L_aa, b_a/L_aa
// at offset a(a+1)/2 of the term's block, so that t_a = b_a/L_aa - sum_c (L_ac/L_aa) y_c.
// It also stores Phi(b_0/L_00), the exact value of a term with K = 0.
//
// Censored plans (Section 4, eq. (11)): plan positions below n_obs are sites
// whose value is observed. Their q neighbours among those sites are placed
// first, then the censored neighbours, then i. With E the first q variables,
// the lower-right block of L is the Cholesky factor of the covariance of the
// rest given X_E = b_E, and their conditional mean is L_{A,E} w with
// w = L_EE^-1 b_E; the rows written are those of the rest, with b_a replaced by
// b_a - sum_{c<q} L_ac w_c, so the chain runs in K = k - q dimensions. For an
// observed site i every neighbour is observed (q = k) and the term is the
// Gaussian conditional density of eq. (4) at scale r, times the Jacobian 1 / r:
//     log f = -log(2 pi)/2 - log L_kk - z^2/2 + log(1/r),  z = (b_k - sum_{c<k} L_kc w_c) / L_kk.
//
// Block plans (joint terms, Section 3.2): term i's variables are listed
// explicitly (conditioning set first, then the group) and the rows of all of
// them are written; the QMC kernel takes the denominator at the term's split.
//
// A pivot <= 0 (or NaN) marks the term NOT_PD: its outputs become NaN and the
// instance's bad_term is lowered to i.
//
// Infinite thresholds: +inf leaves a variable unconstrained (its factor is 1;
// the FP32 rows cap the scaled limit at 2^20, where Phi is 1 in FP32 as well).
// A term with a limit of -inf, or with an observed site whose value is
// infinite (zero density), is 0: e0 = -1 marks it, lt0 = -inf is its value
// with SE 0, and its rows get finite limits so the QMC kernels run a harmless
// chain whose sums are never read.
#include "device_cov.h"
#include "device_math_f64.h"
#include "fp32_math_coeffs.h"
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

// Set-up of global term t by the calling wave (one wave per block). redo: the
// term of an FP32 evaluation is run again in FP64; only its FP64 rows are
// written, in place of its FP32 rows. KV: the most variables of any term of
// the batch (16, 32 or 64); the LDS blocks are sized for it, so that smaller
// conditioning sets fit more waves on a compute unit.
template <int KV>
__device__ __forceinline__ void setup_term(const InstDesc* __restrict__ insts, int n_inst,
                                           const int64_t* __restrict__ term_bases, Aux64* __restrict__ aux64,
                                           Aux32* __restrict__ aux32, int64_t t, bool redo) {
  __shared__ double C[KV][KV + 1];
  __shared__ double px[KV], py[KV], pb[KV], pw[KV];
  __shared__ long long pslot;
  __shared__ int pv[KV];
  __shared__ double piv;
  const int lane = threadIdx.x;
  const int ii = find_inst(term_bases, n_inst, t);
  const InstDesc& I = insts[ii];
  const int64_t i = t - term_bases[ii];
  const bool blk = I.bvars != nullptr;
  const int boff = blk ? I.bvar_off[i] : 0;
  const int k = blk ? I.bvar_off[i + 1] - boff - 1 : I.kcnt[i];
  const int n = k + 1;
  if (n > KV) {   // the host sizes KV for every term of the batch; never taken
    if (lane == 0) atomicMin((long long*)I.bad_term, (long long)i);
    return;
  }
  // variable slot of each lane's neighbour: observed neighbours first (censored
  // plans only), each group in the stored order, i last
  const int64_t v = blk ? (lane < n ? (int64_t)I.bvars[boff + lane] : 0)
                        : (lane < k ? (int64_t)I.nbr[i * I.m + lane] : i);
  const bool eq = lane < k && v < I.n_obs;
  const uint64_t eq_mask = __ballot(eq);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int q = __popcll(eq_mask);
  const int slot = lane >= k ? lane : eq ? __popcll(eq_mask & below) : q + (lane - __popcll(eq_mask & below));
  double bl = 0.0;
  if (lane < n) {
    pv[slot] = (int)v;
    if (!I.covmat) {
      px[slot] = I.xs[v];
      py[slot] = I.ys[v];
    }
    bl = I.x[I.perm[v]] * I.inv_scale;
    pb[slot] = bl;
  }
  const bool zero = __ballot(lane < n && (bl == -HUGE_VAL || (v < I.n_obs && __builtin_isinf(bl)))) != 0;
  __syncthreads();
  for (int idx = lane; idx < n * n; idx += 64) {
    const int a = idx / n;
    const int c = idx - a * n;
    if (c > a) continue;
    double cv;
    if (I.covmat) {
      cv = I.covmat[(int64_t)pv[a] * I.D + pv[c]];
    } else {
#pragma clang fp contract(off)
      const double dx = px[a] - px[c];
      const double dy = py[a] - py[c];
      cv = cov_kernel(sqrt(dx * dx + dy * dy), I.family, I.nu, I.sigma2, I.range);
      if (a == c) cv += I.nugget;
    }
    C[a][c] = cv;
  }
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    if (lane >= j && lane < n) {
      s = C[lane][j];
      for (int p = 0; p < j; ++p) s -= C[lane][p] * C[j][p];
    }
    if (lane == j) piv = s;
    __syncthreads();
    const double d = piv;
    if (!(d > 0.0)) bad = true;
    const double ljj = sqrt(d);
    if (lane > j && lane < n) C[lane][j] = s / ljj;
    if (lane == j) C[j][j] = ljj;
    __syncthreads();
  }
  // w = L_EE^-1 b_E (forward substitution, q <= k steps) and the shifted limits
  if (lane == 0) {
    for (int c = 0; c < q; ++c) {
      double acc = pb[c];
      for (int p = 0; p < c; ++p) acc -= C[c][p] * pw[p];
      pw[c] = acc / C[c][c];
    }
  }
  __syncthreads();
  double bs = 0.0;
  if (lane >= q && lane < n) {
    bs = pb[lane];
    for (int c = 0; c < q; ++c) bs -= C[lane][c] * pw[c];
    pb[lane] = bs;
  }
  __syncthreads();
  // FP32 instances: a chain variable whose limit lies below kPromoteZ standard
  // deviations of its distribution given the observed sites (limit bs, variance
  // the row norm of the conditional block of L) sends the term to the FP64
  // kernel: deep lower tails are where the FP32 loop's rounding of the scaled
  // limits shows
  double zc = HUGE_VAL;
  if (lane >= q && lane < n) {
    double r2 = 0.0;
    for (int c = q; c <= lane; ++c) r2 += C[lane][c] * C[lane][c];
    zc = bs / sqrt(r2);
  }
  const bool want_promote = !redo && I.precision == VECCHIA_FP32_LOOP && __ballot(zc < kPromoteZ) != 0;
  const double nan = __builtin_nan("");
  const bool f32 = I.precision == VECCHIA_FP32_LOOP;
  const bool density = i < I.n_obs;
  // a promoted term takes the next slot of the batch's list, which has room for
  // every term; its FP64 rows replace its FP32 rows
  bool promoted = redo;
  if (want_promote && !density && !bad && !zero && n - q >= 2) {
    if (lane == 0) pslot = (long long)atomicAdd(reinterpret_cast<unsigned long long*>(I.pctr), 1ULL);
    __syncthreads();
    promoted = true;
  }
  if (promoted && lane >= q && lane < n) {
    const int a = lane - q;
    const double laa = C[lane][lane];
    double* row = prep_f64(I, i) + (int64_t)a * (a + 1) / 2;
    for (int c = 0; c < a; ++c) row[c] = C[lane][q + c] / laa;
    row[a] = bs / laa;
  }
  if (redo) return;
  if (f32 && lane == 0) {
    I.promote[t] = promoted ? 1 : 0;
    if (promoted && pslot < I.plist_cap) I.plist[pslot] = (int32_t)t;
  }
  if (!density && !promoted && lane >= q && lane < n) {
    const int a = lane - q;   // row of the conditional block
    const double laa = C[lane][lane];
    const int64_t off = i * (int64_t)I.prep_stride + (int64_t)a * (a + 1) / 2;
    if (f32) {
      // the FP32 loop works with v = kappa t (exp(-t^2/2) = 2^(-v^2))
      const double sc = kPhiScale / laa;
      float* row = reinterpret_cast<float*>(I.prep) + off;
      for (int c = 0; c < a; ++c) row[c] = (float)(C[lane][q + c] * sc);
      double bv = bs * sc;
      if (bv > 0x1p20) bv = 0x1p20;
      row[a] = bad ? __builtin_nanf("") : zero ? 0.0f : (float)bv;
    } else {
      double* row = reinterpret_cast<double*>(I.prep) + off;
      for (int c = 0; c < a; ++c) row[c] = C[lane][q + c] / laa;
      row[a] = bad ? nan : zero ? 0.0 : bs / laa;
    }
  }
  if (lane == 0) {
    if (density) {
      const double lkk = C[k][k];
      const double z = pb[k] / lkk;
      const double lf = -0.91893853320467274178 - log(lkk) - 0.5 * z * z + log(I.inv_scale);
      aux64[t].e0 = bad ? nan : exp(lf);
      aux64[t].lt0 = bad ? nan : lf;
      if (f32) aux32[t] = Aux32{0.0f, 0.0f, 0.0f, 0.0f};
    } else {
      const double b0 = pb[q] / C[q][q];
      const double e0 = bad ? nan : phi64(b0);
      aux64[t].e0 = e0;
      aux64[t].lt0 = bad ? nan : log(e0);
      if (f32) {
        // e0 as em0 * 2^en0: split only below 2^-100 (the loop's first quantile
        // argument w e0 then stays a normal FP32 number)
        Aux32 a;
        a.neg0 = b0 <= 0.0 ? 1.0f : 0.0f;
        if (e0 < 0x1p-100) {
          int ex = 0;
          const double mt = frexp(e0, &ex);
          a.em0 = (float)mt;
          a.en0 = (float)ex;
        } else {
          a.em0 = (float)e0;
          a.en0 = 0.0f;
        }
        a.ec0 = bad ? __builtin_nanf("") : (float)phi64(-b0);
        aux32[t] = a;
      }
    }
    if (zero && !bad) {
      aux64[t].e0 = -1.0;
      aux64[t].lt0 = -HUGE_VAL;
      if (f32) aux32[t] = Aux32{0.5f, 0.0f, 0.5f, 1.0f};
    }
    if (bad) atomicMin((long long*)I.bad_term, (long long)i);
  }
}

template <int KV>
__global__ __launch_bounds__(64) void term_setup(const InstDesc* __restrict__ insts, int n_inst,
                                                 const int64_t* __restrict__ term_bases,
                                                 Aux64* __restrict__ aux64,
                                                 Aux32* __restrict__ aux32, int64_t term_base) {
  setup_term<KV>(insts, n_inst, term_bases, aux64, aux32, term_base + (int64_t)blockIdx.x, false);
}

// The re-run list's terms, one per wave in turn; every wave leaves once the
// list (read once, written by the finalize before this launch) is used up.
template <int KV>
__global__ __launch_bounds__(64) void term_setup_redo(const InstDesc* __restrict__ insts, int n_inst,
                                                      const int64_t* __restrict__ term_bases,
                                                      Aux64* __restrict__ aux64, Aux32* __restrict__ aux32,
                                                      const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ count, int64_t cap) {
  const int64_t n = min(*count, cap);
  for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
    setup_term<KV>(insts, n_inst, term_bases, aux64, aux32, (int64_t)list[e], true);
    __syncthreads();   // the next term reuses the LDS blocks
  }
}

}  // namespace

// Tile size for the batch's largest term: 16, 32 or 64 variables.
static int setup_tile(int max_vars) { return max_vars <= 16 ? 16 : max_vars <= 32 ? 32 : 64; }

template <int KV>
static hipError_t launch_setup_kv(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                                  int64_t total_terms, Aux64* aux64, Aux32* aux32, hipStream_t s) {
  constexpr int64_t kPer = kMaxLaunchThreads / 64;   // terms (one wave each) per launch
  for (int64_t b = 0; b < total_terms; b += kPer) {
    const unsigned n = (unsigned)(total_terms - b < kPer ? total_terms - b : kPer);
    hipLaunchKernelGGL(term_setup<KV>, dim3(n), dim3(64), 0, s, d_insts, n_inst, d_term_bases, aux64, aux32, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_setup(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                        int64_t total_terms, int max_vars, Aux64* aux64, Aux32* aux32, hipStream_t s) {
  if (total_terms <= 0) return hipSuccess;
  if (total_terms > 0x7fffffffLL || max_vars < 1 || max_vars > kMaxVars) return hipErrorInvalidValue;
  switch (setup_tile(max_vars)) {
    case 16: return launch_setup_kv<16>(d_insts, n_inst, d_term_bases, total_terms, aux64, aux32, s);
    case 32: return launch_setup_kv<32>(d_insts, n_inst, d_term_bases, total_terms, aux64, aux32, s);
    default: return launch_setup_kv<64>(d_insts, n_inst, d_term_bases, total_terms, aux64, aux32, s);
  }
}

hipError_t launch_setup_redo(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases, int max_vars,
                             Aux64* aux64, Aux32* aux32, const int32_t* list, const int64_t* count, int64_t cap,
                             hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  if (max_vars < 1 || max_vars > kMaxVars) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(cap < 1024 ? cap : 1024);
  switch (setup_tile(max_vars)) {
    case 16:
      hipLaunchKernelGGL(term_setup_redo<16>, dim3(grid), dim3(64), 0, s, d_insts, n_inst, d_term_bases, aux64,
                         aux32, list, count, cap);
      break;
    case 32:
      hipLaunchKernelGGL(term_setup_redo<32>, dim3(grid), dim3(64), 0, s, d_insts, n_inst, d_term_bases, aux64,
                         aux32, list, count, cap);
      break;
    default:
      hipLaunchKernelGGL(term_setup_redo<64>, dim3(grid), dim3(64), 0, s, d_insts, n_inst, d_term_bases, aux64,
                         aux32, list, count, cap);
  }
  return hipGetLastError();
}

}  // namespace vecchia
