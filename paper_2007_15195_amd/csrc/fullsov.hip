// Full-dimension SOV estimate of log Phi_D(x / scale) (Genz's method over all D
// variables), the comparator the paper checks the Vecchia approximation
// against (Section 3.1, Figures 1-4), on the plan's ordering and covariance.
//
//   1. full_cov_build: the dense D x D covariance (plan order, FP64) and b = x / scale;
//   2. blocked right-looking Cholesky, block 32: chol_diag (one wave, LDS),
//      chol_panel (one thread per row below the block), chol_update (16 x 16
//      tiles of the trailing lower triangle);
//   3. chol_mirror copies L into the upper triangle (L^T), so that a column of L
//      is contiguous;
//   4. full_sov: one thread per lattice point, one workgroup per 256 points of
//      one shift. Dimensions advance in blocks of 16: the block's partial sums
//      b_a - sum_{c<j0} L_ac y_c come from the earlier y (read back from HBM,
//      coalesced, each load feeding 16 FMAs) against the column L[j0.., c] read
//      through the scalar cache (uniform across the workgroup); inside the block
//      the recursion runs in registers:
//          e_a = Phi(t_a), log prod += log Phi(t_a), y_a = Phi^-1(max(w_a e_a, DBL_MIN)).
//      Each workgroup leaves {max, sum exp(. - max)} of its points' log products;
//   5. full_final: per shift l_r = log mean over points, then
//      log F = log mean_r exp(l_r) and the delta-method SE over the shifts.
// Lattice: Z_j from the first D - 1 primes; the shift of dimension j in
// replicate r is SplitMix64 output 2^63 + r 2^32 + j of the call's seed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "device_cov.h"
#include "lattice.h"
#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr int kCholB = 32;     // Cholesky block
constexpr int kSovB = 32;      // SOV dimension block (registers)
constexpr int kSovThreads = 256;

struct CovArgs {
  const double* xs;
  const double* ys;
  const double* covmat;
  const int32_t* perm;
  const double* x;
  double inv_scale, sigma2, range, nugget, nu;
  int32_t family;
};

__global__ __launch_bounds__(256) void full_cov_build(CovArgs a, int64_t D, double* __restrict__ A,
                                                      double* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x & 15);
  const int64_t i = (int64_t)blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= D || j > i) return;
  double v;
  if (a.covmat) {
    v = a.covmat[i * D + j];
  } else {
#pragma clang fp contract(off)
    const double dx = a.xs[i] - a.xs[j];
    const double dy = a.ys[i] - a.ys[j];
    v = cov_kernel(sqrt(dx * dx + dy * dy), a.family, a.nu, a.sigma2, a.range);
    if (i == j) v += a.nugget;
  }
  A[i * D + j] = v;
  if (j == 0) b[i] = a.x[a.perm[i]] * a.inv_scale;
}

// Factor the diagonal block [k0, k0 + n) in place (one wave; left-looking, one
// lane per row). A non-positive pivot writes NaN on the diagonal.
__global__ __launch_bounds__(64) void chol_diag(double* __restrict__ A, int64_t D, int64_t k0, int n) {
  __shared__ double C[kCholB][kCholB + 1];
  __shared__ double piv;
  const int lane = threadIdx.x;
  for (int idx = lane; idx < n * n; idx += 64) {
    const int r = idx / n, c = idx - r * n;
    if (c <= r) C[r][c] = A[(k0 + r) * D + k0 + c];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    if (lane >= j && lane < n) {
      s = C[lane][j];
      for (int p = 0; p < j; ++p) s -= C[lane][p] * C[j][p];
    }
    if (lane == j) piv = s;
    __syncthreads();
    const double d = piv;
    const double ljj = d > 0.0 ? sqrt(d) : __builtin_nan("");
    if (lane > j && lane < n) C[lane][j] = s / ljj;
    if (lane == j) C[j][j] = ljj;
    __syncthreads();
  }
  for (int idx = lane; idx < n * n; idx += 64) {
    const int r = idx / n, c = idx - r * n;
    if (c <= r) A[(k0 + r) * D + k0 + c] = C[r][c];
  }
}

// Rows i >= k0 + n: L[i, k0:k0+n] = A[i, k0:k0+n] L_kk^-T (forward substitution).
__global__ __launch_bounds__(256) void chol_panel(double* __restrict__ A, int64_t D, int64_t k0, int n) {
  __shared__ double Lk[kCholB][kCholB + 1];
  for (int idx = threadIdx.x; idx < n * n; idx += 256) {
    const int r = idx / n, c = idx - r * n;
    Lk[r][c] = c <= r ? A[(k0 + r) * D + k0 + c] : 0.0;
  }
  __syncthreads();
  const int64_t i = k0 + n + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= D) return;
  double* row = A + i * D + k0;
  double xr[kCholB];
#pragma unroll
  for (int c = 0; c < kCholB; ++c) {
    if (c < n) {
      double v = row[c];
#pragma unroll
      for (int d = 0; d < c; ++d) v -= xr[d] * Lk[c][d];
      xr[c] = v / Lk[c][c];
      row[c] = xr[c];
    }
  }
}

// Trailing update of the lower triangle: A[i][j] -= sum_c L[i][k0+c] L[j][k0+c]
// for k0 + n <= j <= i (16 x 16 tiles; tiles above the diagonal exit).
__global__ __launch_bounds__(256) void chol_update(double* __restrict__ A, int64_t D, int64_t k0, int n) {
  const int64_t base = k0 + n;
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double Pi[16][kCholB + 1], Pj[16][kCholB + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int idx = threadIdx.x; idx < 16 * n; idx += 256) {
    const int r = idx / n, c = idx - r * n;
    const int64_t ri = base + ti * 16 + r, rj = base + tj * 16 + r;
    Pi[r][c] = ri < D ? A[ri * D + k0 + c] : 0.0;
    Pj[r][c] = rj < D ? A[rj * D + k0 + c] : 0.0;
  }
  __syncthreads();
  const int64_t i = base + ti * 16 + ty, j = base + tj * 16 + tx;
  if (i >= D || j > i) return;
  double s = 0.0;
  for (int c = 0; c < n; ++c) s += Pi[ty][c] * Pj[tx][c];
  A[i * D + j] -= s;
}

// Upper triangle := L^T (A[j][i] = A[i][j] for j < i), 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void chol_mirror(double* __restrict__ A, int64_t D) {
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double T[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = ti * 32 + r, j = tj * 32 + tx;
    T[r][tx] = (i < D && j < D && j < i) ? A[i * D + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = tj * 32 + r, i = ti * 32 + tx;   // write A[j][i] = L[i][j]
    if (i < D && j < D && j < i) A[j * D + i] = T[tx][r];
  }
}

__device__ __forceinline__ double log_ncdf(double t) {
  return t < 0.0 ? log(0.5 * erfcx(-t * 0.70710678118654752440)) - 0.5 * t * t
                 : log1p(-0.5 * erfc(t * 0.70710678118654752440));
}

// The FP64 quantile stays out of line: inlined, it takes full_sov to the full
// register file with spills.
__device__ __forceinline__ double ncdf_full(double t) { return normcdf(t); }
__device__ __noinline__ double ncdfinv_full(double u) { return normcdfinv(u); }

// L: D x D with L in the lower triangle and L^T in the upper; b: D limits;
// Z: D - 1 generators; Y: (D - 1) x S (S = N R), the y of every point,
// dimension-major; part: R x gridDim.x partial {max, sum exp}. Separate
// restrict-qualified arguments let the uniform column reads of L go through
// the scalar cache.
struct SovSizes {
  int64_t D, N, S;
  uint64_t seed;
};

__global__ __launch_bounds__(kSovThreads) void full_sov(const double* __restrict__ L, const double* __restrict__ bl,
                                                        const uint64_t* __restrict__ Zt, double* __restrict__ Y,
                                                        double2* __restrict__ part, SovSizes a) {
  __shared__ double Ld[2 * kSovB][kSovB + 1];   // the block's own rows, then zeros
  __shared__ double red_m[kSovThreads / 64], red_s[kSovThreads / 64];
  const int r = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * kSovThreads + threadIdx.x;   // point p + 1
  const bool live = p < a.N;
  const int64_t s = (int64_t)r * a.N + (live ? p : 0);
  const int64_t D = a.D;
  double lp = 0.0, e = 0.0;
  for (int64_t j0 = 0; j0 < D; j0 += kSovB) {
    const int nb = (int)(D - j0 < kSovB ? D - j0 : kSovB);
    double acc[kSovB];
#pragma unroll
    for (int q = 0; q < kSovB; ++q) acc[q] = q < nb ? bl[j0 + q] : 0.0;
    // earlier dimensions: acc_q -= sum_{c < j0} L[j0 + q][c] y_c, the column
    // L[j0.., c] being row c of the mirrored upper triangle (c < j0 <= j0 + q).
    // All kSovB entries are read (wide scalar loads); in a last, ragged block
    // the ones past the row end fall in row c + 1 or in the limits that follow A
    // in the workspace, and only feed acc entries that are never used.
    const double* __restrict__ Lu = L + j0;
#pragma unroll 2
    for (int64_t c = 0; c < j0; ++c) {
      // streamed past the caches: each y is read once per block
      const double yc = __builtin_nontemporal_load(&Y[c * a.S + s]);
      const double* __restrict__ col = Lu + c * D;
#pragma unroll
      for (int q = 0; q < kSovB; ++q) acc[q] -= col[q] * yc;
    }
    // the block's own rows, zero past its end, so that row q + 1 + i below is
    // always in the array
    __syncthreads();
    for (int idx = threadIdx.x; idx < 2 * kSovB * kSovB; idx += kSovThreads) {
      const int q = idx / kSovB, c = idx - q * kSovB;
      Ld[q][c] = (q < nb && c <= q) ? L[(j0 + q) * D + j0 + c] : 0.0;
    }
    __syncthreads();
    // The recursion inside the block, right-looking: acc[0] always holds the
    // current dimension's (b - sum L y); once its y is drawn, the later entries
    // take their term in it and move down one place. The loop is not unrolled,
    // so the Phi and Phi^-1 code is inlined once and acc stays in registers.
#pragma unroll 1
    for (int q = 0; q < nb; ++q) {
      const double t = acc[0] / Ld[q][q];
      e = ncdf_full(t);
      lp += log_ncdf(t);
      const int64_t dim = j0 + q;
      double y = 0.0;
      if (dim < D - 1) {
        const uint64_t S = splitmix64(a.seed, (1ULL << 63) | ((uint64_t)r << 32) | (uint64_t)dim);
        const uint64_t U = (uint64_t)(p + 1) * Zt[dim] + S;
        const double w = lattice_coord_f64(U);
        y = ncdfinv_full(fmax(w * e, 2.2250738585072014e-308));
        if (live) Y[dim * a.S + s] = y;
      }
#pragma unroll
      for (int i = 0; i + 1 < kSovB; ++i) acc[i] = acc[i + 1] - Ld[q + 1 + i][q] * y;
    }
  }
  // workgroup {max, sum exp(lp - max)} over its live points
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double m = live ? lp : -HUGE_VAL;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (lane == 0) red_m[wv] = m;
  __syncthreads();
  double M = red_m[0];
  for (int k = 1; k < kSovThreads / 64; ++k) M = fmax(M, red_m[k]);
  double x = (live && M > -HUGE_VAL) ? exp(lp - M) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if (lane == 0) red_s[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int k = 0; k < kSovThreads / 64; ++k) sum += red_s[k];
    part[(int64_t)r * gridDim.x + blockIdx.x] = make_double2(M, sum);
  }
}

// log of the mean over points of shift r, from its workgroup partials (in order)
__device__ double shift_logmean(const double2* __restrict__ part, int nblk, int r, int64_t N) {
  double M = -HUGE_VAL;
  for (int k = 0; k < nblk; ++k) M = fmax(M, part[(int64_t)r * nblk + k].x);
  if (!(M > -HUGE_VAL)) return M;
  double sum = 0.0;
  for (int k = 0; k < nblk; ++k) {
    const double2 v = part[(int64_t)r * nblk + k];
    if (v.x > -HUGE_VAL) sum += v.y * exp(v.x - M);
  }
  return M + log(sum) - log((double)N);
}

// One thread: the shifts' log means, then log F and the delta-method SE.
__global__ void full_final(const double2* __restrict__ part, int nblk, int R, int64_t N, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double top = -HUGE_VAL;
  for (int r = 0; r < R; ++r) top = fmax(top, shift_logmean(part, nblk, r, N));
  double logF = top, se = __builtin_nan("");
  if (top > -HUGE_VAL) {
    double sum = 0.0;
    for (int r = 0; r < R; ++r) sum += exp(shift_logmean(part, nblk, r, N) - top);
    logF = top + log(sum) - log((double)R);
    if (R > 1) {
      double acc = 0.0;
      for (int r = 0; r < R; ++r) {
        const double d = exp(shift_logmean(part, nblk, r, N) - logF) - 1.0;
        acc += d * d;
      }
      se = sqrt(acc / ((double)R * (R - 1)));
    }
  }
  out[0] = logF;
  out[1] = se;
}

}  // namespace
}  // namespace vecchia

extern "C" vecchia_status vecchia_full_logcdf(vecchia_plan_t plan, const double* x_dev, double scale,
                                              const vecchia_cov* cov_override, const vecchia_qmc* q,
                                              double* out_dev, void* hip_stream) {
  using namespace vecchia;
  if (!plan || !q || !x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::string why;
  if (!valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (q->precision != VECCHIA_FP64) return set_error(VECCHIA_E_INVALID, "the full-dimension estimator runs in FP64");
  if (q->n_shifts > 1024) return set_error(VECCHIA_E_INVALID, "n_shifts must be at most 1024 here");
  if (plan->n_obs > 0) return set_error(VECCHIA_E_INVALID, "not defined for a censored plan");
  if (!(std::isfinite(scale) && scale > 0)) return set_error(VECCHIA_E_INVALID, "scale must be finite and > 0");
  const vecchia_cov c = cov_override ? *cov_override : plan->cov;
  if (cov_override) {
    if (!valid_cov(c, &why)) return set_error(VECCHIA_E_INVALID, why);
    if (!plan->matrix && (c.family != plan->cov.family || (c.family == VECCHIA_COV_MATERN && c.nu != plan->cov.nu)))
      return set_error(VECCHIA_E_INVALID, "covariance override must keep the plan's family and nu");
  }
  const int64_t D = plan->D, N = q->n_points, R = q->n_shifts;
  const int64_t S = N * R;
  // workspace: A (D x D), b (D), Y ((D-1) x S), then the partials at a 16-byte offset
  const int64_t n_head = D * D + D + std::max<int64_t>(1, D - 1) * S;
  const int64_t n_head_even = n_head + (n_head & 1);
  const double bytes = 8.0 * (double)n_head_even + 16.0 * R * ((N + kSovThreads - 1) / kSovThreads);
  if (D > 40000 || bytes > 64e9)
    return set_error(VECCHIA_E_INVALID, "the full-dimension estimator needs D <= 40000 and at most 64 GB of workspace");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::lock_guard<std::mutex> lk(plan->mu);
  hipError_t e = hipSuccess;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "device query");
  const uint64_t* Zt = device_lattice_table_n(dev, (int)std::max<int64_t>(1, D - 1), &e);
  if (!Zt) return hip_error(e, "lattice table");
  const size_t need = (size_t)bytes + 1024;
  if (plan->full_bytes < need) {
    hipFree(plan->d_full);
    plan->d_full = nullptr;
    plan->full_bytes = 0;
    e = hipMalloc(&plan->d_full, need);
    if (e != hipSuccess) {
      plan->d_full = nullptr;
      return hip_error(e, "full-dimension workspace");
    }
    plan->full_bytes = need;
  }
  double* A = reinterpret_cast<double*>(plan->d_full);
  double* b = A + D * D;
  double* Y = b + D;
  double2* part = reinterpret_cast<double2*>(A + n_head_even);
  CovArgs ca{plan->d_xs, plan->d_ys, plan->d_cov, plan->d_perm, x_dev, 1.0 / scale, c.sigma2, c.range, c.nugget,
             c.family == VECCHIA_COV_EXPONENTIAL ? 0.5 : c.nu, c.family};
  const unsigned tiles = (unsigned)((D + 15) / 16);
  hipLaunchKernelGGL(full_cov_build, dim3(tiles, tiles), dim3(256), 0, s, ca, D, A, b);
  e = hipGetLastError();
  for (int64_t k0 = 0; k0 < D && e == hipSuccess; k0 += kCholB) {
    const int n = (int)std::min<int64_t>(kCholB, D - k0);
    hipLaunchKernelGGL(chol_diag, dim3(1), dim3(64), 0, s, A, D, k0, n);
    e = hipGetLastError();
    const int64_t rest = D - k0 - n;
    if (e == hipSuccess && rest > 0) {
      hipLaunchKernelGGL(chol_panel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, A, D, k0, n);
      e = hipGetLastError();
      const unsigned t = (unsigned)((rest + 15) / 16);   // 16 x 16 tiles of the trailing triangle
      if (e == hipSuccess) {
        hipLaunchKernelGGL(chol_update, dim3(t, t), dim3(256), 0, s, A, D, k0, n);
        e = hipGetLastError();
      }
    }
  }
  if (e == hipSuccess) {
    const unsigned t32 = (unsigned)((D + 31) / 32);
    hipLaunchKernelGGL(chol_mirror, dim3(t32, t32), dim3(256), 0, s, A, D);
    e = hipGetLastError();
  }
  const unsigned nblk = (unsigned)((N + kSovThreads - 1) / kSovThreads);
  if (e == hipSuccess) {
    SovSizes sz{D, N, S, q->seed};
    hipLaunchKernelGGL(full_sov, dim3(nblk, (unsigned)R), dim3(kSovThreads), 0, s, A, b, Zt, Y, part, sz);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(full_final, dim3(1), dim3(64), 0, s, part, (int)nblk, (int)R, N, out_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_error(e, "full-dimension launch");
  return VECCHIA_OK;
}
