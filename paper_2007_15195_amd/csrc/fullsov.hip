// Full-dimension SOV estimate of log Phi_D(x / scale) (Genz's method over all D
// variables), the comparator the paper checks the Vecchia approximation
// against (Section 3.1, Figures 1-4), on the plan's ordering and covariance.
//
//   1. full_cov_build: the dense D x D covariance (plan order, FP64) and b = x / scale;
//   2. blocked right-looking Cholesky, block 32: chol_diag (one wave, rows in registers),
//      chol_panel (one thread per row below the block), chol_update (64 x 64
//      tiles of the trailing lower triangle on the FP64 matrix cores);
//   3. chol_mirror copies L into the upper triangle (L^T), so that a column of L
//      is contiguous;
//   4. full_sov: one workgroup per 16 to 64 consecutive lattice points of one
//      shift (16 per wave) for the whole chain; dimensions advance in blocks of
//      64. The part of each block's limits that comes from earlier dimensions,
//      b_a - sum_{c<j0} L_ac y_c, is a product of 64 rows of L by the earlier y
//      of the workgroup's points, run on the FP64 matrix cores
//      (v_mfma_f64_16x16x4); the block's own recursion then runs from LDS in
//      each wave (its four 16-lane groups evaluate the same 16 points, and each
//      group updates every fourth later row):
//          e_a = Phi(t_a), log prod += log Phi(t_a), y_a = Phi^-1(max(w_a e_a, DBL_MIN)).
//      Each wave leaves {max, sum exp(. - max)} of its points' log products;
//   5. full_final (one workgroup, fixed-order trees): per shift l_r = log mean
//      over points, then log F = log mean_r exp(l_r) and the delta-method SE
//      over the shifts.
// Lattice: Z_j from the first D - 1 primes; the shift of dimension j in
// replicate r is SplitMix64 output 2^63 + r 2^32 + j of the call's seed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "device_cov.h"
#include "device_math_f64.h"
#include "lattice.h"
#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr int kCholB = 32;     // Cholesky block
constexpr int kFsB = 64;       // SOV dimension block
constexpr int kFsWavePts = 16; // lattice points per wave (one MFMA column tile)

// v_mfma_f64_16x16x4f64, D = A B + C with A 16 x 4, B 4 x 16: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], and holds D[4 e + l / 16][l % 16] in
// element e of its four-double result (checked on gfx950).
typedef double fs_d4 __attribute__((ext_vector_type(4)));

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

// Factor the diagonal block [k0, k0 + n) in place (one wave; right-looking,
// lane r holds row r of the block in registers). Column j's pivot is broadcast
// from lane j, the column goes through LDS, and each lane updates its own row
// with independent FMAs. A non-positive pivot writes NaN on the diagonal.
__global__ __launch_bounds__(64) void chol_diag(double* __restrict__ A, int64_t D, int64_t k0, int n) {
  __shared__ double col[kCholB];
  const int lane = threadIdx.x;
  double c[kCholB];
#pragma unroll
  for (int p = 0; p < kCholB; ++p) c[p] = (lane < n && p <= lane) ? A[(k0 + lane) * D + k0 + p] : 0.0;
#pragma unroll
  for (int j = 0; j < kCholB; ++j) {
    if (j < n) {
      const double d = __shfl(c[j], j, 64);
      const double ljj = d > 0.0 ? sqrt(d) : __builtin_nan("");
      c[j] = lane > j ? c[j] / ljj : (lane == j ? ljj : c[j]);
      if (lane < kCholB) col[lane] = c[j];
      __syncthreads();
#pragma unroll
      for (int p = j + 1; p < kCholB; ++p)
        if (p <= lane) c[p] -= c[j] * col[p];
      __syncthreads();   // every lane has read the column before the next one is written
    }
  }
#pragma unroll
  for (int p = 0; p < kCholB; ++p)
    if (lane < n && p <= lane) A[(k0 + lane) * D + k0 + p] = c[p];
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
// for k0 + n <= j <= i, in 64 x 64 tiles (tiles above the diagonal exit). The
// tile's two panels are staged in LDS column-major (Pt[c][row], zero past the
// panel or the matrix), and each of the four waves takes a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f64_16x16x4 over the panel's kCholB columns.
__global__ __launch_bounds__(256) void chol_update(double* __restrict__ A, int64_t D, int64_t k0, int n) {
  const int64_t base = k0 + n;
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double Pi[kCholB][64 + 1], Pj[kCholB][64 + 1];
  for (int idx = threadIdx.x; idx < 64 * kCholB; idx += 256) {
    const int r = idx / kCholB, c = idx - r * kCholB;
    const int64_t ri = base + ti * 64 + r, rj = base + tj * 64 + r;
    Pi[c][r] = (c < n && ri < D) ? A[ri * D + k0 + c] : 0.0;
    Pj[c][r] = (c < n && rj < D) ? A[rj * D + k0 + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wi = wv >> 1, wj = wv & 1;
  const int m = lane & 15, kq = lane >> 4;
  fs_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = fs_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < kCholB / 4; ++ks) {
    const int c = 4 * ks + kq;
    const double a0 = Pi[c][32 * wi + m], a1 = Pi[c][32 * wi + 16 + m];
    const double b0 = Pj[c][32 * wj + m], b1 = Pj[c][32 * wj + 16 + m];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // acc[a][b] element e (the MFMA's output layout): row 32 wi + 16 a + 4 e + kq,
  // column 32 wj + 16 b + m of the tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = base + ti * 64 + 32 * wi + 16 * a + 4 * e + kq;
        const int64_t j = base + tj * 64 + 32 * wj + 16 * b + m;
        if (i < D && j <= i) A[i * D + j] -= acc[a][b][e];
      }
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

// The FP64 normal CDF and quantile of device_math_f64.h, both out of line:
// inlined into the recursion they would take registers the product loop needs.
__device__ __noinline__ double ncdf_full(double t) { return phi64(t); }
__device__ __noinline__ double ncdfinv_full(double u) { return ninv64(u); }

// L: D x D with L in the lower triangle and L^T in the upper; b: D limits;
// Z: D - 1 generators; Y: (D - 1) x S (S = N R), the y of every point,
// dimension-major; part: R x gridDim.x partial {max, sum exp}.
struct SovSizes {
  int64_t D, N, S;
  uint64_t seed;
};

// Each wave owns 16 consecutive lattice points of one shift (blockIdx.y) for the
// whole chain, and a workgroup holds NW such waves; dimensions advance in
// blocks of kFsB. A wave depends only on its own points' y:
//  * Earlier dimensions: T[q][p] = b_{j0+q} - sum_{c<j0} L[j0+q][c] y_c[p] is a
//    (kFsB x j0) by (j0 x 16) product, taken as four 16 x 16 tiles of
//    v_mfma_f64_16x16x4: the A operand is L[j0 + 16 i + m][c0 + k] (row c0 + k
//    of the mirrored upper triangle, 16 consecutive doubles per k), the B
//    operand y_{c0 + k} of the wave's 16 points (16 consecutive doubles of Y);
//    four MFMAs per step of 4, the next step's loads issued before them.
//  * The block itself: T goes to the wave's LDS slice and the wave runs the
//    recursion right-looking over the block's rows (the block's triangle of L
//    staged in LDS once per workgroup); lane group g = lane / 16 updates the
//    rows q' = q + 1 + g, q + 5 + g, ... of the wave's 16 points:
//        e = Phi(t_q), log prod += log Phi(t_q), y_q = Phi^-1(max(w_q e, DBL_MIN)),
//        T[q'] -= L[j0 + q'][j0 + q] y_q for q' > q.
// Two workgroup barriers per block guard the shared triangle; the wave's own y
// (global) and T (LDS) need only its own ordering.
template <int NW>
__global__ __launch_bounds__(64 * NW) void full_sov(const double* __restrict__ L, const double* __restrict__ bl,
                                                    const uint64_t* __restrict__ Zt, double* __restrict__ Y,
                                                    double2* __restrict__ part, SovSizes a) {
  __shared__ double T[NW][kFsB][kFsWavePts + 1];
  __shared__ double Lb[kFsB * (kFsB + 1) / 2];   // the block's lower triangle, packed by rows
  __shared__ double dinv[kFsB];                  // reciprocals of the block's diagonal
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = blockIdx.y;
  const int64_t D = a.D, S = a.S, N = a.N;
  // this lane's point (column m of the wave's tile) and step offset / update group kq
  const int m = lane & 15, kq = lane >> 4;
  const int64_t pt = (int64_t)(blockIdx.x * NW + wv) * kFsWavePts + m;
  const bool live = pt < N;
  const int64_t pc = live ? pt : N - 1;   // past the shift's last point: any point of it (results unused)
  const int64_t s_own = (int64_t)r * N + pc;
  const double* __restrict__ yB = Y + s_own + (int64_t)kq * S;
  double (*Tw)[kFsWavePts + 1] = T[wv];
  double lp = 0.0;
  for (int64_t j0 = 0; j0 < D; j0 += kFsB) {
    const int nb = (int)(D - j0 < kFsB ? D - j0 : kFsB);
    fs_d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = fs_d4{0.0, 0.0, 0.0, 0.0};
    // rows past D in a last, ragged block read other entries of L (in the array
    // while j0 > 0, since then D > kFsB); their sums are never used
    const double* __restrict__ aA = L + j0 + m + (int64_t)kq * D;
    // j0 is a multiple of kFsB: whole steps of 4 earlier dimensions (a multiple
    // of 16 steps); the loads of step c0 + 4 are issued before the MFMAs of
    // step c0 (two register sets)
    const int steps = (int)(j0 / 4);
    double av[2][4], bv[2];
    auto load_step = [&](int st, int buf) {
      const int64_t c0 = (int64_t)st * 4;
      bv[buf] = __builtin_nontemporal_load(yB + c0 * S);
      const double* __restrict__ ar = aA + c0 * D;
#pragma unroll
      for (int i = 0; i < 4; ++i) av[buf][i] = ar[16 * i];
    };
    auto mfma_step = [&](int buf) {
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[buf][i], bv[buf], acc[i], 0, 0, 0);
    };
    // the loads past the last step re-read it: with every load unconditional
    // the compiler's wait counts stay exact across the loop
    if (steps > 0) {
      load_step(0, 0);
      for (int st = 0; st < steps; st += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int nx = st + u + 1;
          load_step(nx < steps ? nx : steps - 1, (u + 1) & 1);
          mfma_step(u);
        }
      }
    }
    // acc[i] element e (the MFMA's output layout): row 16 i + 4 e + kq of the
    // block, point m of the wave's tile
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * i + 4 * e + kq;
        Tw[q][m] = (q < nb ? bl[j0 + q] : 0.0) - acc[i][e];
      }
    }
    __syncthreads();   // every wave is done with the previous block's triangle
    for (int idx = tid; idx < kFsB * (kFsB + 1) / 2; idx += 64 * NW) {
      int q = (int)((__builtin_sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (q * (q + 1) / 2 > idx) --q;
      while ((q + 1) * (q + 2) / 2 <= idx) ++q;
      const int c = idx - q * (q + 1) / 2;
      Lb[idx] = q < nb ? L[(j0 + q) * D + j0 + c] : 0.0;
    }
    for (int q = tid; q < kFsB; q += 64 * NW) dinv[q] = q < nb ? 1.0 / L[(j0 + q) * D + j0 + q] : 0.0;
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < nb; ++q) {
      // every lane group evaluates the same point's factor; group 0 keeps it
      const double t = Tw[q][m] * dinv[q];
      const double e = ncdf_full(t);
      // log Phi(t) from Phi(t) itself while Phi(t) > 1e-197 (its relative
      // error is then that of the log's absolute error); the scaled
      // complementary form only where some lane's limit is at or below -30
      double lt = log(e);
      if (__builtin_expect(__any(t <= -30.0), 0)) {
        if (t <= -30.0) lt = log_ncdf(t);
      }
      lp += lt;
      const int64_t dim = j0 + q;
      if (dim < D - 1) {
        const uint64_t Sh = splitmix64(a.seed, (1ULL << 63) | ((uint64_t)r << 32) | (uint64_t)dim);
        const uint64_t U = (uint64_t)(pc + 1) * Zt[dim] + Sh;
        const double w = lattice_coord_f64(U);
        const double y = ncdfinv_full(fmax(w * e, 2.2250738585072014e-308));
        if (kq == 0 && live) Y[dim * S + s_own] = y;
#pragma unroll 2
        for (int q2 = q + 1 + kq; q2 < nb; q2 += 4) Tw[q2][m] -= Lb[q2 * (q2 + 1) / 2 + q] * y;
      }
    }
    // the wave's own y stores are read back by its next product (other lanes)
    __threadfence_block();
  }
  // the wave's {max, sum exp(lp - max)} over its live points (lane group 0)
  const bool own = live && kq == 0;
  double mx = own ? lp : -HUGE_VAL;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  double x = (own && mx > -HUGE_VAL) ? exp(lp - mx) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if (lane == 0) part[((int64_t)r * gridDim.x + blockIdx.x) * NW + wv] = make_double2(mx, x);
}

// Waves per workgroup (16 points each) for N points per shift and R shifts: four
// (one wave on each SIMD of a compute unit, sharing the workgroup's loads of L)
// unless that leaves compute units without a workgroup; then the most that
// still give every compute unit one.
int full_sov_waves(int64_t N, int64_t R, int n_cu) {
  for (int nw = 4; nw > 1; --nw) {
    const int64_t P = (int64_t)kFsWavePts * nw;
    if ((N + P - 1) / P * R >= n_cu) return nw;
  }
  return 1;
}

// One workgroup of 256: per shift r, l_r = log mean over points from the waves'
// {max, sum exp} partials (strided partial reductions, then a fixed tree, so the
// result does not depend on scheduling); then log F = log mean_r exp(l_r) and
// the delta-method SE over shifts.
__global__ __launch_bounds__(256) void full_final(const double2* __restrict__ part, int nblk, int R, int64_t N,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  auto tree = [&](double v, bool is_max) {
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] = is_max ? fmax(red[tid], red[tid + o]) : red[tid] + red[tid + o];
      __syncthreads();
    }
    const double res = red[0];
    __syncthreads();
    return res;
  };
  auto logmean = [&](int r) {
    const double2* __restrict__ pr = part + (int64_t)r * nblk;
    double mx = -HUGE_VAL;
    for (int k = tid; k < nblk; k += 256) mx = fmax(mx, pr[k].x);
    const double M = tree(mx, true);
    if (!(M > -HUGE_VAL)) return M;
    double sm = 0.0;
    for (int k = tid; k < nblk; k += 256) {
      const double2 v = pr[k];
      if (v.x > -HUGE_VAL) sm += v.y * exp(v.x - M);
    }
    return M + log(tree(sm, false)) - log((double)N);
  };
  double top = -HUGE_VAL;
  for (int r = 0; r < R; ++r) top = fmax(top, logmean(r));
  double logF = top, se = __builtin_nan("");
  if (top > -HUGE_VAL) {
    double sum = 0.0;
    for (int r = 0; r < R; ++r) sum += exp(logmean(r) - top);
    logF = top + log(sum) - log((double)R);
    if (R > 1) {
      double acc = 0.0;
      for (int r = 0; r < R; ++r) {
        const double d = exp(logmean(r) - logF) - 1.0;
        acc += d * d;
      }
      se = sqrt(acc / ((double)R * (R - 1)));
    }
  }
  if (tid == 0) {
    out[0] = logF;
    out[1] = se;
  }
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
  // partials: one per wave, at most ceil(N / 16) + 3 per shift (the last workgroup of a shift)
  const double bytes = 8.0 * (double)n_head_even + 16.0 * R * ((N + kFsWavePts - 1) / kFsWavePts + 3);
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
      const unsigned t = (unsigned)((rest + 63) / 64);   // 64 x 64 tiles of the trailing triangle
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
  hipDeviceProp_t prop{};
  int n_cu = 256;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) n_cu = prop.multiProcessorCount;
  const int nw = full_sov_waves(N, R, n_cu);
  const int64_t P = (int64_t)kFsWavePts * nw;
  const unsigned nblk = (unsigned)((N + P - 1) / P);
  // measurement hook: HIP events around the product-and-recursion kernel,
  // recorded with its D(D-1)/2 FMAs per point
  hipEvent_t pa = nullptr, pb = nullptr;
  const bool prof = e == hipSuccess && profiling_enabled() && profile_events(&pa, &pb) == hipSuccess;
  if (prof) e = hipEventRecord(pa, s);
  if (e == hipSuccess) {
    SovSizes sz{D, N, S, q->seed};
    const dim3 grid(nblk, (unsigned)R), block(64 * nw);
    if (nw == 4) hipLaunchKernelGGL(full_sov<4>, grid, block, 0, s, A, b, Zt, Y, part, sz);
    else if (nw == 3) hipLaunchKernelGGL(full_sov<3>, grid, block, 0, s, A, b, Zt, Y, part, sz);
    else if (nw == 2) hipLaunchKernelGGL(full_sov<2>, grid, block, 0, s, A, b, Zt, Y, part, sz);
    else hipLaunchKernelGGL(full_sov<1>, grid, block, 0, s, A, b, Zt, Y, part, sz);
    e = hipGetLastError();
  }
  if (prof && e == hipSuccess) {
    e = hipEventRecord(pb, s);
    if (e == hipSuccess) profile_record(VECCHIA_PROFILE_FULL_SOV, VECCHIA_FP64, pa, pb, D * (D - 1) / 2 * N * R);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(full_final, dim3(1), dim3(256), 0, s, part, (int)nblk * nw, (int)R, N, out_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_error(e, "full-dimension launch");
  return VECCHIA_OK;
}
