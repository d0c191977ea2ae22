// Plan-time kernel: nearest preceding neighbours (Section 2.1, after eq. (4);
// Section 2.2, after eq. (6)): for every plan position i, the k_i = min(m, i)
// positions j < i with the smallest keys (d^2, j), d^2 = dx*dx + dy*dy in FP64
// without fused multiply-add, listed in ascending key order.
//
// One wave per query, 8 queries per block. The block stages candidate
// coordinates through LDS in tiles, in increasing j; lane l of a wave takes the
// tile's candidates l, l+64, ... (again increasing j) and keeps its own sorted
// top-M list in registers (M is a template parameter, so the insertion network
// has static indices; a candidate tied in d^2 with a kept one never displaces
// it). The wave then merges its 64 lists: M rounds of a lexicographic
// (d^2, j) argmin butterfly across lanes, the winning lane popping its head.
#include "vecchia_internal.h"

namespace vecchia {
namespace {

constexpr int kKnnWaves = 8;
constexpr int kKnnTile = 512;

template <int M>
__global__ __launch_bounds__(64 * kKnnWaves) void knn_preceding(const double* __restrict__ xs,
                                                                const double* __restrict__ ys, int64_t D,
                                                                int32_t* __restrict__ nbr,
                                                                int32_t* __restrict__ kcnt, int64_t q_base) {
#pragma clang fp contract(off)
  __shared__ double2 tile[kKnnTile];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q0 = q_base + (int64_t)blockIdx.x * kKnnWaves;
  const int64_t i = q0 + wave;
  const bool valid = i < D;
  const double qx = valid ? xs[i] : 0.0;
  const double qy = valid ? ys[i] : 0.0;
  double bd[M];
  int bj[M];
#pragma unroll
  for (int s = 0; s < M; ++s) {
    bd[s] = HUGE_VAL;
    bj[s] = -1;
  }
  const int64_t last_query = (q0 + kKnnWaves < D ? q0 + kKnnWaves : D) - 1;
  for (int64_t t0 = 0; t0 < last_query; t0 += kKnnTile) {
    __syncthreads();
    for (int c = threadIdx.x; c < kKnnTile; c += 64 * kKnnWaves) {
      const int64_t j = t0 + c;
      if (j < D) tile[c] = make_double2(xs[j], ys[j]);
    }
    __syncthreads();
    const int64_t lim = (valid ? i : 0) - t0;
    const int cmax = (int)(lim < kKnnTile ? (lim > 0 ? lim : 0) : kKnnTile);
    for (int c = lane; c < cmax; c += 64) {
      const double2 p = tile[c];
      const double dx = p.x - qx;
      const double dy = p.y - qy;
      const double d2 = dx * dx + dy * dy;
      if (d2 < bd[M - 1]) {
        const int jj = (int)(t0 + c);
#pragma unroll
        for (int s = M - 1; s > 0; --s) {
          const bool up = d2 < bd[s - 1];
          const bool here = !up && d2 < bd[s];
          bd[s] = up ? bd[s - 1] : (here ? d2 : bd[s]);
          bj[s] = up ? bj[s - 1] : (here ? jj : bj[s]);
        }
        if (d2 < bd[0]) {
          bd[0] = d2;
          bj[0] = jj;
        }
      }
    }
  }
  if (!valid) return;
  const int k = (int)(i < M ? i : M);
  int mine = -1;   // lane s keeps the s-th neighbour
  for (int s = 0; s < k; ++s) {
    double d = bd[0];
    int j = bj[0];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double od = __shfl_xor(d, o, 64);
      const int oj = __shfl_xor(j, o, 64);
      const bool take = od < d || (od == d && oj < j);
      d = take ? od : d;
      j = take ? oj : j;
    }
    if (lane == s) mine = j;
    if (bj[0] == j) {   // the winning lane pops its head (indices are unique across lanes)
#pragma unroll
      for (int t = 0; t < M - 1; ++t) {
        bd[t] = bd[t + 1];
        bj[t] = bj[t + 1];
      }
      bd[M - 1] = HUGE_VAL;
      bj[M - 1] = -1;
    }
  }
  if (lane < M) nbr[i * M + lane] = lane < k ? mine : -1;
  if (lane == 0) kcnt[i] = k;
}

__global__ void fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int M>
hipError_t knn_dispatch(const double* xs, const double* ys, int64_t D, int32_t* nbr, int32_t* kcnt,
                        hipStream_t s) {
  constexpr int64_t kPer = kMaxLaunchThreads / 64;   // queries (one wave each) per launch
  for (int64_t b = 0; b < D; b += kPer) {
    const int64_t n = D - b < kPer ? D - b : kPer;
    const unsigned blocks = (unsigned)((n + kKnnWaves - 1) / kKnnWaves);
    hipLaunchKernelGGL(knn_preceding<M>, dim3(blocks), dim3(64 * kKnnWaves), 0, s, xs, ys, D, nbr, kcnt, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int... Ms>
hipError_t knn_switch(int m, const double* xs, const double* ys, int64_t D, int32_t* nbr,
                      int32_t* kcnt, hipStream_t s, std::integer_sequence<int, Ms...>) {
  hipError_t err = hipErrorInvalidValue;
  ((m == Ms + 1 ? (err = knn_dispatch<Ms + 1>(xs, ys, D, nbr, kcnt, s), 0) : 0), ...);
  return err;
}

}  // namespace

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_knn(const double* xs, const double* ys, int64_t D, int m, int32_t* nbr,
                      int32_t* kcnt, hipStream_t s) {
  if (D <= 0) return hipSuccess;
  if (m == 0) {
    hipLaunchKernelGGL(fill_i32, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, kcnt, D, 0);
    return hipGetLastError();
  }
  if (m < 1 || m > kMaxM) return hipErrorInvalidValue;
  return knn_switch(m, xs, ys, D, nbr, kcnt, s, std::make_integer_sequence<int, kMaxM>{});
}

}  // namespace vecchia
