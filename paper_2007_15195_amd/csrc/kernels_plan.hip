// Plan-time kernel: nearest preceding neighbours (Section 2.1, after eq. (4);
// Section 2.2, after eq. (6)): for every plan position i, the k_i = min(m, i)
// positions j < i with the smallest keys (d^2, j), d^2 = dx*dx + dy*dy in FP64
// without fused multiply-add, listed in ascending key order.
//
// One thread per query; a 128-query block stages candidate coordinates through
// LDS in increasing j, so a candidate tied in d^2 with a kept one never displaces
// it (ties resolve to the lower index). The sorted top-M list lives in registers
// (M is a template parameter, so the insertion network has static indices).
#include "vecchia_internal.h"

namespace vecchia {
namespace {

constexpr int kKnnTile = 128;

template <int M>
__global__ __launch_bounds__(kKnnTile) void knn_preceding(const double* __restrict__ xs,
                                                          const double* __restrict__ ys, int64_t D,
                                                          int32_t* __restrict__ nbr,
                                                          int32_t* __restrict__ kcnt) {
#pragma clang fp contract(off)
  __shared__ double2 tile[kKnnTile];
  const int64_t q0 = (int64_t)blockIdx.x * kKnnTile;
  const int64_t i = q0 + threadIdx.x;
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
  const int64_t last_query = (q0 + kKnnTile < D ? q0 + kKnnTile : D) - 1;
  for (int64_t t0 = 0; t0 < last_query; t0 += kKnnTile) {
    __syncthreads();
    const int64_t j = t0 + threadIdx.x;
    if (j < D) tile[threadIdx.x] = make_double2(xs[j], ys[j]);
    __syncthreads();
    int64_t lim = (valid ? i : 0) - t0;
    const int cmax = (int)(lim < kKnnTile ? (lim > 0 ? lim : 0) : kKnnTile);
    for (int c = 0; c < cmax; ++c) {
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
#pragma unroll
  for (int s = 0; s < M; ++s) nbr[i * M + s] = s < k ? bj[s] : -1;
  kcnt[i] = k;
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
  const unsigned blocks = (unsigned)((D + kKnnTile - 1) / kKnnTile);
  hipLaunchKernelGGL(knn_preceding<M>, dim3(blocks), dim3(kKnnTile), 0, s, xs, ys, D, nbr, kcnt);
  return hipGetLastError();
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
