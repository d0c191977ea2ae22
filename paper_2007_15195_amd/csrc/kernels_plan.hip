// Plan-time kernel: nearest preceding neighbours (Section 2.1, after eq. (4);
// Section 2.2, after eq. (6)): for every plan position i, the k_i = min(m, i)
// positions j < i with the smallest keys (d^2, j), d^2 = dx*dx + dy*dy in FP64
// without fused multiply-add, listed in ascending key order.
//
// With group = p > 1 (joint block terms, Section 3.2) the candidates of query i
// are the positions before its group, j < i - i mod p.
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
                                                                int32_t* __restrict__ kcnt, int64_t q_base,
                                                                int64_t q_end, int group, int m) {
#pragma clang fp contract(off)
  __shared__ double2 tile[kKnnTile];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q0 = q_base + (int64_t)blockIdx.x * kKnnWaves;
  const int64_t i = q0 + wave;
  const bool valid = i < q_end;
  const int64_t lim_i = group > 1 ? i - i % group : i;   // candidates j < lim_i
  const double qx = valid ? xs[i] : 0.0;
  const double qy = valid ? ys[i] : 0.0;
  double bd[M];
  int bj[M];
#pragma unroll
  for (int s = 0; s < M; ++s) {
    bd[s] = HUGE_VAL;
    bj[s] = -1;
  }
  const int64_t last_query = (q0 + kKnnWaves < q_end ? q0 + kKnnWaves : q_end) - 1;
  for (int64_t t0 = 0; t0 < last_query; t0 += kKnnTile) {
    __syncthreads();
    for (int c = threadIdx.x; c < kKnnTile; c += 64 * kKnnWaves) {
      const int64_t j = t0 + c;
      if (j < D) tile[c] = make_double2(xs[j], ys[j]);
    }
    __syncthreads();
    const int64_t lim = (valid ? lim_i : 0) - t0;
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
  const int k = (int)(lim_i < m ? lim_i : m);   // m <= M: the list keeps the M best
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
  if (lane < m) nbr[i * m + lane] = lane < k ? mine : -1;
  if (lane == 0) kcnt[i] = k;
}

__device__ __forceinline__ int grid_cell(double v, double lo, double w, int G) {
  const int c = (int)floor((v - lo) / w);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

__global__ __launch_bounds__(256) void grid_count(const double* __restrict__ xs, const double* __restrict__ ys,
                                                  int64_t D, KnnGrid g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= D) return;
  const int c = grid_cell(xs[i], g.x0, g.wx, g.G) * g.G + grid_cell(ys[i], g.y0, g.wy, g.G);
  g.cell[i] = c;
  atomicAdd(&g.cursor[c], 1);   // counts (the cursor array starts at zero)
}

// Exclusive scan of the G*G counts (in cursor) into start[0..G*G]; cursor then
// holds each cell's first slot. One block of 1024 threads, each a contiguous
// segment.
__global__ __launch_bounds__(1024) void grid_scan(KnnGrid g) {
  __shared__ int64_t part[1024];
  const int64_t n = (int64_t)g.G * g.G;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = (int64_t)threadIdx.x * per;
  const int64_t e = b + per < n ? b + per : n;
  int64_t sum = 0;
  for (int64_t c = b; c < e; ++c) sum += g.cursor[c];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan of the partial sums
    const int64_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - sum;   // exclusive prefix of this segment
  for (int64_t c = b; c < e; ++c) {
    const int32_t cnt = g.cursor[c];
    g.start[c] = (int32_t)run;
    g.cursor[c] = (int32_t)run;
    run += cnt;
  }
  if (threadIdx.x == 1023) g.start[n] = (int32_t)part[1023];
}

__global__ __launch_bounds__(256) void grid_scatter(const double* __restrict__ xs, const double* __restrict__ ys,
                                                    int64_t D, KnnGrid g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= D) return;
  const int q = atomicAdd(&g.cursor[g.cell[i]], 1);
  g.gx[q] = xs[i];
  g.gy[q] = ys[i];
  g.gid[q] = (int32_t)i;
}

template <int M>
__global__ __launch_bounds__(256) void knn_grid(const double* __restrict__ xs, const double* __restrict__ ys,
                                                int64_t D, KnnGrid g, int32_t* __restrict__ nbr,
                                                int32_t* __restrict__ kcnt, int64_t q_base, int m) {
#pragma clang fp contract(off)
  const int64_t i = q_base + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= D) return;
  const int k = (int)(i < m ? i : m);   // m <= M: the list keeps the M best
  kcnt[i] = k;
  if (k == 0) {
    for (int s = 0; s < m; ++s) nbr[i * m + s] = -1;
    return;
  }
  const double qx = xs[i], qy = ys[i];
  const int cx = grid_cell(qx, g.x0, g.wx, g.G), cy = grid_cell(qy, g.y0, g.wy, g.G);
  double bd[M];
  int bj[M];
#pragma unroll
  for (int s = 0; s < M; ++s) {
    bd[s] = HUGE_VAL;
    bj[s] = 0x7fffffff;
  }
  const int G = g.G;
  for (int r = 0;; ++r) {
    const int xl = cx - r, xh = cx + r, yl = cy - r, yh = cy + r;
    for (int x = (xl < 0 ? 0 : xl); x <= (xh > G - 1 ? G - 1 : xh); ++x) {
      // the ring's cells in column x: all of [yl, yh] on the edge columns, else
      // its two ends
      const bool edge_col = x == xl || x == xh;
      const int y0 = edge_col ? (yl < 0 ? 0 : yl) : yl;
      const int y1 = edge_col ? (yh > G - 1 ? G - 1 : yh) : yh;
      const int dy_step = edge_col ? 1 : (yh > yl ? yh - yl : 1);
      for (int y = y0; y <= y1; y += dy_step) {
        if (y < 0 || y > G - 1) continue;
        const int c = x * G + y;
        const int q1 = g.start[c + 1];
        for (int q = g.start[c]; q < q1; ++q) {
          const int j = g.gid[q];
          if (j >= i) continue;
          const double dx = g.gx[q] - qx;
          const double dy = g.gy[q] - qy;
          const double d2 = dx * dx + dy * dy;
          if (d2 < bd[M - 1] || (d2 == bd[M - 1] && j < bj[M - 1])) {
#pragma unroll
            for (int s = M - 1; s > 0; --s) {
              const bool up = d2 < bd[s - 1] || (d2 == bd[s - 1] && j < bj[s - 1]);
              const bool here = !up && (d2 < bd[s] || (d2 == bd[s] && j < bj[s]));
              bd[s] = up ? bd[s - 1] : (here ? d2 : bd[s]);
              bj[s] = up ? bj[s - 1] : (here ? j : bj[s]);
            }
            if (d2 < bd[0] || (d2 == bd[0] && j < bj[0])) {
              bd[0] = d2;
              bj[0] = j;
            }
          }
        }
      }
    }
    if (xl <= 0 && yl <= 0 && xh >= G - 1 && yh >= G - 1) break;   // every cell visited
    // k-th smallest key so far (selected with static indices: a dynamic index
    // would move the list out of registers)
    double kth = bd[0];
#pragma unroll
    for (int s = 1; s < M; ++s) kth = s == k - 1 ? bd[s] : kth;
    if (kth < HUGE_VAL) {
      // every unvisited point is at least `edge` away from the query
      double edge = HUGE_VAL;
      if (xl > 0) edge = fmin(edge, qx - (g.x0 + xl * g.wx));
      if (xh < G - 1) edge = fmin(edge, (g.x0 + (xh + 1) * g.wx) - qx);
      if (yl > 0) edge = fmin(edge, qy - (g.y0 + yl * g.wy));
      if (yh < G - 1) edge = fmin(edge, (g.y0 + (yh + 1) * g.wy) - qy);
      edge -= g.margin;
      if (edge > 0.0 && kth < edge * edge) break;
    }
  }
#pragma unroll
  for (int s = 0; s < M; ++s)
    if (s < m) nbr[i * m + s] = s < k ? bj[s] : -1;
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
                        const KnnGrid* grid, int group, int m, hipStream_t s) {
  // queries below q_split scan their i preceding points with a wave each; the
  // rest (large plans only) search the grid, where preceding points are dense
  const int64_t q_split = grid ? (D < kKnnGridMinD ? D : kKnnGridMinD) : D;
  if (grid) {
    constexpr int64_t kPer = kMaxLaunchThreads;   // queries (one thread each) per launch
    for (int64_t b = q_split; b < D; b += kPer) {
      const int64_t n = D - b < kPer ? D - b : kPer;
      hipLaunchKernelGGL(knn_grid<M>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xs, ys, D, *grid, nbr,
                         kcnt, b, m);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  constexpr int64_t kPerWave = kMaxLaunchThreads / 64;   // queries (one wave each) per launch
  for (int64_t b = 0; b < q_split; b += kPerWave) {
    const int64_t n = q_split - b < kPerWave ? q_split - b : kPerWave;
    const unsigned blocks = (unsigned)((n + kKnnWaves - 1) / kKnnWaves);
    hipLaunchKernelGGL(knn_preceding<M>, dim3(blocks), dim3(64 * kKnnWaves), 0, s, xs, ys, D, nbr, kcnt, b,
                       q_split, group, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int... Ms>
hipError_t knn_switch(int m, const double* xs, const double* ys, int64_t D, int32_t* nbr,
                      int32_t* kcnt, const KnnGrid* grid, int group, hipStream_t s,
                      std::integer_sequence<int, Ms...>) {
  hipError_t err = hipErrorInvalidValue;
  ((m == Ms + 1 ? (err = knn_dispatch<Ms + 1>(xs, ys, D, nbr, kcnt, grid, group, m, s), 0) : 0), ...);
  return err;
}

hipError_t build_grid(const double* xs, const double* ys, int64_t D, const KnnGrid& g, hipStream_t s) {
  const int64_t cells = (int64_t)g.G * g.G;
  hipLaunchKernelGGL(fill_i32, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, g.cursor, cells, 0);
  hipError_t e = hipGetLastError();
  const unsigned blocks = (unsigned)((D + 255) / 256);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(grid_count, dim3(blocks), dim3(256), 0, s, xs, ys, D, g);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(grid_scan, dim3(1), dim3(1024), 0, s, g);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(grid_scatter, dim3(blocks), dim3(256), 0, s, xs, ys, D, g);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_knn(const double* xs, const double* ys, int64_t D, int m, int32_t* nbr,
                      int32_t* kcnt, const KnnGrid* grid, hipStream_t s, int group) {
  if (D <= 0) return hipSuccess;
  if (group < 1 || (group > 1 && grid)) return hipErrorInvalidValue;   // the grid search has no group limit
  if (m == 0) {
    hipLaunchKernelGGL(fill_i32, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, kcnt, D, 0);
    return hipGetLastError();
  }
  if (m < 1 || m > kMaxM) return hipErrorInvalidValue;
  if (grid) {
    if (D > 0x7fffffffLL || (int64_t)grid->G * grid->G + 1 > 0x7fffffffLL) return hipErrorInvalidValue;
    const hipError_t e = build_grid(xs, ys, D, *grid, s);
    if (e != hipSuccess) return e;
  }
  if (m <= kMaxUnrolledK)
    return knn_switch(m, xs, ys, D, nbr, kcnt, grid, group, s, std::make_integer_sequence<int, kMaxUnrolledK>{});
  // larger sets: lists of capacity 40, 48, 56 or 64 holding the m wanted
  if (m <= 40) return knn_dispatch<40>(xs, ys, D, nbr, kcnt, grid, group, m, s);
  if (m <= 48) return knn_dispatch<48>(xs, ys, D, nbr, kcnt, grid, group, m, s);
  if (m <= 56) return knn_dispatch<56>(xs, ys, D, nbr, kcnt, grid, group, m, s);
  return knn_dispatch<64>(xs, ys, D, nbr, kcnt, grid, group, m, s);
}

}  // namespace vecchia
