// Test hooks: the device's own normal CDF / quantile pieces and lattice points,
// evaluated elementwise on caller data, so that tests can pin them directly
// against library routines and the exact integer lattice definition. Nothing
// here is on the evaluation path.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_math_f32.h"
#include "device_math_f64.h"
#include "lattice.h"
#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr int kProbeThreads = 256;

// what (see vecchia_probe_math): out has 3 doubles per input
__global__ __launch_bounds__(kProbeThreads) void probe_math(int what, int64_t n, const double* __restrict__ in,
                                                            double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  if (i >= n) return;
  const double x = in[i];
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  if (what == VECCHIA_PROBE_PHI_F32) {
    // the SOV loop's factor at t = x: v = kappa t in FP32; the smaller tail as
    // the main path forms it, and as the deep path splits it (em * 2^fl)
    const float v = (float)(x * kPhiScale);
    const PhiParts ph = phi_f32(v);
    const float f = fmaxf(ph.f, -1048576.0f);
    const float fl = floorf(f);
    o0 = ph.m;
    o1 = fast_exp2(f - fl) * ph.R;
    o2 = fl;
  } else if (what == VECCHIA_PROBE_NINV_F32) {
    // the SOV loop's quantile of q = x (0 < q <= 1/2, rounded to FP32):
    // z = -Phi^{-1}(q) from log2 q
    const float q = (float)x;
    o0 = ninv_tail_from_log2(fast_log2(q));
    o1 = q;
  } else if (what == VECCHIA_PROBE_NINV_LOG2_F32) {
    // the split path's quantile from log2 q = x directly (its exponents reach -2^20)
    o0 = ninv_tail_from_log2_split((float)x);
  } else if (what == VECCHIA_PROBE_PHI_F64) {
    o0 = phi64(x);
  } else {
    o0 = ninv64(x);
  }
  out[3 * i] = o0;
  out[3 * i + 1] = o1;
  out[3 * i + 2] = o2;
}

__global__ __launch_bounds__(kProbeThreads) void probe_lattice(const uint64_t* __restrict__ Z, uint64_t seed,
                                                               int64_t term, int r, int dim, int second, int64_t n,
                                                               double* __restrict__ w64, float* __restrict__ w32) {
  const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  if (i >= n) return;
  const uint64_t U = (uint64_t)(i + 1) * Z[dim] + lattice_shift(seed, term, r, dim, second != 0);
  if (w64) w64[i] = lattice_coord_f64(U);
  if (w32) w32[i] = lattice_coord_f32((uint32_t)(U >> 32)).w;
}

}  // namespace
}  // namespace vecchia

extern "C" {

vecchia_status vecchia_probe_math(int32_t what, int64_t n, const double* in_dev, double* out_dev,
                                  void* hip_stream) {
  using namespace vecchia;
  if (what < VECCHIA_PROBE_PHI_F32 || what > VECCHIA_PROBE_NINV_F64)
    return set_error(VECCHIA_E_INVALID, "unknown probe");
  if (n < 0 || n > (1LL << 30)) return set_error(VECCHIA_E_INVALID, "n must be in 0..2^30");
  if (n == 0) return VECCHIA_OK;
  if (!in_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  const unsigned blocks = (unsigned)((n + kProbeThreads - 1) / kProbeThreads);
  hipLaunchKernelGGL(probe_math, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(hip_stream), what,
                     n, in_dev, out_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "probe launch");
  return VECCHIA_OK;
}

vecchia_status vecchia_probe_lattice(uint64_t seed, int64_t term, int32_t shift, int32_t dim, int32_t second,
                                     int64_t n, double* w64_dev, float* w32_dev, void* hip_stream) {
  using namespace vecchia;
  if (term < 0 || term >= (1LL << 31) || shift < 0 || shift >= VECCHIA_MAX_SHIFTS || dim < 0 || dim >= kMaxM ||
      (second != 0 && second != 1))
    return set_error(VECCHIA_E_INVALID, "term, shift, dim or second out of range");
  if (n < 0 || n > (1LL << 30)) return set_error(VECCHIA_E_INVALID, "n must be in 0..2^30");
  if (n == 0) return VECCHIA_OK;
  if (!w64_dev && !w32_dev) return set_error(VECCHIA_E_INVALID, "no output");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "device query");
  const uint64_t* Z = device_lattice_table(dev, &e);
  if (!Z) return hip_error(e, "lattice table");
  const unsigned blocks = (unsigned)((n + kProbeThreads - 1) / kProbeThreads);
  hipLaunchKernelGGL(probe_lattice, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(hip_stream), Z,
                     seed, term, shift, dim, second, n, w64_dev, w32_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "probe launch");
  return VECCHIA_OK;
}

}  // extern "C"
