// Measurement hook: issue rates of the vector ALU on this device, in wave64
// instructions per compute unit per nanosecond, for a full-rate FP32 FMA and for
// the transcendental instructions the FP32 SOV step uses (v_exp_f32, v_log_f32,
// v_rcp_f32, v_sqrt_f32). Each kernel runs 8 independent dependency chains per
// lane (enough to keep the SIMDs issuing) for a fixed number of rounds over a
// grid of many waves per CU; the rate is instructions issued / (CUs x elapsed).
// These rates bound what the SOV loop's instruction mix can reach.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr int kChains = 8;
constexpr int kRounds = 2048;
constexpr int kBlock = 256;

enum Op { OP_FMA = 0, OP_EXP, OP_LOG, OP_RCP, OP_SQRT, OP_COUNT };

template <int OP>
__global__ __launch_bounds__(kBlock) void valu_rate(float* out, int rounds) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = 0.3f + 0.01f * c + 1e-6f * threadIdx.x;
  for (int i = 0; i < rounds; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if (OP == OP_FMA) v[c] = fmaf(v[c], 0.999f, 0.001f);
      if (OP == OP_EXP) v[c] = __builtin_amdgcn_exp2f(-v[c]);           // converges in (0, 1)
      if (OP == OP_LOG) v[c] = __builtin_amdgcn_logf(v[c] + 2.5f);      // one add per log
      if (OP == OP_RCP) v[c] = __builtin_amdgcn_rcpf(v[c]);             // alternates x, 1/x
      if (OP == OP_SQRT) v[c] = __builtin_amdgcn_sqrtf(v[c]);           // tends to 1
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

template <int OP>
hipError_t launch_rate(float* out, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(valu_rate<OP>, dim3(blocks), dim3(kBlock), 0, s, out, kRounds);
  return hipGetLastError();
}

hipError_t launch_op(int op, float* out, unsigned blocks, hipStream_t s) {
  switch (op) {
    case OP_FMA: return launch_rate<OP_FMA>(out, blocks, s);
    case OP_EXP: return launch_rate<OP_EXP>(out, blocks, s);
    case OP_LOG: return launch_rate<OP_LOG>(out, blocks, s);
    case OP_RCP: return launch_rate<OP_RCP>(out, blocks, s);
    default: return launch_rate<OP_SQRT>(out, blocks, s);
  }
}

}  // namespace
}  // namespace vecchia

extern "C" vecchia_status vecchia_calibrate_valu(void* hip_stream, double* rates_out) {
  using namespace vecchia;
  if (!rates_out) return set_error(VECCHIA_E_INVALID, "rates_out must hold 5 values");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || cus <= 0) return hip_error(e, "device query");
  const unsigned blocks = (unsigned)cus * 32u;   // 128 waves per CU: several rounds of full occupancy
  float* out = nullptr;
  e = hipMalloc(&out, sizeof(float) * (size_t)blocks * kBlock);
  if (e != hipSuccess) return hip_error(e, "calibration buffer");
  hipEvent_t a = nullptr, b = nullptr;
  e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  for (int op = 0; op < OP_COUNT && e == hipSuccess; ++op) {
    e = launch_op(op, out, blocks, s);   // warm-up
    float best = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(a, s);
      if (e == hipSuccess) e = launch_op(op, out, blocks, s);
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e == hipSuccess && (best == 0.0f || ms < best)) best = ms;
    }
    if (e == hipSuccess) {
      const double instr = (double)blocks * (kBlock / 64) * kRounds * kChains;
      rates_out[op] = instr / ((double)cus * (double)best * 1e6);
    }
  }
  // the log kernel issues an add beside every log: remove its time (at the FMA
  // kernel's rate) so that rates_out[OP_LOG] is the log instruction's own rate
  if (e == hipSuccess) {
    const double t_log = 1.0 / rates_out[OP_LOG] - 1.0 / rates_out[OP_FMA];
    if (t_log > 0.0) rates_out[OP_LOG] = 1.0 / t_log;
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(out);
  if (e != hipSuccess) return hip_error(e, "calibration");
  return VECCHIA_OK;
}
