// Autotuner for the QMC launch shape: the number of lattice points one work
// item (one wave) evaluates, i.e. 64 x the samples each lane takes in turn.
// Fewer, longer items amortise the per-item set-up (descriptor decode, lattice
// start points, the three wave reductions and the partial-sum store); more,
// shorter items fill the 256 CUs better when a launch has few terms. The best
// trade-off depends on the conditioning-set size K (the chain's register
// footprint and its length), so it is measured per (precision, K).
//
// For each requested K the tuner builds a synthetic instance with the real path
// (uniform points, coordinate ordering, Matern 3/2, m = K, thresholds 1), so
// nearly every term has K neighbours, then times the K launch for each
// candidate with HIP events (median of three after a warm-up run) and keeps the
// fastest. Instances created afterwards with that m use the choice; results
// depend on it only through the FP64 grouping of the partial sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr int kCandidates[] = {256, 512, 1024, 2048, 4096, 8192};

// SplitMix64 stream for the synthetic geometry (the tuner's own inputs).
uint64_t mix(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct DeviceBuffer {
  void* p = nullptr;
  ~DeviceBuffer() {
    if (p) hipFree(p);
  }
};

struct PlanGuard {
  vecchia_plan_t p = nullptr;
  ~PlanGuard() {
    if (p) vecchia_plan_destroy(p);
  }
};

vecchia_status tune_one(int precision, int n_points, int n_shifts, int K, hipStream_t s, int* best_chunk,
                        float* best_ms) {
  // enough terms for two full rounds of waves (256 CUs x 4 SIMDs x 8 waves)
  // even at the largest candidate, so that no candidate is judged on a tail
  const int cap = ((n_points + 63) / 64) * 64;
  const int largest = std::min(cap, kCandidates[sizeof(kCandidates) / sizeof(int) - 1]);
  const int64_t c_min = (n_points + largest - 1) / largest;
  const int64_t T = std::max<int64_t>(64, std::min<int64_t>(1 << 16, (16384 + n_shifts * c_min - 1) /
                                                                      (n_shifts * c_min)));
  const int64_t D = T + K;
  std::vector<double> locs(2 * D);
  uint64_t st = 0x5EEDull + (uint64_t)K;
  for (auto& v : locs) v = (double)(mix(st) >> 11) * 0x1p-53;
  vecchia_cov cov{VECCHIA_COV_MATERN, 0, 1.5, 1.0, 0.1, 1e-8};
  PlanGuard plan;
  vecchia_status r = vecchia_plan(locs.data(), D, 2, VECCHIA_ORDER_COORD, nullptr, K, &cov, s, &plan.p);
  if (r != VECCHIA_OK) return r;
  DeviceBuffer x, out;
  hipError_t e = hipMalloc(&x.p, sizeof(double) * D);
  if (e == hipSuccess) e = hipMalloc(&out.p, sizeof(double) * 2);
  if (e != hipSuccess) return hip_error(e, "autotune buffers");
  const std::vector<double> ones(D, 1.0);
  e = hipMemcpy(x.p, ones.data(), sizeof(double) * D, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "autotune thresholds");
  vecchia_qmc q{n_points, n_shifts, 0x7u, precision, 0};
  const int saved = tuned_chunk(precision, K);
  *best_chunk = 0;
  *best_ms = 0.0f;
  for (int cand : kCandidates) {
    if (cand > cap && cand != kCandidates[0]) break;   // larger chunks all equal the cap
    set_tuned_chunk(precision, K, cand);
    std::unique_ptr<Batch> b;
    std::vector<vecchia_plan_s*> plans{plan.p};
    std::vector<vecchia_qmc> qs{q};
    r = Batch::create(plans, qs, &b);
    if (r == VECCHIA_OK) r = b->run((const double*)x.p, nullptr, nullptr, (double*)out.p, nullptr, nullptr, s);
    float ms = 0.0f;
    if (r == VECCHIA_OK) r = b->time_main_launch(s, 3, &ms);
    if (r == VECCHIA_OK) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) r = hip_error(e, "autotune wait");
    }
    if (r != VECCHIA_OK) {
      set_tuned_chunk(precision, K, saved);
      return r;
    }
    if (*best_chunk == 0 || ms < *best_ms) {
      *best_chunk = std::min(cand, cap);
      *best_ms = ms;
    }
  }
  set_tuned_chunk(precision, K, *best_chunk);
  return VECCHIA_OK;
}

}  // namespace
}  // namespace vecchia

extern "C" {

vecchia_status vecchia_autotune(int32_t precision, int32_t n_points, int32_t n_shifts, const int32_t* ms,
                                int32_t n_ms, void* hip_stream, int32_t* chunk_out, float* ms_out) {
  using namespace vecchia;
  if (precision != VECCHIA_FP64 && precision != VECCHIA_FP32_LOOP)
    return set_error(VECCHIA_E_INVALID, "precision must be VECCHIA_FP64 or VECCHIA_FP32_LOOP");
  vecchia_qmc q{n_points, n_shifts, 0, precision, 0};
  std::string why;
  if (!valid_qmc(q, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (!ms || n_ms < 1 || n_ms > kMaxM) return set_error(VECCHIA_E_INVALID, "ms must list 1..VECCHIA_MAX_M sizes");
  for (int k = 0; k < n_ms; ++k)
    if (ms[k] < 1 || ms[k] > kMaxM) return set_error(VECCHIA_E_INVALID, "each m must be in 1..VECCHIA_MAX_M");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  for (int k = 0; k < n_ms; ++k) {
    int chunk = 0;
    float t = 0.0f;
    const vecchia_status r = tune_one(precision, n_points, n_shifts, ms[k], s, &chunk, &t);
    if (r != VECCHIA_OK) return r;
    if (chunk_out) chunk_out[k] = chunk;
    if (ms_out) ms_out[k] = t;
  }
  return VECCHIA_OK;
}

vecchia_status vecchia_tuning_get(int32_t precision, int32_t m, int32_t* chunk_points) {
  using namespace vecchia;
  if ((precision != VECCHIA_FP64 && precision != VECCHIA_FP32_LOOP) || m < 0 || m > kMaxM || !chunk_points)
    return set_error(VECCHIA_E_INVALID, "tuning_get: bad precision, m or output pointer");
  *chunk_points = tuned_chunk(precision, m);
  return VECCHIA_OK;
}

vecchia_status vecchia_tuning_set(int32_t precision, int32_t m, int32_t chunk_points) {
  using namespace vecchia;
  if ((precision != VECCHIA_FP64 && precision != VECCHIA_FP32_LOOP) || m < 0 || m > kMaxM)
    return set_error(VECCHIA_E_INVALID, "tuning_set: bad precision or m");
  if (chunk_points != 0 && (chunk_points < 64 || chunk_points % 64 != 0 || chunk_points > (1 << 24)))
    return set_error(VECCHIA_E_INVALID, "chunk_points must be 0 (default) or a multiple of 64 in [64, 2^24]");
  set_tuned_chunk(precision, m, chunk_points);
  return VECCHIA_OK;
}

}  // extern "C"
