// vecchia_logcdf_noalloc: the single-instance evaluation of vecchia_logcdf
// (Section 2.2, eq. (6)) for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The evaluation's workspace (descriptors, per-term set-up values, partial QMC
// sums, term results, the hand-over lists and their counters) lives in
// `scratch`, a static device array of kScratchBytes per GPU, held until the
// process ends. Its first 512 bytes hold the lattice generators; the batch
// workspace follows at kWsOffset. The host never names the array directly in a
// kernel argument or copy: the array's device address comes from
// hipGetSymbolAddress, once per device on the first call with that device
// current, and every later use goes through that address.
//
// Each call writes what it reads before reading it: the generators and the
// workspace header (by kernels that take them as arguments), then the batch's
// own fills (bad-term and counter words) and every per-term and per-item
// array. Calls that overlap on one GPU share the array and race: order them on
// one stream.
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace vecchia {

constexpr size_t kScratchBytes = VECCHIA_NOALLOC_SCRATCH_BYTES;
constexpr size_t kWsOffset = 4096;   // generators first, then the workspace
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};   // the device address of scratch on each device
uint64_t g_Z[kMaxM];             // the lattice generators (host copy)
bool g_Z_ready = false;

// Payload of one store launch, passed by value (under the kernel-argument limit).
constexpr int kStoreWords = 256;
struct StoreArgs {
  uint64_t w[kStoreWords];
};

__global__ __launch_bounds__(kStoreWords) void store_words(uint64_t* __restrict__ dst, StoreArgs a, int n) {
  const int j = threadIdx.x;
  if (j < n) dst[j] = a.w[j];
}

}  // namespace

hipError_t launch_store_bytes(void* dst, const void* src_host, size_t bytes, hipStream_t s) {
  if ((reinterpret_cast<uintptr_t>(dst) & 7) != 0) return hipErrorInvalidValue;
  const char* src = static_cast<const char*>(src_host);
  uint64_t* d = static_cast<uint64_t*>(dst);
  const size_t words = (bytes + 7) / 8;
  for (size_t w0 = 0; w0 < words; w0 += kStoreWords) {
    StoreArgs a;
    const int n = (int)(words - w0 < (size_t)kStoreWords ? words - w0 : (size_t)kStoreWords);
    std::memset(a.w, 0, sizeof(a.w));
    const size_t b0 = w0 * 8;
    std::memcpy(a.w, src + b0, bytes - b0 < (size_t)n * 8 ? bytes - b0 : (size_t)n * 8);
    hipLaunchKernelGGL(store_words, dim3(1), dim3(kStoreWords), 0, s, d + w0, a, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vecchia

using namespace vecchia;

extern "C" vecchia_status vecchia_logcdf_noalloc(vecchia_plan_t plan, const double* x_dev, double scale,
                                                 const vecchia_cov* cov_override, const vecchia_qmc* q,
                                                 double* out_dev, double* terms_dev, void* hip_stream) {
  if (!plan || !q || !x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::string why;
  if (!valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return set_error(VECCHIA_E_INVALID, "device index beyond the scratch table");
  if (plan->device != dev) return set_error(VECCHIA_E_INVALID, "plan belongs to another device");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
      g_ptr[dev] = static_cast<char*>(p);
    }
    base = g_ptr[dev];
    if (!g_Z_ready) {
      host_lattice_table(g_Z, kMaxM);
      g_Z_ready = true;
    }
  }
  // the host-side layout of the one-instance batch (host memory only)
  std::unique_ptr<Batch> b;
  vecchia_status st = Batch::create({plan}, {*q}, &b);
  if (st != VECCHIA_OK) return st;
  if (b->workspace_bytes() > kScratchBytes - kWsOffset)
    return set_error(VECCHIA_E_INVALID, "evaluation needs " + std::to_string(b->workspace_bytes()) +
                                            " bytes of workspace; the static scratch holds " +
                                            std::to_string(kScratchBytes - kWsOffset));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  e = launch_store_bytes(base, g_Z, sizeof(g_Z), s);
  if (e != hipSuccess) return hip_error(e, "generator store");
  const uint64_t seed = q->seed;
  std::lock_guard<std::mutex> lk(plan->mu);
  return b->run_noalloc(base + kWsOffset, reinterpret_cast<const uint64_t*>(base), x_dev, &scale, cov_override,
                        out_dev, terms_dev, &seed, s);
}
