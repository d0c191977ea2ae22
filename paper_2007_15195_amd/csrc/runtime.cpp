// Host runtime: error state, lattice table, and the Batch engine that lays out
// and enqueues one evaluation (setup -> QMC per conditioning-set size, largest
// first -> segmented sum), optionally replayed from a captured HIP graph.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>

namespace vecchia {

namespace {
thread_local std::string g_err;
std::mutex g_dev_mu;
std::map<int, uint64_t*> g_Z;

// floor(frac(sqrt(p)) * 2^64) for a non-square p < 2^32, by bisection on the
// exact condition (f 2^64 + Z)^2 <= p 2^128 with f = floor(sqrt(p)), i.e.
// Z^2 + 2 f Z 2^64 <= (p - f^2) 2^128, evaluated in three 64-bit limbs.
uint64_t frac_sqrt_fixed(uint64_t p) {
  uint64_t f = (uint64_t)std::sqrt((double)p);
  while (f * f > p) --f;
  while ((f + 1) * (f + 1) <= p) ++f;
  const uint64_t c = p - f * f;
  auto fits = [&](uint64_t Z) {
    const unsigned __int128 zz = (unsigned __int128)Z * Z;
    const unsigned __int128 fz = (unsigned __int128)(2 * f) * Z;   // < 2^70
    const uint64_t l1a = (uint64_t)(zz >> 64);
    const uint64_t l1b = (uint64_t)fz;
    const uint64_t l1 = l1a + l1b;
    const uint64_t carry = l1 < l1a;
    const unsigned __int128 l2 = (unsigned __int128)(uint64_t)(fz >> 64) + carry;
    (void)l1;
    return l2 < c || (l2 == c && l1 == 0 && (uint64_t)zz == 0);
  };
  uint64_t Z = 0;
  for (int b = 63; b >= 0; --b) {
    const uint64_t cand = Z | (1ULL << b);
    if (fits(cand)) Z = cand;
  }
  return Z;
}
}  // namespace

namespace {
std::map<int, std::pair<uint64_t*, int>> g_Zn;   // device -> (table, length)
}  // namespace

const uint64_t* device_lattice_table_n(int device, int n, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_Zn.find(device);
  if (it != g_Zn.end() && it->second.second >= n) {
    *err = hipSuccess;
    return it->second.first;
  }
  const int len = std::max(n, it != g_Zn.end() ? 2 * it->second.second : 64);
  std::vector<uint64_t> primes;
  primes.reserve(len);
  for (uint64_t c = 2; (int)primes.size() < len; ++c) {
    bool prime = true;
    for (uint64_t q : primes) {
      if (q * q > c) break;
      if (c % q == 0) {
        prime = false;
        break;
      }
    }
    if (prime) primes.push_back(c);
  }
  std::vector<uint64_t> Z(len);
  for (int j = 0; j < len; ++j) Z[j] = frac_sqrt_fixed(primes[j]);
  uint64_t* d = nullptr;
  *err = hipMalloc(&d, sizeof(uint64_t) * len);
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(d, Z.data(), sizeof(uint64_t) * len, hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    hipFree(d);
    return nullptr;
  }
  // an older, shorter table is kept (a call in flight may still read it)
  g_Zn[device] = {d, len};
  return d;
}

namespace {
struct ProfRec {
  int K, precision;
  hipEvent_t a, b;
  int64_t steps;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
}  // namespace

std::vector<hipEvent_t> g_prof_pool;   // events returned by reset, reused

hipError_t profile_events(hipEvent_t* a, hipEvent_t* b) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof_pool.size() >= 2) {
      *a = g_prof_pool.back();
      g_prof_pool.pop_back();
      *b = g_prof_pool.back();
      g_prof_pool.pop_back();
      return hipSuccess;
    }
  }
  hipError_t e = hipEventCreate(a);
  if (e == hipSuccess) e = hipEventCreate(b);
  return e;
}

bool profiling_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

void profile_record(int K, int precision, hipEvent_t a, hipEvent_t b, int64_t steps) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(ProfRec{K, precision, a, b, steps});
}

vecchia_status set_error(vecchia_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

vecchia_status hip_error(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? VECCHIA_E_NOMEM : VECCHIA_E_HIP,
                   std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error_message() { return g_err.c_str(); }

void host_lattice_table(uint64_t* Z, int n) {
  int found = 0;
  for (uint64_t c = 2; found < n; ++c) {
    bool prime = true;
    for (uint64_t d = 2; d * d <= c; ++d)
      if (c % d == 0) { prime = false; break; }
    if (prime) Z[found++] = frac_sqrt_fixed(c);
  }
}

const uint64_t* device_lattice_table(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_Z.find(device);
  if (it != g_Z.end()) {
    *err = hipSuccess;
    return it->second;
  }
  uint64_t Z[kMaxM];
  host_lattice_table(Z, kMaxM);
  uint64_t* d = nullptr;
  *err = hipMalloc(&d, sizeof(Z));
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(d, Z, sizeof(Z), hipMemcpyHostToDevice);
  if (*err != hipSuccess) return nullptr;
  g_Z[device] = d;
  return d;
}

bool valid_cov(const vecchia_cov& c, std::string* why) {
  if (c.family != VECCHIA_COV_EXPONENTIAL && c.family != VECCHIA_COV_MATERN) {
    *why = "unknown covariance family";
    return false;
  }
  if (c.family == VECCHIA_COV_MATERN && !(c.nu == 0.5 || c.nu == 1.5 || c.nu == 2.5)) {
    *why = "Matern nu must be 0.5, 1.5 or 2.5";
    return false;
  }
  if (!(std::isfinite(c.sigma2) && c.sigma2 > 0)) { *why = "sigma2 must be finite and > 0"; return false; }
  if (!(std::isfinite(c.range) && c.range > 0)) { *why = "range must be finite and > 0"; return false; }
  if (!(std::isfinite(c.nugget) && c.nugget >= 0)) { *why = "nugget must be finite and >= 0"; return false; }
  return true;
}

bool valid_qmc(const vecchia_qmc& q, std::string* why) {
  if (q.n_points < 1 || q.n_points > VECCHIA_MAX_POINTS) { *why = "n_points out of range"; return false; }
  if (q.n_shifts < 1 || q.n_shifts > VECCHIA_MAX_SHIFTS) { *why = "n_shifts out of range"; return false; }
  if (q.precision != VECCHIA_FP64 && q.precision != VECCHIA_FP32_LOOP) {
    *why = "precision must be VECCHIA_FP64 or VECCHIA_FP32_LOOP";
    return false;
  }
  if (q.flags != 0 && q.flags != VECCHIA_QMC_INDEPENDENT) {
    *why = "flags must be 0 or VECCHIA_QMC_INDEPENDENT";
    return false;
  }
  return true;
}

// Lattice points per QMC work item (a multiple of 64): small enough that a
// launch has many more items than the GPU has wave slots (so the last round of
// items is short), large enough to amortise each item's set-up. Results depend
// on it only through the FP64 summation grouping; it is a function of the
// instance alone, so an instance evaluates identically alone or in any batch.
namespace {
std::atomic<int> g_chunk[2][kMaxM + 1];   // [precision][m]; 0 = untuned
}  // namespace

int tuned_chunk(int precision, int m) {
  if ((precision != VECCHIA_FP64 && precision != VECCHIA_FP32_LOOP) || m < 0 || m > kMaxM) return 0;
  return g_chunk[precision][m].load(std::memory_order_relaxed);
}

void set_tuned_chunk(int precision, int m, int chunk_points) {
  g_chunk[precision][m].store(chunk_points, std::memory_order_relaxed);
}

int chunk_points_for(int m, int precision, int n_points) {
  int base = tuned_chunk(precision, m);
  if (base <= 0) base = precision == VECCHIA_FP32_LOOP ? 2048 : 512;
  const int cap = ((n_points + 63) / 64) * 64;
  return std::max(64, std::min(base, cap));
}

// ------------------------------------------------------------------ Batch ---

Batch::~Batch() {
  if (graph_exec_) hipGraphExecDestroy(graph_exec_);
  for (int k = 0; k < kSideStreams; ++k) {
    if (side_[k] && own_side_) {
      hipStreamSynchronize(side_[k]);
      hipStreamDestroy(side_[k]);
    }
    if (join_ev_[k]) hipEventDestroy(join_ev_[k]);
  }
  if (fork_ev_) hipEventDestroy(fork_ev_);
  for (auto& e : stage_ev_)
    if (e) hipEventDestroy(e);
  if (done_ev_) hipEventDestroy(done_ev_);
  if (h_stage_) hipHostFree(h_stage_);
  if (d_ws_) hipFree(d_ws_);
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

vecchia_status Batch::create(const std::vector<vecchia_plan_s*>& plans,
                             const std::vector<vecchia_qmc>& qmcs, std::unique_ptr<Batch>* out) {
  if (plans.empty() || plans.size() != qmcs.size())
    return set_error(VECCHIA_E_INVALID, "batch needs n >= 1 plans and as many qmc settings");
  if (plans.size() > 0x7fffffff) return set_error(VECCHIA_E_INVALID, "too many instances");
  std::unique_ptr<Batch> b(new Batch());
  b->plans_ = plans;
  b->qmcs_ = qmcs;
  int dev = 0;
  hipGetDevice(&dev);
  b->device_ = dev;
  const int n = (int)plans.size();
  b->term_bases_.resize(n + 1);
  b->desc_.resize(n);
  b->prep_off_.resize(n);
  int64_t tb = 0, sb = 0;
  size_t prep = 0;
  std::map<std::tuple<int, int, bool>, std::vector<RangeDesc>> by_k;   // (K, precision, block) -> ranges
  for (int j = 0; j < n; ++j) {
    vecchia_plan_s* P = plans[j];
    std::string why;
    if (!P) return set_error(VECCHIA_E_INVALID, "null plan in batch");
    if (P->device != dev) return set_error(VECCHIA_E_INVALID, "plan belongs to another device");
    if (!valid_qmc(qmcs[j], &why)) return set_error(VECCHIA_E_INVALID, "instance " + std::to_string(j) + ": " + why);
    const int R = qmcs[j].n_shifts;
    const int passes = qmcs[j].flags == VECCHIA_QMC_INDEPENDENT ? 2 : 1;   // a second lattice for the denominators
    const int prec = qmcs[j].precision;
    const int nv = P->block > 0 ? P->block_nv : P->m + 1;   // variables per term, at most
    b->max_vars_ = std::max(b->max_vars_, nv);
    // FP32 rows leave room for the FP64 rows of a term handed to the FP64 kernels
    const int stride = prec == VECCHIA_FP32_LOOP ? 2 * (int)align_up((size_t)nv * (nv + 1) / 2, 2)
                                                 : (int)align_up((size_t)nv * (nv + 1) / 2, 2);
    InstDesc& d = b->desc_[j];
    std::memset(&d, 0, sizeof(d));
    d.xs = P->d_xs;
    d.ys = P->d_ys;
    d.covmat = P->d_cov;
    d.perm = P->d_perm;
    d.nbr = P->d_nbr;
    d.kcnt = P->d_kcnt;
    d.sovk = (P->n_obs > 0 || P->block > 0) ? P->d_sovk : P->d_kcnt;   // as sov_dims()
    d.n_obs = P->n_obs;
    d.D = P->D;
    d.n_terms = P->terms();
    d.bvar_off = P->block > 0 ? P->d_bvar_off : nullptr;
    d.bvars = P->block > 0 ? P->d_bvars : nullptr;
    d.split = P->block > 0 ? P->d_split : nullptr;
    d.term_base = tb;
    d.sums_base = sb;
    d.m = P->m;
    d.n_points = qmcs[j].n_points;
    d.n_shifts = R;
    d.passes = passes;
    d.seed = qmcs[j].seed;
    d.prep_stride = stride;
    d.precision = prec;
    d.chunk_points = chunk_points_for(P->m, prec, qmcs[j].n_points);
    d.n_chunks = (qmcs[j].n_points + d.chunk_points - 1) / d.chunk_points;
    const int C = d.n_chunks;
    b->term_bases_[j] = tb;
    b->prep_off_[j] = prep;
    const int64_t NT = P->terms();
    prep += align_up((size_t)NT * stride * (prec == VECCHIA_FP32_LOOP ? 4 : 8), 256);
    if (prec == VECCHIA_FP32_LOOP) b->any_f32_ = true;
    // runs of equal k >= 1 become ranges of the launch for that k
    const std::vector<int32_t>& sk = P->sov_dims();
    int64_t i = 0;
    while (i < NT) {
      const int k = sk[i];
      int64_t e = i + 1;
      while (e < NT && sk[e] == k) ++e;
      if (k >= 1) {
        RangeDesc r;
        r.item_begin = e - i;   // term count; turned into the item prefix below
        r.term_begin = i;
        r.inst = j;
        r.K = k;
        r.items_per_term = passes * R * C;
        r.n_chunks = C;
        by_k[{k, prec, P->block > 0}].push_back(r);
      }
      i = e;
    }
    if ((int64_t)passes * R * C > 0x7fffffffLL / std::max<int64_t>(1, NT))
      return set_error(VECCHIA_E_INVALID, "instance " + std::to_string(j) + " has more than 2^31 work items");
    tb += NT;
    sb += NT * (int64_t)passes * R * C;
  }
  b->term_bases_[n] = tb;
  b->total_terms_ = tb;
  b->total_sums_ = sb;
  b->prep_bytes_ = prep;
  if (tb > 0x7fffffffLL) return set_error(VECCHIA_E_INVALID, "more than 2^31-1 terms in one batch");
  // one launch per (K, precision); the launch with the most work runs on the
  // caller's stream, the others (mostly the few terms with k < m) run beside it
  for (auto it = by_k.begin(); it != by_k.end(); ++it) {
    Launch L;
    L.K = std::get<0>(it->first);
    L.precision = std::get<1>(it->first);
    L.block = std::get<2>(it->first);
    L.range_off = (int)b->ranges_.size();
    L.n_ranges = (int)it->second.size();
    int64_t items = 0;
    L.sov_steps = 0;
    for (RangeDesc r : it->second) {
      const int64_t nterms = r.item_begin;
      r.item_begin = items;
      items += nterms * r.items_per_term;
      L.sov_steps += nterms * (int64_t)b->desc_[r.inst].passes * b->desc_[r.inst].n_shifts *
                     b->desc_[r.inst].n_points * r.K;
      b->ranges_.push_back(r);
    }
    L.n_items = items;
    if (items > 0x7fffffffLL) return set_error(VECCHIA_E_INVALID, "more than 2^31-1 work items in one launch");
    b->launches_.push_back(L);
  }
  std::stable_sort(b->launches_.begin(), b->launches_.end(),
                   [](const Launch& a, const Launch& c) { return a.sov_steps * (a.precision == VECCHIA_FP64 ? 8 : 1) >
                                                                 c.sov_steps * (c.precision == VECCHIA_FP64 ? 8 : 1); });
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  take(sizeof(InstDesc) * n);
  take(sizeof(int64_t) * (n + 1));
  take(sizeof(RangeDesc) * std::max<size_t>(1, b->ranges_.size()));
  take(sizeof(Aux64) * tb);
  if (b->any_f32_) take(sizeof(Aux32) * tb);
  take(sizeof(double) * 3 * sb);
  take(sizeof(double2) * tb);
  take(sizeof(int64_t) * n);
  take(prep);
  if (b->any_f32_) {
    // terms handed to FP64 (FP32 instances): flags, two lists with room for
    // every term, and their counters
    b->plist_cap_ = (int32_t)tb;
    take(sizeof(int32_t) * tb);
    take(sizeof(int32_t) * 2 * (size_t)tb);
    take(sizeof(int64_t) * 4);
  }
  b->ws_bytes_ = off;
  *out = std::move(b);
  return VECCHIA_OK;
}

void Batch::carve(char* base) {
  const int n = (int)plans_.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off = align_up(off + bytes, 256);
    return p;
  };
  d_desc_ = reinterpret_cast<InstDesc*>(take(sizeof(InstDesc) * n));
  d_term_bases_ = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (n + 1)));
  d_ranges_ = reinterpret_cast<RangeDesc*>(take(sizeof(RangeDesc) * std::max<size_t>(1, ranges_.size())));
  d_aux64_ = reinterpret_cast<Aux64*>(take(sizeof(Aux64) * total_terms_));
  if (any_f32_) d_aux32_ = reinterpret_cast<Aux32*>(take(sizeof(Aux32) * total_terms_));
  d_sums_ = reinterpret_cast<double*>(take(sizeof(double) * 3 * total_sums_));
  d_term_res_ = reinterpret_cast<double2*>(take(sizeof(double2) * total_terms_));
  d_bad_ = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * n));
  d_prep_ = take(prep_bytes_);
  if (any_f32_) {
    d_promote_ = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * total_terms_));
    d_plist_ = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2 * (size_t)total_terms_));
    d_pctr_ = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 4));
  }
  ipt_max_ = 0;
  for (int j = 0; j < n; ++j) {
    desc_[j].prep = d_prep_ + prep_off_[j];
    desc_[j].bad_term = d_bad_ + j;
    const bool f32 = desc_[j].precision == VECCHIA_FP32_LOOP;
    desc_[j].promote = f32 ? d_promote_ : nullptr;
    desc_[j].plist = f32 ? d_plist_ : nullptr;
    desc_[j].pctr = f32 ? d_pctr_ : nullptr;
    desc_[j].plist_cap = plist_cap_;
    if (f32) ipt_max_ = std::max(ipt_max_, desc_[j].passes * desc_[j].n_shifts * desc_[j].n_chunks);
  }
}

vecchia_status Batch::allocate() {
  if (d_ws_ || d_desc_) return VECCHIA_OK;
  hipError_t e;
  d_Z_ = device_lattice_table(device_, &e);
  if (!d_Z_) return hip_error(e, "lattice table");
  char* base = ext_ws_;
  if (!base) {
    e = hipMalloc(&d_ws_, ws_bytes_);
    if (e != hipSuccess) {
      d_ws_ = nullptr;
      return hip_error(e, "workspace allocation");
    }
    base = d_ws_;
  }
  const int n = (int)plans_.size();
  carve(base);
  if (!ext_stage_) {
    e = hipHostMalloc(reinterpret_cast<void**>(&h_stage_), sizeof(InstDesc) * n * kRing, hipHostMallocDefault);
    if (e != hipSuccess) {
      h_stage_ = nullptr;
      return hip_error(e, "pinned staging");
    }
    for (auto& ev : stage_ev_) {
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_error(e, "event");
    }
  }
  e = hipEventCreateWithFlags(&done_ev_, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork_ev_, hipEventDisableTiming);
  // batches on caller-provided resources use the caller's side streams, if
  // any, and otherwise keep every launch on the caller's stream
  own_side_ = !ext_stage_;
  for (int k = 0; k < kSideStreams && e == hipSuccess && (own_side_ || ext_side_[0]); ++k) {
    if (own_side_)
      e = hipStreamCreateWithFlags(&side_[k], hipStreamNonBlocking);
    else
      side_[k] = ext_side_[k] ? ext_side_[k] : ext_side_[0];
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join_ev_[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_error(e, "streams and events");
  return VECCHIA_OK;
}

vecchia_status Batch::enqueue(hipStream_t s, bool allow_profile) {
  const int n = (int)plans_.size();
  const bool prof = allow_profile && profiling_enabled();
  hipError_t e = launch_fill_i64(d_bad_, n, INT64_MAX, s);
  if (e == hipSuccess && any_f32_) e = launch_fill_i64(d_pctr_, 4, 0, s);
  if (e == hipSuccess)
    e = launch_setup(d_desc_, n, d_term_bases_, total_terms_, max_vars_, d_aux64_, d_aux32_, s);
  // fork: side streams start after the setup kernel
  const int n_side = side_[0] ? std::min<int>((int)launches_.size() - 1, kSideStreams) : 0;
  if (e == hipSuccess && n_side > 0) {
    e = hipEventRecord(fork_ev_, s);
    for (int k = 0; k < n_side && e == hipSuccess; ++k) e = hipStreamWaitEvent(side_[k], fork_ev_, 0);
  }
  for (size_t li = 0; li < launches_.size() && e == hipSuccess; ++li) {
    const Launch& L = launches_[li];
    hipStream_t ls = (li == 0 || n_side == 0) ? s : side_[(li - 1) % n_side];
    hipEvent_t a = nullptr, b = nullptr;
    if (prof) {
      e = profile_events(&a, &b);
      if (e == hipSuccess) e = hipEventRecord(a, ls);
      if (e != hipSuccess) break;
    }
    e = launch_qmc(L.K, L.precision, L.block, d_desc_, d_ranges_ + L.range_off, L.n_ranges, L.n_items,
                   d_aux64_, d_aux32_, d_Z_, d_sums_, ls);
    if (prof && e == hipSuccess) {
      e = hipEventRecord(b, ls);
      profile_record(L.K, L.precision, a, b, L.sov_steps);
    }
  }
  // join
  for (int k = 0; k < n_side && e == hipSuccess; ++k) {
    e = hipEventRecord(join_ev_[k], side_[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join_ev_[k], 0);
  }
  // FP32 instances: the terms promoted at set-up, in FP64 (a short persistent
  // grid that finds nothing to do when no term was promoted)
  const bool redo = any_f32_ && ipt_max_ > 0;
  if (e == hipSuccess && redo)
    e = launch_qmc_promoted(d_desc_, n, d_term_bases_, d_aux64_, d_Z_, d_sums_, d_plist_, d_pctr_, plist_cap_,
                            ipt_max_, s);
  if (e == hipSuccess)
    e = launch_finalize_terms(d_desc_, n, d_term_bases_, total_terms_, d_aux64_, d_sums_, d_term_res_, redo, s);
  // then the terms whose FP32 estimate the finalize found heavy-tailed: FP64
  // rows, FP64 items and their finalize (three grids that exit at once when
  // the list is empty)
  if (e == hipSuccess && redo)
    e = launch_setup_redo(d_desc_, n, d_term_bases_, max_vars_, d_aux64_, d_aux32_, d_plist_ + plist_cap_, d_pctr_ + 2,
                          plist_cap_, s);
  if (e == hipSuccess && redo)
    e = launch_qmc_promoted(d_desc_, n, d_term_bases_, d_aux64_, d_Z_, d_sums_, d_plist_ + plist_cap_, d_pctr_ + 2,
                            plist_cap_, ipt_max_, s);
  if (e == hipSuccess && redo)
    e = launch_finalize_redo(d_desc_, n, d_term_bases_, d_aux64_, d_sums_, d_term_res_, d_plist_ + plist_cap_,
                             d_pctr_ + 2, plist_cap_, s);
  if (e == hipSuccess) e = launch_logsum(d_desc_, n, d_term_res_, s);
  if (e != hipSuccess) return hip_error(e, "kernel launch");
  return VECCHIA_OK;
}

vecchia_status Batch::fill_desc(const double* x_dev, const double* scales, const vecchia_cov* covs,
                                double* out_dev, double* terms_dev, const uint64_t* seeds,
                                std::vector<InstDesc>* out) const {
  const int n = (int)plans_.size();
  int64_t xo = 0;
  std::vector<InstDesc>& d = *out;
  d = desc_;
  for (int j = 0; j < n; ++j) {
    vecchia_plan_s* P = plans_[j];
    const vecchia_cov c = covs ? covs[j] : P->cov;
    std::string why;
    if (covs) {
      if (!valid_cov(c, &why)) return set_error(VECCHIA_E_INVALID, "instance " + std::to_string(j) + ": " + why);
      if (!P->matrix && (c.family != P->cov.family || (c.family == VECCHIA_COV_MATERN && c.nu != P->cov.nu)))
        return set_error(VECCHIA_E_INVALID, "covariance override must keep the plan's family and nu");
    }
    const double sc = scales ? scales[j] : 1.0;
    if (!(std::isfinite(sc) && sc > 0)) return set_error(VECCHIA_E_INVALID, "scale must be finite and > 0");
    d[j].x = !x_ptrs_.empty() ? x_ptrs_[j] : !x_off_.empty() ? x_dev + x_off_[j] : shared_x_ ? x_dev : x_dev + xo;
    d[j].out = out_dev + 2 * j;
    d[j].terms_out = terms_dev;
    d[j].inv_scale = 1.0 / sc;
    d[j].family = c.family;
    d[j].nu = c.family == VECCHIA_COV_EXPONENTIAL ? 0.5 : c.nu;
    d[j].sigma2 = c.sigma2;
    d[j].range = c.range;
    d[j].nugget = c.nugget;
    if (seeds) d[j].seed = seeds[j];
    xo += P->D;
  }
  if (n > 1 && terms_dev) return set_error(VECCHIA_E_INVALID, "per-term output is for single instances");
  for (int j = 0; j < n; ++j) {
    // every address a kernel dereferences must be set before anything is enqueued
    const InstDesc& q = d[j];
    const bool geom_ok = q.covmat || (q.xs && q.ys);
    if (!q.prep || !q.bad_term || !q.x || !q.out || !q.kcnt || !q.sovk || !q.perm || !geom_ok ||
        (q.m > 0 && !q.nbr) || !d_desc_ || !d_term_bases_ || !d_ranges_ || !d_aux64_ || !d_sums_ ||
        !d_Z_ || (any_f32_ && !d_aux32_))
      return set_error(VECCHIA_E_HIP, "internal error: incomplete device descriptor");
  }
  return VECCHIA_OK;
}

vecchia_status Batch::run(const double* x_dev, const double* scales, const vecchia_cov* covs,
                          double* out_dev, double* terms_dev, const uint64_t* seeds, hipStream_t s) {
  const int n = (int)plans_.size();
  if (!x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "x_dev and out_dev must be device pointers");
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != device_) return set_error(VECCHIA_E_INVALID, "current device differs from the batch's device");
  // device buffers first: the descriptors below carry their addresses
  vecchia_status st = allocate();
  if (st != VECCHIA_OK) return st;
  std::vector<InstDesc> d;
  st = fill_desc(x_dev, scales, covs, out_dev, terms_dev, seeds, &d);
  if (st != VECCHIA_OK) return st;
  hipError_t e = hipSuccess;
  if (!tables_uploaded_) {
    // host tables live as long as the batch, so the asynchronous copy is safe
    e = hipMemcpyAsync(d_term_bases_, term_bases_.data(), sizeof(int64_t) * (n + 1),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !ranges_.empty())
      e = hipMemcpyAsync(d_ranges_, ranges_.data(), sizeof(RangeDesc) * ranges_.size(),
                         hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_error(e, "batch tables");
    tables_uploaded_ = true;
  }
  // stage the descriptors in pinned memory no earlier copy still reads
  InstDesc* h = ext_stage_;
  int slot = -1;
  if (!h) {
    slot = stage_next_;
    stage_next_ = (stage_next_ + 1) % kRing;
    if (stage_used_[slot]) e = hipEventSynchronize(stage_ev_[slot]);
    if (e != hipSuccess) return hip_error(e, "staging wait");
    h = h_stage_ + (size_t)slot * n;
  }
  std::memcpy(h, d.data(), sizeof(InstDesc) * n);
  e = hipMemcpyAsync(d_desc_, h, sizeof(InstDesc) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && slot >= 0) e = hipEventRecord(stage_ev_[slot], s);
  if (e != hipSuccess) return hip_error(e, "descriptor copy");
  if (slot >= 0) stage_used_[slot] = true;

  static const bool no_graph = std::getenv("VECCHIA_NO_GRAPH") != nullptr;
  const bool use_graph = !no_graph && !graph_failed_ && s != nullptr && eager_runs_ >= 1 && !ext_stage_ &&
                         !profiling_enabled();
  if (use_graph) {
    if (graph_exec_ && graph_stream_ != s) {
      // graphs are replayed on the stream they were captured for
      hipGraphExecDestroy(graph_exec_);
      graph_exec_ = nullptr;
    }
    if (!graph_exec_) {
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        st = enqueue(s, true);
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (st == VECCHIA_OK && e2 == hipSuccess && g) {
          e2 = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
          if (e2 != hipSuccess) graph_exec_ = nullptr;
        }
        if (g) hipGraphDestroy(g);
        if (!graph_exec_) graph_failed_ = true;
      } else {
        graph_failed_ = true;
      }
      hipGetLastError();
      graph_stream_ = s;
    }
  }
  if (graph_exec_ && use_graph) {
    e = hipGraphLaunch(graph_exec_, s);
    if (e != hipSuccess) return hip_error(e, "graph launch");
  } else {
    st = enqueue(s, true);
    if (st != VECCHIA_OK) return st;
    ++eager_runs_;
  }
  e = hipEventRecord(done_ev_, s);
  if (e != hipSuccess) return hip_error(e, "event record");
  last_stream_ = s;
  ran_ = true;
  return VECCHIA_OK;
}

vecchia_status Batch::run_noalloc(char* ws, const uint64_t* Z_dev, const double* x_dev, const double* scales,
                                  const vecchia_cov* covs, double* out_dev, double* terms_dev,
                                  const uint64_t* seeds, hipStream_t s) {
  if (!x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "x_dev and out_dev must be device pointers");
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != device_) return set_error(VECCHIA_E_INVALID, "current device differs from the batch's device");
  if (d_ws_ || h_stage_) return set_error(VECCHIA_E_INVALID, "internal error: batch already holds resources");
  carve(ws);
  d_Z_ = Z_dev;
  std::vector<InstDesc> d;
  vecchia_status st = fill_desc(x_dev, scales, covs, out_dev, terms_dev, seeds, &d);
  if (st != VECCHIA_OK) return st;
  // the workspace opens with the descriptors, the term bases and the ranges:
  // one host image of that header, written by kernels that take it by value
  const int n = (int)plans_.size();
  const size_t hdr = (size_t)(reinterpret_cast<char*>(d_aux64_) - ws);
  std::vector<char> img(hdr, 0);
  std::memcpy(img.data(), d.data(), sizeof(InstDesc) * n);
  std::memcpy(img.data() + (reinterpret_cast<char*>(d_term_bases_) - ws), term_bases_.data(),
              sizeof(int64_t) * (n + 1));
  if (!ranges_.empty())
    std::memcpy(img.data() + (reinterpret_cast<char*>(d_ranges_) - ws), ranges_.data(),
                sizeof(RangeDesc) * ranges_.size());
  hipError_t e = launch_store_bytes(ws, img.data(), hdr, s);
  if (e != hipSuccess) return hip_error(e, "descriptor store");
  st = enqueue(s, false);
  if (st != VECCHIA_OK) return st;
  last_stream_ = s;
  return VECCHIA_OK;
}

vecchia_status Batch::status(std::vector<int64_t>* bad) {
  const int n = (int)plans_.size();
  bad->assign(n, -1);
  if (!ran_) return VECCHIA_OK;
  hipError_t e = hipEventSynchronize(done_ev_);
  if (e != hipSuccess) return hip_error(e, "wait");
  std::vector<int64_t> h(n);
  e = hipMemcpy(h.data(), d_bad_, sizeof(int64_t) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "status copy");
  vecchia_status st = VECCHIA_OK;
  for (int j = 0; j < n; ++j) {
    if (h[j] != INT64_MAX) {
      (*bad)[j] = h[j];
      if (st == VECCHIA_OK)
        st = set_error(VECCHIA_E_NOT_PD, "instance " + std::to_string(j) + ": covariance block of plan term " +
                                             std::to_string(h[j]) + " is not positive definite");
    }
  }
  return st;
}

vecchia_status Batch::time_main_launch(hipStream_t s, int reps, float* median_ms) {
  if (!ran_ || launches_.empty() || reps < 1) return set_error(VECCHIA_E_INVALID, "nothing to time");
  const Launch& L = launches_[0];
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(ev[2 * r], s);
    if (e == hipSuccess)
      e = launch_qmc(L.K, L.precision, L.block, d_desc_, d_ranges_ + L.range_off, L.n_ranges, L.n_items, d_aux64_,
                     d_aux32_, d_Z_, d_sums_, s);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * r + 1], s);
  }
  std::vector<float> t(reps, 0.0f);
  if (e == hipSuccess) e = hipEventSynchronize(ev[2 * reps - 1]);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
  for (auto& x : ev)
    if (x) hipEventDestroy(x);
  if (e != hipSuccess) return hip_error(e, "timing");
  std::sort(t.begin(), t.end());
  *median_ms = t[reps / 2];
  return VECCHIA_OK;
}

}  // namespace vecchia

extern "C" {

vecchia_status vecchia_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(vecchia::g_prof_mu);
  vecchia::g_prof_on = on != 0;
  return VECCHIA_OK;
}

vecchia_status vecchia_profile_read(int32_t K, int32_t precision, double* total_ms, int64_t* launches,
                                    int64_t* sov_steps) {
  std::lock_guard<std::mutex> lk(vecchia::g_prof_mu);
  double ms = 0.0;
  int64_t nl = 0, st = 0;
  for (const auto& r : vecchia::g_prof) {
    if (r.K != K || r.precision != precision) continue;
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return vecchia::hip_error(e, "profile read");
    ms += t;
    ++nl;
    st += r.steps;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = nl;
  if (sov_steps) *sov_steps = st;
  return VECCHIA_OK;
}

vecchia_status vecchia_profile_reset(void) {
  std::lock_guard<std::mutex> lk(vecchia::g_prof_mu);
  for (auto& r : vecchia::g_prof) {
    hipEventSynchronize(r.b);
    vecchia::g_prof_pool.push_back(r.a);
    vecchia::g_prof_pool.push_back(r.b);
  }
  vecchia::g_prof.clear();
  return VECCHIA_OK;
}

}  // extern "C"
