// Host runtime objects behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "vecchia_internal.h"

struct vecchia_plan_s;

namespace vecchia {

vecchia_status set_error(vecchia_status st, const std::string& msg);
// kernel timing hook (vecchia_profile_*)
bool profiling_enabled();
hipError_t profile_events(hipEvent_t* a, hipEvent_t* b);
void profile_record(int K, int precision, hipEvent_t a, hipEvent_t b, int64_t sov_steps);
vecchia_status hip_error(hipError_t e, const char* what);
const uint64_t* device_lattice_table(int device, hipError_t* err);
// Generators Z_j of the first n primes, computed on the host.
void host_lattice_table(uint64_t* Z, int n);
// Generators Z_j of the first n primes (n >= 1), cached per device and grown on
// demand; the returned table stays valid until the process ends.
const uint64_t* device_lattice_table_n(int device, int n, hipError_t* err);
bool valid_cov(const vecchia_cov& c, std::string* why);
bool valid_qmc(const vecchia_qmc& q, std::string* why);
// Lattice points per QMC work item for an instance with conditioning-set size
// m: the autotuner's choice for (precision, m) when one was made, else the
// default (2048 FP32 / 512 FP64), capped at N rounded up to 64.
int chunk_points_for(int m, int precision, int n_points);
int tuned_chunk(int precision, int m);            // 0 = not tuned
void set_tuned_chunk(int precision, int m, int chunk_points);

// Everything one evaluation of a fixed set of instances needs on the device.
class Batch {
 public:
  ~Batch();
  // Validates and lays out the workspace; allocates nothing yet.
  static vecchia_status create(const std::vector<vecchia_plan_s*>& plans,
                               const std::vector<vecchia_qmc>& qmcs, std::unique_ptr<Batch>* out);
  // Bytes of device memory run() needs (workspace + descriptors).
  size_t workspace_bytes() const { return ws_bytes_; }
  vecchia_status run(const double* x_dev, const double* scales, const vecchia_cov* covs,
                     double* out_dev, double* terms_dev, const uint64_t* seeds, hipStream_t s);
  vecchia_status status(std::vector<int64_t>* bad);  // waits for the last run
  // As run(), on a caller-provided device workspace only: ws (workspace_bytes(),
  // 256-byte aligned) and Z_dev (the lattice generators, kMaxM entries). Nothing
  // is allocated: descriptors and tables reach the device as kernel arguments,
  // every launch runs on s, and no event, graph or timing hook is used. The
  // batch must not have run() before; NOT_PD shows only as NaN outputs.
  vecchia_status run_noalloc(char* ws, const uint64_t* Z_dev, const double* x_dev, const double* scales,
                             const vecchia_cov* covs, double* out_dev, double* terms_dev, const uint64_t* seeds,
                             hipStream_t s);
  // Run on caller-owned memory instead of allocating: ws (workspace_bytes(),
  // 256-byte aligned, device) and stage (n() descriptors, pinned host, not
  // reused by the caller before this batch's work has been consumed).
  // Optional side streams (caller-owned) let such a batch run its smaller
  // launches beside the largest one, as a batch with its own streams does.
  void bind_external(char* ws, InstDesc* stage, hipStream_t side0 = nullptr, hipStream_t side1 = nullptr) {
    ext_ws_ = ws;
    ext_stage_ = stage;
    ext_side_[0] = side0;
    ext_side_[1] = side1;
  }
  // Instance j reads its thresholds at x[j] (n() device pointers) instead of a
  // slice of one buffer: requests of the serving loop, each with its own.
  void set_x_ptrs(std::vector<const double*> x) { x_ptrs_ = std::move(x); }
  const int64_t* device_bad_terms() const { return d_bad_; }
  int n() const { return (int)plans_.size(); }
  const std::vector<vecchia_qmc>& qmcs() const { return qmcs_; }
  int chunk_points(int j) const { return desc_[j].chunk_points; }
  // Every instance reads the same thresholds (x_dev itself, D values) instead of
  // consecutive slices of x_dev: several instances of one plan at different
  // scales, as the scale-mixture quadrature needs.
  void set_shared_x(bool on) { shared_x_ = on; }
  // Instance j reads its thresholds at x_dev + off[j] (n() offsets): several
  // instances of each of several plans, as the batched scale mixture needs.
  void set_x_offsets(std::vector<int64_t> off) { x_off_ = std::move(off); }
  // After a completed run(): re-launches the launch with the most work `reps`
  // times on s between HIP events and returns the median duration (autotuner).
  vecchia_status time_main_launch(hipStream_t s, int reps, float* median_ms);
  hipStream_t last_stream() const { return last_stream_; }

 private:
  struct Launch {
    int K;
    int precision;
    bool block;
    int range_off;
    int n_ranges;
    int64_t n_items;
    int64_t sov_steps;   // sum over the launch's terms of n_shifts * n_points * K
  };
  vecchia_status allocate();
  void carve(char* base);   // workspace arrays at base (the layout of create())
  vecchia_status fill_desc(const double* x_dev, const double* scales, const vecchia_cov* covs, double* out_dev,
                           double* terms_dev, const uint64_t* seeds, std::vector<InstDesc>* out) const;
  vecchia_status enqueue(hipStream_t s, bool allow_profile);

  std::vector<vecchia_plan_s*> plans_;
  std::vector<vecchia_qmc> qmcs_;
  std::vector<InstDesc> desc_;          // host template of the descriptors
  std::vector<int64_t> term_bases_;     // n + 1
  std::vector<RangeDesc> ranges_;
  std::vector<Launch> launches_;
  std::vector<size_t> prep_off_;        // byte offset of each instance's prep block
  int64_t total_terms_ = 0;
  int64_t total_sums_ = 0;              // triples
  size_t prep_bytes_ = 0;
  bool any_f32_ = false;
  size_t ws_bytes_ = 0;
  int device_ = 0;

  char* d_ws_ = nullptr;
  InstDesc* d_desc_ = nullptr;
  int64_t* d_term_bases_ = nullptr;
  RangeDesc* d_ranges_ = nullptr;
  Aux64* d_aux64_ = nullptr;
  Aux32* d_aux32_ = nullptr;
  double* d_sums_ = nullptr;
  double2* d_term_res_ = nullptr;
  int64_t* d_bad_ = nullptr;
  char* d_prep_ = nullptr;
  const uint64_t* d_Z_ = nullptr;
  // terms of FP32 instances handed to FP64 (see InstDesc)
  int32_t* d_promote_ = nullptr;
  int32_t* d_plist_ = nullptr;
  int64_t* d_pctr_ = nullptr;
  int32_t plist_cap_ = 0;
  int32_t ipt_max_ = 0;
  int max_vars_ = 1;   // most variables of any term (sizes the set-up kernel's tiles)

  static constexpr int kRing = 4;       // pinned descriptor staging slots
  InstDesc* h_stage_ = nullptr;
  hipEvent_t stage_ev_[kRing] = {};
  bool stage_used_[kRing] = {};
  int stage_next_ = 0;

  // side streams: the QMC launches after the largest run beside it
  static constexpr int kSideStreams = 2;
  hipStream_t side_[kSideStreams] = {};
  hipEvent_t fork_ev_ = nullptr;
  hipEvent_t join_ev_[kSideStreams] = {};

  hipEvent_t done_ev_ = nullptr;
  hipStream_t last_stream_ = nullptr;
  bool ran_ = false;

  char* ext_ws_ = nullptr;
  InstDesc* ext_stage_ = nullptr;
  hipStream_t ext_side_[kSideStreams] = {};
  bool own_side_ = false;
  std::vector<const double*> x_ptrs_;
  bool tables_uploaded_ = false;
  bool shared_x_ = false;
  std::vector<int64_t> x_off_;

  hipGraphExec_t graph_exec_ = nullptr;
  hipStream_t graph_stream_ = nullptr;
  bool graph_failed_ = false;
  int eager_runs_ = 0;
};

}  // namespace vecchia

struct vecchia_plan_s {
  int device = 0;
  int64_t D = 0;
  int32_t m = 0;
  vecchia_cov cov{};
  bool matrix = false;
  std::vector<int64_t> perm;       // plan position -> user index
  std::vector<int32_t> kcnt;       // host copy of k_i
  // censored plans (eq. (11)): plan positions < n_obs are the uncensored sites;
  // sovk[i] is the SOV dimension of term i (0 for a density term, else the
  // number of censored neighbours); empty with n_obs = 0
  int64_t n_obs = 0;
  std::vector<int32_t> sovk;
  int32_t* d_sovk = nullptr;
  // block plans (joint terms of p sites, Section 3.2): n_terms groups, each with
  // its variable list (CSR, conditioning set first) and denominator split;
  // sovk holds each term's SOV dimension (variables - 1)
  int32_t block = 0;
  int32_t block_nv = 0;            // most variables of any term
  int64_t n_terms = 0;
  std::vector<int32_t> bvar_off, bvars, split;
  int32_t* d_bvar_off = nullptr;
  int32_t* d_bvars = nullptr;
  int32_t* d_split = nullptr;
  const std::vector<int32_t>& sov_dims() const { return (n_obs > 0 || block > 0) ? sovk : kcnt; }
  int64_t terms() const { return block > 0 ? n_terms : D; }
  // geometry plans keep {xs, ys (D doubles each), perm (D int32)} in one
  // allocation, d_geo, laid out as the replan staging, so one copy moves them
  void* d_geo = nullptr;
  double* d_xs = nullptr;
  double* d_ys = nullptr;
  double* d_cov = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_nbr = nullptr;
  int32_t* d_kcnt = nullptr;
  // neighbour-search grid of large plans (kKnnGridMinD); geometry refreshed by replan
  bool has_grid = false;
  vecchia::KnnGrid grid{};
  std::unique_ptr<vecchia::Batch> single;   // cached one-instance batch of vecchia_logcdf
  // scale-mixture evaluation (vecchia_mixture_logcdf): the two passes' batches
  // and a device buffer for their per-node results (2 x (2 + max nodes) doubles)
  std::unique_ptr<vecchia::Batch> mix1, mix2;
  double* d_mix = nullptr;
  // workspace of vecchia_full_logcdf (covariance / Cholesky factor, limits,
  // the points' y, partial sums), grown on demand
  void* d_full = nullptr;
  size_t full_bytes = 0;
  // pinned staging for vecchia_replan: {xs, ys (D doubles), perm (D int32)} x 2
  char* h_replan[2] = {nullptr, nullptr};
  hipEvent_t replan_ev[2] = {nullptr, nullptr};
  bool replan_used[2] = {false, false};
  int replan_next = 0;
  std::atomic<int> inflight{0};
  std::mutex mu;
};

struct vecchia_batch_s {
  std::unique_ptr<vecchia::Batch> b;
};
