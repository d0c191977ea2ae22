// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/vecchia.h"

namespace vecchia {

constexpr int kMaxM = VECCHIA_MAX_M;   // conditioning-set size limit
constexpr int kMaxVars = kMaxM + 1;    // variables per term
constexpr double kPromoteZ = -4.0;     // FP32 instances: terms with a limit below this many SDs run in FP64
constexpr double kRedoSe = 0.02;       // FP32 instances: terms whose log-term SE exceeds this run again in FP64
// Chains of up to this many steps run fully unrolled with y in registers;
// longer ones (up to kMaxM) run in the general kernel with y in LDS.
constexpr int kMaxUnrolledK = 31;
constexpr int kFinalizeThreads = 256;
// A launch may hold fewer than 2^32 work-items in total; per-term and per-item
// kernels are split into launches of at most this many threads.
constexpr int64_t kMaxLaunchThreads = (int64_t)1 << 31;

// One log-CDF instance of a launch (device-resident descriptor).
struct InstDesc {
  const double* xs;        // plan-order x coordinates (geometry plans)
  const double* ys;        // plan-order y coordinates
  const double* covmat;    // explicit D x D covariance (matrix plans) or null
  const int32_t* perm;     // plan position -> user index
  const int32_t* nbr;      // D x m conditioning sets (plan indices), -1 padded
  const int32_t* kcnt;     // D: size k_i of each conditioning set
  const int32_t* sovk;     // D: SOV dimension of each term (= kcnt unless censored)
  const double* x;         // thresholds, user order
  double* out;             // {log F, SE}
  double* terms_out;       // D x 2 user order, or null
  void* prep;              // per-term scaled Cholesky rows (double or float), term 0
  // FP32 instances hand some terms to FP64 kernels on the same lattice points:
  //  - at set-up, terms with a chain limit below kPromoteZ standard deviations
  //    (of the variable given the observed sites); their FP32 items exit at once;
  //  - after the FP32 pass, terms whose estimate is heavy-tailed (SE of the
  //    log-term above kRedoSe), evaluated again.
  // promote[t] (global term index) is 0, 1 (set-up) or 2 (re-run). A handed-over
  // term's FP64 rows take the place of its FP32 rows: prep_f64(I, i). plist holds
  // two lists of global term indices, plist_cap (= the batch's term count) each:
  // [0, cap) the set-up promotions, [cap, 2 cap) the re-runs; pctr = {count,
  // work counter} of each. Every qualifying term gets a slot, so a term's value
  // depends only on its instance. Shared by the batch.
  int32_t* promote;
  int32_t* plist;
  int64_t* pctr;
  int32_t plist_cap;
  int32_t pad0_;
  int64_t D;
  int64_t n_terms;         // terms: D, or the number of groups of a block plan
  // block plans (joint terms, Section 3.2): term i's variables are
  // bvars[bvar_off[i] .. bvar_off[i+1]) (plan indices, conditioning set first);
  // its denominator is the CDF of the first split[i] of them. Null otherwise.
  const int32_t* bvar_off;
  const int32_t* bvars;
  const int32_t* split;
  int64_t n_obs;           // plan positions < n_obs are uncensored sites (eq. (11)); 0 = plain
  int64_t term_base;       // global index of plan term 0 (aux arrays)
  int64_t sums_base;       // index of (term 0, shift 0, chunk 0) in the sums triples
  int64_t* bad_term;       // first plan-order term whose Cholesky failed (min)
  double inv_scale, sigma2, range, nugget, nu;
  int32_t family;          // VECCHIA_COV_*
  int32_t m;
  int32_t n_points, n_shifts;
  int32_t passes;          // 2: the denominators come from a second lattice (VECCHIA_QMC_INDEPENDENT)
  int32_t pad_;
  uint64_t seed;
  int32_t prep_stride;     // elements per term in prep (FP32 instances: even, room for the FP64 rows)
  int32_t precision;       // VECCHIA_FP64 / VECCHIA_FP32_LOOP
  int32_t chunk_points;    // lattice points per work item (a multiple of 64)
  int32_t n_chunks;        // ceil(n_points / chunk_points)
};

// A contiguous run of terms with the same K inside one instance. Its work items
// are (term, pass, shift, chunk), n_terms * passes * n_shifts * n_chunks of
// them, in that nesting order.
struct RangeDesc {
  int64_t item_begin;      // exclusive prefix of items over the ranges of a launch
  int64_t term_begin;      // plan index of the first term
  int32_t inst;            // instance index
  int32_t K;               // conditioning-set size of every term of the range
  int32_t items_per_term;  // passes * n_shifts * n_chunks
  int32_t n_chunks;
};

// Auxiliary per-term values written by term_setup.
// Phi(b_0/L_00) and its log; e0 = -1 marks a term that is 0 (a -inf limit),
// whose value lt0 = -inf is exact.
struct Aux64 { double e0; double lt0; };
// FP32 form of e0 = Phi(b_0/L_00): e0 = em0 * 2^en0 (en0 = 0 unless b_0/L_00 <= 0),
// ec0 = 1 - e0, neg0 = 1 if b_0/L_00 <= 0.
struct Aux32 { float em0, en0, ec0, neg0; };

// Uniform grid over the bounding box for the nearest-neighbour search of large
// plans: G x G cells, points of cell c at [start[c], start[c+1]) of gx/gy/gid.
struct KnnGrid {
  int32_t G;
  double x0, y0, wx, wy;
  double margin;        // absolute slack for rounding in cell bounds
  int32_t* cell;        // D: cell of each plan point
  int32_t* start;       // G*G + 1
  int32_t* cursor;      // G*G (scatter positions)
  double* gx;           // D, points in cell order
  double* gy;
  int32_t* gid;         // D: plan index of each slot
};
// Plans with more points than this search neighbours through the grid.
constexpr int64_t kKnnGridMinD = 16384;

// FP64 rows of plan term i of an FP32 instance, in place of its FP32 rows
// (a term handed to the FP64 kernels; row a at offset a (a + 1) / 2).
__host__ __device__ inline double* prep_f64(const InstDesc& I, int64_t i) {
  return reinterpret_cast<double*>(I.prep) + i * (int64_t)(I.prep_stride / 2);
}

// Launchers (kernels_*.hip).
// group > 1: query i's candidates are j < i - i mod group (no grid then).
hipError_t launch_knn(const double* xs, const double* ys, int64_t D, int m, int32_t* nbr,
                      int32_t* kcnt, const KnnGrid* grid, hipStream_t s, int group = 1);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
// Copies `bytes` bytes of host memory to dst (device, 8-byte aligned) by kernels
// that take them as arguments (no staging buffer, no memcpy node).
hipError_t launch_store_bytes(void* dst, const void* src_host, size_t bytes, hipStream_t s);
// max_vars: the most variables (conditioning set and the term's own) of any
// term of the batch, at most kMaxVars; it sizes the kernel's LDS tiles.
hipError_t launch_setup(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                        int64_t total_terms, int max_vars, Aux64* aux64, Aux32* aux32, hipStream_t s);
// The FP64 rows of the terms on a device-side list (count at *count, at most
// cap entries): the re-runs of an FP32 evaluation. A persistent grid that
// finds nothing to do when the list is empty.
hipError_t launch_setup_redo(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases, int max_vars,
                             Aux64* aux64, Aux32* aux32, const int32_t* list, const int64_t* count, int64_t cap,
                             hipStream_t s);
// block: the launch's instances are block plans (denominator split per term).
hipError_t launch_qmc(int K, int precision, bool block, const InstDesc* d_insts, const RangeDesc* d_ranges,
                      int n_ranges, int64_t n_items, const Aux64* aux64, const Aux32* aux32,
                      const uint64_t* d_Z, double* sums, hipStream_t s);
// The handed-over terms of FP32 instances in FP64: a persistent grid takes
// (term, item) pairs from a device-side list (ctr[0] entries, at most cap;
// ipt_max items per term at most; ctr[1] is the work counter) until none is left.
hipError_t launch_qmc_promoted(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases, const Aux64* aux64,
                               const uint64_t* d_Z, double* sums, const int32_t* list, int64_t* ctr,
                               int64_t cap, int ipt_max, hipStream_t s);
// Scale-mixture quadrature weights (log), passed by value to the combine kernel.
constexpr int kMaxMixNodes = 64;
constexpr int kMixSearch = VECCHIA_MIX_SEARCH_NODES;
struct MixWeights {
  double logw[kMaxMixNodes];
  int32_t n;
};
// out[0] = log sum_k exp(logw_k + logF_k), out[1] = sqrt(sum_k (c_k / G)^2 se_k^2)
// from node_out (n x {log F_k, se_k}); nodes_out (optional) receives a copy of node_out.
hipError_t launch_mixture_combine(const double* node_out, const MixWeights& mw, double* out, double* nodes_out,
                                  hipStream_t s);
// n_mix mixtures of n_nodes nodes each (node_out: n_mix x n_nodes x {log F, se};
// logw: n_mix x n_nodes); out: n_mix x {log G, se}; total (optional): the sum of
// the log G and the root sum of squares of the SEs.
hipError_t launch_mixture_combine_many(const double* node_out, const double* logw, int n_nodes, int64_t n_mix,
                                       double* out, double* total, hipStream_t s);
// term_finalize over every term, then (redo_list non-null) over the re-run list
// after its FP64 pass, then the per-instance sums. Without a list the first
// pass hands nothing over.
hipError_t launch_finalize_terms(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                                 int64_t total_terms, const Aux64* aux64, const double* sums,
                                 double2* term_res, bool allow_redo, hipStream_t s);
hipError_t launch_finalize_redo(const InstDesc* d_insts, int n_inst, const int64_t* d_term_bases,
                                const Aux64* aux64, const double* sums, double2* term_res,
                                const int32_t* list, const int64_t* count, int64_t cap, hipStream_t s);
hipError_t launch_logsum(const InstDesc* d_insts, int n_inst, const double2* term_res, hipStream_t s);

}  // namespace vecchia
