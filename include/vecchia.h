/*
 * vecchia.h - C ABI of the MI355X (gfx950) Vecchia Gaussian log-CDF library.
 *
 * Method: Nascimento & Shaby, "A Vecchia Approximation for High-Dimensional
 * Gaussian Cumulative Distribution Functions Arising from Spatial Data".
 *   log F(x) ~= log Phi(x_1) + sum_{i>=2} [log Phi(x_{i,N_i}) - log Phi(x_{N_i})]
 * (Section 2.2, eq. (6)), N_i = the min(m, i-1) nearest preceding locations
 * (Section 2.1 after eq. (4)), each ratio estimated by Genz's separation of
 * variables and a randomized rank-1 lattice QMC rule (Section 2.2 after eq.
 * (6)), computed on the log scale and summed at the end (Section 3.1).
 * The process is zero-mean with a stationary isotropic covariance; callers
 * pass x - mu.
 *
 * Conventions for every entry point:
 *  - No exception crosses the ABI. A non-OK status sets a thread-local message
 *    readable with vecchia_last_error().
 *  - "_host" pointers are host memory, "_dev" pointers are device memory of the
 *    current HIP device. The caller owns both and every stream.
 *  - Objects (plans, batches, servers) are owned by the library and released by
 *    their _destroy call.
 *  - Streams are hipStream_t passed as void* (NULL = the default stream).
 *  - Calls that enqueue GPU work are asynchronous on the given stream; their
 *    device outputs are valid once the stream reaches that point. A numerically
 *    failed term (Cholesky pivot <= 0) makes the affected instance's outputs NaN
 *    and is reported by vecchia_plan_status / vecchia_batch_status.
 *  - Calls on one plan (or one batch) must be ordered on one stream at a time:
 *    the plan's workspace is reused by every call.
 */
#ifndef VECCHIA_H
#define VECCHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vecchia_plan_s* vecchia_plan_t;
typedef struct vecchia_batch_s* vecchia_batch_t;
typedef struct vecchia_server_s* vecchia_server_t;
typedef struct vecchia_mixbatch_s* vecchia_mixbatch_t;

typedef enum {
  VECCHIA_OK = 0,
  VECCHIA_E_INVALID = 1,     /* bad argument; nothing was enqueued                         */
  VECCHIA_E_NOMEM = 2,       /* device or host allocation failed, or over the HBM budget    */
  VECCHIA_E_NOT_PD = 3,      /* a term's covariance block is not positive definite          */
  VECCHIA_E_HIP = 4,         /* a HIP runtime call failed                                   */
  VECCHIA_E_BUSY = 5,        /* object still has requests in flight                         */
  VECCHIA_E_NOT_READY = 6,   /* result not available yet                                    */
  VECCHIA_E_NONFINITE = 7    /* non-finite input                                            */
} vecchia_status;

/* Orderings applied before neighbour selection (the paper orders components
 * before choosing nearest neighbours, Section 3.2, and names no rule).
 * COORD: lexicographic by (x, y, index). MAXMIN: first the point nearest the
 * bounding-box centre, then repeatedly the point farthest from the selected
 * set (ties: lowest index). GIVEN: a caller permutation. */
enum { VECCHIA_ORDER_GIVEN = 0, VECCHIA_ORDER_COORD = 1, VECCHIA_ORDER_MAXMIN = 2 };

/* Covariance families: exponential sigma2*exp(-h/range) (the paper's model,
 * Sections 3 and 4.1) and Matern with nu in {0.5, 1.5, 2.5},
 * K(h) = sigma2 2^(1-nu)/Gamma(nu) (sqrt(2 nu) h/range)^nu K_nu(sqrt(2 nu) h/range). */
enum { VECCHIA_COV_EXPONENTIAL = 0, VECCHIA_COV_MATERN = 1 };

/* Arithmetic of the QMC sample loop. FP64: every step in double precision.
 * FP32_LOOP: the SOV chain (Phi, Phi^-1, products in log space) in single
 * precision; covariance, Cholesky, per-term means and the sum in double. */
enum { VECCHIA_FP64 = 0, VECCHIA_FP32_LOOP = 1 };

#define VECCHIA_MAX_M 63          /* conditioning-set size limit (term dimension <= 64) */
#define VECCHIA_MAX_SHIFTS 65536
#define VECCHIA_MAX_POINTS 1073741824
#define VECCHIA_MIX_SEARCH_NODES 24   /* search points of the scale-mixture rule */

typedef struct {
  int32_t family;   /* VECCHIA_COV_*                                  */
  int32_t reserved; /* must be 0                                      */
  double nu;        /* Matern smoothness: 0.5, 1.5 or 2.5             */
  double sigma2;    /* marginal variance > 0                          */
  double range;     /* range parameter > 0                            */
  double nugget;    /* >= 0, added to the diagonal                    */
} vecchia_cov;

/* vecchia_qmc.flags: estimate each term's numerator and denominator from
 * separate point sets (the literal reading of Section 2.2, which asks for a QM
 * estimate of each): the numerator from the term's lattice, the denominator
 * from a second lattice whose shifts are SplitMix64 outputs key + 2^61. Twice
 * the QMC work; the two estimates are independent, so
 * se^2 = [sum_r (n_r/n - 1)^2 + sum_r (d_r/d - 1)^2] / (R (R - 1)) (per-shift
 * means n_r, d_r). The default (flags = 0) shares one lattice, whose SE is
 * several times smaller at the same work. */
#define VECCHIA_QMC_INDEPENDENT 1

typedef struct {
  int32_t n_points;   /* N lattice points per shift, 1..VECCHIA_MAX_POINTS          */
  int32_t n_shifts;   /* R random shifts, 1..VECCHIA_MAX_SHIFTS (R = 1: SE is NaN)  */
  uint64_t seed;      /* keys the random shifts                                     */
  int32_t precision;  /* VECCHIA_FP64 or VECCHIA_FP32_LOOP (terms with a limit below -4
                         standard deviations run in FP64 within an FP32 evaluation) */
  int32_t flags;      /* 0 or VECCHIA_QMC_INDEPENDENT                               */
} vecchia_qmc;

/* Mixing law of the Gaussian scale mixture X = R W (Section 4, eqs. (7)-(8)):
 * F_R(r) = 1 - exp{-gamma (r^beta - 1) / beta} for beta > 0, and the Pareto law
 * 1 - r^-gamma for beta = 0 (eq. (8) prints 1 - r^gamma, negative for r > 1),
 * both on r >= 1. */
typedef struct {
  double beta;        /* >= 0                                                   */
  double gamma;       /* > 0                                                    */
  int32_t n_nodes;    /* Gauss-Legendre nodes of the outer integral, 1..64     */
  int32_t reserved;   /* must be 0                                              */
} vecchia_mixture;

/* Message for the calling thread's last non-OK status ("" if none). */
const char* vecchia_last_error(void);

/* Ordering only, on the host (no GPU work). locs_host: D x 2 row-major
 * (x, y). perm_in_host: the permutation for VECCHIA_ORDER_GIVEN, else NULL.
 * perm_out_host[i] = user index placed at plan position i (D entries).
 * Errors: INVALID (D < 1, non-finite coordinates, bad ordering or permutation). */
vecchia_status vecchia_order(const double* locs_host, int64_t D, int32_t ordering,
                             const int64_t* perm_in_host, int64_t* perm_out_host);

/* Anisotropic distance of Section 4.1 as a change of coordinates (host only):
 * h_ij = |(s_i - s_j)^T R(phi)^-1 diag(1, A)| with R(phi) the rotation by phi is
 * the Euclidean distance between the mapped points
 *   s' = (x cos phi - y sin phi, A (x sin phi + y cos phi)),
 * so a plan over out_host (D x 2) with an isotropic covariance of range rho is
 * the anisotropic model, its neighbours the nearest under h. locs_host and
 * out_host may be the same array. Errors: INVALID (null, non-finite phi, A <= 0). */
vecchia_status vecchia_map_anisotropic(const double* locs_host, int64_t D, double phi, double A,
                                       double* out_host);

/* Build a plan: order the D locations, copy them to the device and find, with
 * the GPU kernel knn_preceding, each component's min(m, i) nearest preceding
 * neighbours under the (squared distance, plan index) order (Section 2.1).
 * locs_host: D x dim row-major, dim must be 2. cov: default covariance; family
 * and nu are fixed for the plan, sigma2/range/nugget may be overridden per
 * call. Synchronises hip_stream before returning.
 * Errors: INVALID (D < 1, D >= 2^31, dim != 2, m outside 0..63, bad ordering,
 * permutation or covariance, non-finite locations), NOMEM, HIP. */
vecchia_status vecchia_plan(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                            const int64_t* perm_in_host, int32_t m, const vecchia_cov* cov,
                            void* hip_stream, vecchia_plan_t* out);

/* Plan over an explicit D x D covariance (row-major, host, D <= 4096) with
 * identity ordering: the Vecchia product of Section 2.2, eq. (6), over a given
 * Sigma instead of one built from locations (Section 2.1 writes the
 * approximation for any covariance); used to run closed-form cases through the
 * same kernels.
 * nbr_host: D x m row-major plan indices, each row listing its conditioning set
 * (entries < i, distinct) first, padded with -1; NULL means the min(m, i)
 * immediately preceding indices in ascending order.
 * Errors: INVALID (bad sizes, non-finite or asymmetric matrix, bad lists),
 * NOMEM, HIP. Synchronises hip_stream. */
vecchia_status vecchia_plan_from_cov(const double* cov_host, int64_t D, const int32_t* nbr_host,
                                     int32_t m, void* hip_stream, vecchia_plan_t* out);

/* Censored plan of one replicate (Section 4, eq. (11)). observed_host: D flags
 * in user order, 1 = the site's value is observed (above the censoring
 * threshold: the likelihood takes the density there), 0 = censored (only
 * X_i <= x_i is known, x_i being the threshold). The sites are ordered by
 * `ordering` (as vecchia_plan), then every observed site is moved before every
 * censored one, each group keeping its relative order; neighbours are the m
 * nearest preceding sites in that order. vecchia_logcdf on this plan at scale r
 * returns the Vecchia form of eq. (11)'s integrand,
 *   log L_r(x) = sum_{i observed} log f(x_i / r | x_{N_i} / r) - |I| log r
 *              + sum_{i censored} log P(X_i <= x_i / r | censored neighbours <= x / r,
 *                                            observed neighbours = x / r),
 * each censored term an SOV/QMC ratio of the conditional Gaussian given its
 * observed neighbours (dimension: its censored neighbours + 1); the per-term
 * output holds the density terms with SE 0. vecchia_mixture_logcdf on it
 * returns log G_I(x). With no observed site the plan equals vecchia_plan's.
 * An observed site whose value is infinite has density 0: every term that
 * holds it is -inf (SE 0).
 * Errors: as vecchia_plan, and INVALID for flags other than 0 / 1. */
vecchia_status vecchia_plan_censored(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                                     const int64_t* perm_in_host, const uint8_t* observed_host, int32_t m,
                                     const vecchia_cov* cov, void* hip_stream, vecchia_plan_t* out);

/* Joint (block) conditional plan (Section 3.2). The sites are ordered as by
 * vecchia_plan and cut into consecutive groups of p (the last one ragged). The
 * conditioning set of a group is the union of its members' m nearest
 * neighbours among the sites of earlier groups (in member order, each list in
 * the (d^2, index) order, first occurrence kept), so a term has at most
 * p (m + 1) variables. Term g is Phi(x_{C_g}, x_{G_g}) / Phi(x_{C_g}) (C_g
 * first), estimated by one SOV chain whose denominator is the prefix of its
 * first |C_g| factors; its shift key is g. vecchia_logcdf's per-term output
 * then has one row per group, in group order. p = 1 gives vecchia_plan's plan.
 * The neighbour search scans all earlier sites (no grid). Errors: as
 * vecchia_plan, and INVALID unless 1 <= p and p (m + 1) <= 32. */
vecchia_status vecchia_plan_block(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                                  const int64_t* perm_in_host, int32_t m, int32_t p, const vecchia_cov* cov,
                                  void* hip_stream, vecchia_plan_t* out);

/* The terms of a block plan (host copies): *n_terms; var_off_host (n_terms + 1
 * offsets), vars_host (var_off_host[n_terms] plan indices: each term's
 * conditioning set, then its group) and split_host (n_terms conditioning-set
 * sizes) may each be NULL. Errors: INVALID (not a block plan). */
vecchia_status vecchia_plan_block_terms(vecchia_plan_t plan, int64_t* n_terms, int32_t* var_off_host,
                                        int32_t* vars_host, int32_t* split_host);

/* Plan of explicit joint terms over a D x D covariance (host, D <= 4096):
 * term g has the variables vars_host[var_off_host[g] .. var_off_host[g+1])
 * (1..32 distinct indices in 0..D-1) and the value
 * Phi(all of them) / Phi(the first split_host[g]), 0 <= split < variables.
 * log F is the sum over the n_terms terms; used for closed-form cases.
 * Errors: INVALID (bad sizes, matrix or term lists), NOMEM, HIP. */
vecchia_status vecchia_plan_from_cov_block(const double* cov_host, int64_t D, const int32_t* var_off_host,
                                           const int32_t* vars_host, const int32_t* split_host, int64_t n_terms,
                                           void* hip_stream, vecchia_plan_t* out);

/* Censored plan over an explicit covariance (as vecchia_plan_from_cov) whose
 * first n_observed variables are the observed ones (0 <= n_observed <= D).
 * Errors: as vecchia_plan_from_cov, and INVALID for n_observed outside 0..D. */
vecchia_status vecchia_plan_from_cov_censored(const double* cov_host, int64_t D, const int32_t* nbr_host,
                                              int32_t m, int64_t n_observed, void* hip_stream,
                                              vecchia_plan_t* out);

/* Number of observed sites of a plan (plan positions 0..n-1; 0 for a plain plan). */
vecchia_status vecchia_plan_censoring(vecchia_plan_t plan, int64_t* n_observed);

/* Recompute a geometry plan in place for new locations (same D, m and
 * covariance family): host ordering, then an asynchronous copy and the
 * knn_preceding kernel on hip_stream. Allocates nothing; the host ordering of
 * this call overlaps GPU work already queued. Must be ordered with the plan's
 * other calls on one stream. locs_host / perm_in_host as in vecchia_plan.
 * Errors: INVALID (matrix, censored or block plan, bad arguments), HIP. */
vecchia_status vecchia_replan(vecchia_plan_t plan, const double* locs_host, int32_t ordering,
                              const int64_t* perm_in_host, void* hip_stream);

/* D and m of a plan. */
vecchia_status vecchia_plan_info(vecchia_plan_t plan, int64_t* D, int32_t* m);

/* Copy the plan's ordering and neighbour table to the host:
 * perm_host[i] = user index at plan position i (D entries); nbr_host: D x m
 * row-major plan indices, -1 padded (may be NULL when m = 0). Synchronous. */
vecchia_status vecchia_plan_neighbours(vecchia_plan_t plan, int64_t* perm_host, int32_t* nbr_host);

/* Vecchia log-CDF of one instance: log P(X < x / scale).
 * x_dev: D doubles in user index order. scale > 0 divides the thresholds (the
 * scale-mixture integrand Phi_D(x / r), eq. (9)). cov_override: NULL or a
 * covariance with the plan's family and nu. q: QMC size, seed and precision.
 * out_dev: 2 doubles, {log F, standard error}. terms_dev: NULL or D x 2
 * doubles {log term, standard error} in user index order.
 * Infinite thresholds: +inf leaves a component unconstrained; a -inf threshold
 * gives log F = -inf, every term whose variables include it being exactly -inf
 * with SE 0 (other terms are unchanged). NaN thresholds give NaN.
 * Enqueues term_setup, the QMC kernels and finalize_logsum on hip_stream.
 * Errors: INVALID (bad arguments; nothing enqueued), NOMEM, HIP. */
vecchia_status vecchia_logcdf(vecchia_plan_t plan, const double* x_dev, double scale,
                              const vecchia_cov* cov_override, const vecchia_qmc* q,
                              double* out_dev, double* terms_dev, void* hip_stream);

/* As vecchia_logcdf, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The evaluation's workspace lives in a static device array of
 * VECCHIA_NOALLOC_SCRATCH_BYTES per GPU (held from the first call on that GPU
 * until the process ends); the call allocates no device or pinned memory,
 * creates no stream or event, and enqueues only kernels on hip_stream (the
 * descriptors travel as kernel arguments). Arguments, outputs and results are
 * those of vecchia_logcdf, bit for bit. Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (on any streams) race and must be
 * ordered. A covariance block that is not positive definite makes the outputs
 * NaN; it is not recorded for vecchia_plan_status.
 * Errors: INVALID (bad arguments; a workspace larger than the array, with the
 * bytes needed in the message; nothing enqueued), HIP. */
#define VECCHIA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vecchia_status vecchia_logcdf_noalloc(vecchia_plan_t plan, const double* x_dev, double scale,
                                      const vecchia_cov* cov_override, const vecchia_qmc* q,
                                      double* out_dev, double* terms_dev, void* hip_stream);

/* Wait for the plan's last call and report whether every term factored:
 * OK, or NOT_PD with the first failing plan-order term in *bad_term
 * (-1 when OK) and in the error message. */
vecchia_status vecchia_plan_status(vecchia_plan_t plan, int64_t* bad_term);

/* Release a plan and its device memory (the plan of Section 2.1's ordering and
 * neighbour sets, built once and reused by every evaluation). BUSY if server
 * requests on it are still in flight; the plan is then left intact. */
vecchia_status vecchia_plan_destroy(vecchia_plan_t plan);

/* A batch of n instances evaluated in one pass: one setup launch, one QMC
 * launch per distinct (conditioning-set size, precision) - the largest on the
 * caller's stream, the others on library-owned side streams running beside it -
 * and one segmented-sum launch, replayed from a captured HIP graph after the
 * first call on a non-default stream. plans: n plans (may repeat). qmcs: n QMC
 * settings (copied). */
vecchia_status vecchia_batch_create(const vecchia_plan_t* plans, int32_t n, const vecchia_qmc* qmcs,
                                    vecchia_batch_t* out);

/* Evaluate a batch. x_dev: thresholds of all instances concatenated in batch
 * order (sum of D doubles, each in its plan's user order). scales_host: n
 * scales or NULL (all 1). covs_host: n covariances or NULL (each plan's own).
 * out_dev: n x 2 doubles {log F, SE}. Errors: INVALID, NOMEM, HIP. */
vecchia_status vecchia_batch_logcdf(vecchia_batch_t batch, const double* x_dev,
                                    const double* scales_host, const vecchia_cov* covs_host,
                                    double* out_dev, void* hip_stream);

/* As vecchia_plan_status for every instance of the batch: bad_terms_host (n
 * entries, may be NULL) receives -1 or the first failing plan-order term. */
vecchia_status vecchia_batch_status(vecchia_batch_t batch, int64_t* bad_terms_host);

vecchia_status vecchia_batch_destroy(vecchia_batch_t batch);

/* Kernel timing for measurement tools. While enabled, evaluations record HIP
 * events around every QMC launch on its stream (HIP graphs are then not used).
 * A QMC launch covers the terms of one conditioning-set size K in one
 * precision. vecchia_profile_read waits for the recorded launches of (K,
 * precision) and returns their summed milliseconds, launch count and SOV steps
 * (sum over their terms of n_shifts * n_points * K). With K =
 * VECCHIA_PROFILE_FULL_SOV and VECCHIA_FP64 it reads vecchia_full_logcdf's
 * product-and-recursion kernel instead, whose "steps" are its FMAs over earlier
 * dimensions, D (D - 1) / 2 per lattice point (Section 3.1's comparator).
 * reset drops the records. */
#define VECCHIA_PROFILE_FULL_SOV (-1)
vecchia_status vecchia_profile_enable(int32_t on);
vecchia_status vecchia_profile_read(int32_t K, int32_t precision, double* total_ms, int64_t* launches,
                                    int64_t* sov_steps);
vecchia_status vecchia_profile_reset(void);

/* Scale-mixture marginal CDF, eq. (9): G(x) = int_1^inf h(r) f_R(r) dr with
 * h(r) the plan's vecchia_logcdf value at scale r: Phi_D(x / r) for a plain plan,
 * and for a censored plan (vecchia_plan_censored) the integrand of eq. (11), so
 * that G is the censored likelihood G_I(x). With v = -log(1 - F_R(R)) ~ Exp(1)
 * the integral is int_0^inf e^-v h(r(v)) dv, r(v) = e^(v / gamma) (beta = 0) or
 * (1 + beta v / gamma)^(1 / beta), capped at 1e300. Two batched passes:
 *   1. search: log h at v = 0 and v_j = 1e-4 (2e6)^((j-1)/22), j = 1..23, with
 *      max(64, 64 ceil(n_points / 1024)) lattice points (q's shifts and seed);
 *   2. the window [lo, hi] of vecchia_mixture_rule and n_nodes-point
 *      Gauss-Legendre on it at q's full size, combined on the device:
 *   out_dev[0] = log G = log sum_k w_k e^(-v_k) h(r(v_k)),
 *   out_dev[1] = its standard error (first-order propagation of the node SEs;
 *                0 when G = 0, i.e. every node is 0).
 * Every node uses q->seed (common random numbers). x_dev: D thresholds, user
 * order (device). cov_override as in vecchia_logcdf. nodes_dev (may be NULL):
 * n_nodes x {log h, se} per node (device). Synchronises hip_stream once
 * (after pass 1); the rest is asynchronous. The window holds the mode of
 * log h(v) - v that contains the search maximum (all of the mass for a unimodal
 * integrand). Errors: INVALID, NOMEM, HIP; NOT_PD through vecchia_plan_status. */
vecchia_status vecchia_mixture_logcdf(vecchia_plan_t plan, const double* x_dev, const vecchia_mixture* mix,
                                      const vecchia_cov* cov_override, const vecchia_qmc* q, double* out_dev,
                                      double* nodes_dev, void* hip_stream);

/* The search scales r(v_j) of vecchia_mixture_logcdf's first pass (host only):
 * VECCHIA_MIX_SEARCH_NODES values. Errors: INVALID. */
vecchia_status vecchia_mixture_search(const vecchia_mixture* mix, double* scales_out);

/* The second-pass rule of vecchia_mixture_logcdf for given search values
 * (host only). search_logh: VECCHIA_MIX_SEARCH_NODES values log h(v_j). With
 * l_j = search_logh[j] - v_j and j* its (first) maximum, window_out = {lo, hi}:
 * lo = the v_j nearest below j* with l_j < l_j* - 36 (else 0), hi = the one
 * nearest above (else 200). Then n_nodes Gauss-Legendre points on [lo, hi], in
 * s = log v when lo > 0 and hi / lo > 8, else in v: v_out[k], scales_out[k] =
 * r(v_k) and logw_out[k] = log(w_k times the map's Jacobian) - v_k.
 * Errors: INVALID (bad mixture, a NaN search value). */
vecchia_status vecchia_mixture_rule(const vecchia_mixture* mix, const double* search_logh, double* window_out,
                                    double* v_out, double* scales_out, double* logw_out);

/* Scale mixtures of many plans in one go: the censored log-likelihood of
 * Section 4 is sum_t log G_{I_t}(x_t) over replicates t, each G_{I_t} the
 * vecchia_mixture_logcdf of replicate t's censored plan. Create once per set
 * of plans (n >= 1; n_nodes in 1..64; q: QMC size and precision, shared; the
 * seed of replicate t is q->seed + t); the batch keeps the plans' addresses
 * (destroy it before them) and holds device memory for both passes of every
 * replicate: n x 24 search instances at the reduced lattice size and n x n_nodes
 * node instances. Errors: INVALID, NOMEM, HIP. */
vecchia_status vecchia_mixbatch_create(const vecchia_plan_t* plans, int32_t n, int32_t n_nodes,
                                       const vecchia_qmc* q, vecchia_mixbatch_t* out);

/* Evaluate every replicate's mixture with the rule of vecchia_mixture_logcdf
 * (mix->n_nodes must equal the batch's): one batched search launch set, one
 * synchronisation of hip_stream, one batched node launch set, one wave per
 * replicate to combine. x_dev: the replicates' thresholds concatenated (plan t's
 * D_t values in its user order, device). cov_override: NULL or one covariance
 * for every plan (same family and nu). out_dev: n x {log G_t, se_t} (device);
 * total_dev (may be NULL): {sum_t log G_t, sqrt(sum_t se_t^2)} (device).
 * Replicate t's result equals vecchia_mixture_logcdf on its plan with seed
 * q->seed + t. Errors: INVALID, NOMEM, HIP; NOT_PD through vecchia_mixbatch_status. */
vecchia_status vecchia_mixbatch_logcdf(vecchia_mixbatch_t mb, const double* x_dev, const vecchia_mixture* mix,
                                       const vecchia_cov* cov_override, double* out_dev, double* total_dev,
                                       void* hip_stream);

/* Wait for the last call and report, per replicate, the first plan-order term
 * whose Cholesky failed in the node pass (-1 if none; n entries, may be NULL):
 * OK or NOT_PD. */
vecchia_status vecchia_mixbatch_status(vecchia_mixbatch_t mb, int64_t* bad_terms_host);

/* Wait for outstanding work and free the batch. */
vecchia_status vecchia_mixbatch_destroy(vecchia_mixbatch_t mb);

/* Full-dimension SOV estimate of log Phi_D(x / scale) on the plan's ordering
 * and covariance: Genz's separation of variables over all D variables with a
 * (D-1)-dimensional randomized lattice (the comparator the paper checks the
 * Vecchia approximation against, Section 3.1, Figures 1-4). Builds the dense
 * covariance and its Cholesky factor on the device (blocked, FP64), then
 * evaluates every lattice point's chain with its product kept as a sum of
 * log Phi. Lattice: Z_j from the first D-1 primes; the shift of dimension j in
 * replicate r is SplitMix64 output 2^63 + r 2^32 + j of q->seed.
 * out_dev = {log F, delta-method SE over the shifts} (device); NaN when the
 * covariance is not positive definite. q->precision must be VECCHIA_FP64 and
 * q->n_shifts at most 1024. Workspace D^2 + (D-1) N R doubles, kept in the
 * plan and grown on demand (at most 64 GB; D <= 40000). Asynchronous on
 * hip_stream. Errors: INVALID (censored plan, FP32, sizes), NOMEM, HIP. */
vecchia_status vecchia_full_logcdf(vecchia_plan_t plan, const double* x_dev, double scale,
                                   const vecchia_cov* cov_override, const vecchia_qmc* q, double* out_dev,
                                   void* hip_stream);

/* Launch-shape autotuner (the batched launch of Section 2.2, eq. (6): terms of
 * all instances that share K run in one launch, one wave per work item of
 * chunk_points lattice points of one shift of one term). For each K = ms[k]
 * (n_ms values, each in 1..VECCHIA_MAX_M) it builds a synthetic instance
 * through vecchia_plan (uniform points, coordinate ordering, Matern 3/2,
 * m = K, enough terms for two full rounds of waves), times that K's launch for
 * chunk sizes {256, 512, ..., 8192} (capped at n_points rounded up to 64) with
 * HIP events on hip_stream (median of three), and records the fastest for
 * (precision, K); instances whose plan has m = K use it from then on.
 * chunk_out / ms_out (may be NULL): n_ms entries, the chosen chunk and its
 * median launch time. Synchronises hip_stream; do not evaluate concurrently on
 * other threads. Results depend on the chunk size only through the FP64
 * grouping of partial sums. Errors: INVALID (bad precision, QMC sizes or m
 * list), NOMEM, HIP. */
vecchia_status vecchia_autotune(int32_t precision, int32_t n_points, int32_t n_shifts, const int32_t* ms,
                                int32_t n_ms, void* hip_stream, int32_t* chunk_out, float* ms_out);

/* Read or set the chunk size used for (precision, m); 0 means the built-in
 * default (2048 FP32, 512 FP64). A set value must be a multiple of 64 in
 * [64, 2^24]. Host-only. Errors: INVALID. */
vecchia_status vecchia_tuning_get(int32_t precision, int32_t m, int32_t* chunk_points);
vecchia_status vecchia_tuning_set(int32_t precision, int32_t m, int32_t chunk_points);

/* Measurement hook for the roofline: measured issue rates of the vector ALU on
 * the current device, in wave64 instructions per compute unit per nanosecond,
 * for a full-rate FP32 FMA and for v_exp_f32, v_log_f32, v_rcp_f32 and
 * v_sqrt_f32 (rates_out[0..4], host memory). Each rate comes from a kernel of
 * independent dependency chains over many waves per CU, timed with HIP events
 * on hip_stream (best of three). Synchronises hip_stream. Errors: INVALID
 * (rates_out NULL), HIP. */
vecchia_status vecchia_calibrate_valu(void* hip_stream, double* rates_out);

/* Test hooks: the device's own normal CDF and quantile pieces (Section 2.2's
 * univariate Phi and Phi^{-1} inside Genz's recursion), evaluated elementwise
 * so that tests pin them against library routines. in_dev: n doubles;
 * out_dev: n x 3 doubles {o0, o1, o2} (device). what:
 *   VECCHIA_PROBE_PHI_F32: the FP32 loop's factor at t = in: o0 = Phi(-|t|) as
 *     the main path forms it (2^(-v^2) R, v = kappa t in FP32), and the deep
 *     path's split o1 * 2^o2 of the same tail;
 *   VECCHIA_PROBE_NINV_F32: o0 = -Phi^{-1}(q) as the loop forms it from
 *     log2 q, q = in rounded to FP32 (0 < q <= 1/2), o1 = that q;
 *   VECCHIA_PROBE_NINV_LOG2_F32: o0 = -Phi^{-1}(2^in) from the FP32 log2 in
 *     (the split path, whose exponents reach -2^20);
 *   VECCHIA_PROBE_PHI_F64 / VECCHIA_PROBE_NINV_F64: o0 = the FP64 loop's
 *     normcdf(in) / normcdfinv(in).
 * Asynchronous on hip_stream. Errors: INVALID (unknown what, n outside
 * 0..2^30, null pointers), HIP. */
#define VECCHIA_PROBE_PHI_F32 0
#define VECCHIA_PROBE_NINV_F32 1
#define VECCHIA_PROBE_NINV_LOG2_F32 2
#define VECCHIA_PROBE_PHI_F64 3
#define VECCHIA_PROBE_NINV_F64 4
vecchia_status vecchia_probe_math(int32_t what, int64_t n, const double* in_dev, double* out_dev,
                                  void* hip_stream);

/* Test hook: the lattice coordinates p = 1..n of dimension dim (0..62) in
 * shift `shift` of plan-order term `term`, as the QMC kernels form them
 * (the randomized Richtmyer rule with its SplitMix64 shift; second = 1 for the
 * term's second lattice): w64_dev (n doubles, FP64 coordinates) and w32_dev
 * (n floats, FP32 coordinates), either may be NULL. Asynchronous on
 * hip_stream. Errors: INVALID (arguments out of range), HIP. */
vecchia_status vecchia_probe_lattice(uint64_t seed, int64_t term, int32_t shift, int32_t dim, int32_t second,
                                     int64_t n, double* w64_dev, float* w32_dev, void* hip_stream);

/* Serving: a request loop with continuous batching for the repeated log-CDF
 * evaluations of Section 4 (one Gaussian CDF per temporal replicate and per
 * scale-mixture node, eqs. (9)-(11), as a likelihood optimizer or an MCMC chain
 * issues them). The server reserves one device arena of hbm_budget_bytes and
 * max_slots execution slots (each a stream with two side streams). Whenever a
 * slot is free, a scheduler thread admits the queued requests in arrival order
 * as one group - as many as fit in the arena, up to 64 requests - and runs
 * them as one batch: one QMC launch per conditioning-set size over all of them.
 * Groups on different slots overlap on the device. A request's result is the
 * same alone and in any group. Errors: INVALID (budget 0, max_slots outside
 * 1..64), NOMEM, HIP. */
vecchia_status vecchia_server_create(size_t hbm_budget_bytes, int32_t max_slots, vecchia_server_t* out);

/* Queue one log-CDF request (the vecchia_logcdf of Section 2.2, eq. (6), at
 * thresholds x / scale, eq. (9)); returns at once with a ticket. The server
 * reads x_dev on its own streams, which are not ordered after the caller's:
 * x_dev must hold its final values when vecchia_submit is called (the stream
 * that wrote it synchronized) and stay unchanged until the request is done.
 * Errors: INVALID (bad arguments), NOMEM (the request alone exceeds the HBM
 * budget). */
vecchia_status vecchia_submit(vecchia_server_t server, vecchia_plan_t plan, const double* x_dev,
                              double scale, const vecchia_cov* cov_override, const vecchia_qmc* q,
                              uint64_t* ticket);

/* Result of a request (Section 2.2, eq. (6), with its Section 3.1 log-scale
 * sum). Non-blocking. *done = 1 and {log F, SE} when finished (the ticket is
 * then released), else *done = 0. latency_s (may be NULL): submit-to-completion
 * seconds, for the serving loop's latency figures. Errors: INVALID (unknown
 * ticket), NOT_PD (the request's covariance failed; the ticket is released). */
vecchia_status vecchia_poll(vecchia_server_t server, uint64_t ticket, double* logF, double* se,
                            int32_t* done, double* latency_s);

/* Stop the scheduler after queued and in-flight requests drain (the serving
 * loop of Section 4's repeated evaluations) and free the server. */
vecchia_status vecchia_server_destroy(vecchia_server_t server);

#ifdef __cplusplus
}
#endif
#endif /* VECCHIA_H */
