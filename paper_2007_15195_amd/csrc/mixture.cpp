// Gaussian scale mixture, the outer integral over the random scale R
// (Section 4, eqs. (7)-(9) and (11)): G(x) = int h(r) f_R(r) dr over r >= 1, with
// F_R from eq. (8) (beta > 0, or beta = 0 read as the Pareto law 1 - r^-gamma)
// and h(r) the plan's Vecchia value at scale r (Phi_D(x / r) for a plain plan,
// the censored integrand L_r(x) of eq. (11) for a censored plan).
//
// With v = -log(1 - F_R(R)) ~ Exp(1), G = int_0^inf e^-v h(v) dv where
// r(v) = e^(v/gamma) (beta = 0) or (1 + beta v / gamma)^(1/beta), capped at
// 1e300. l(v) = log h(v) - v peaks at v = 0 for a plain CDF with positive
// thresholds and inside (0, inf) for a censored likelihood, so the rule has two
// batched passes:
//   1. search: l at v = 0 and v_j = 1e-4 (2e6)^((j-1)/22), j = 1..23, with
//      n_points / 16 lattice points (at least 64, a multiple of 64);
//   2. window [lo, hi]: the search points nearest the maximum on each side whose
//      l is more than 36 below it (else 0 and 200); n-point Gauss-Legendre on it,
//      in s = log v when lo > 0 and hi / lo > 8, else in v, at the full size,
//      combined in log space on the device.
// Every node uses the call's seed (common random numbers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"
#include "vecchia.h"

namespace vecchia {
namespace {

constexpr double kRMax = 1e300;
constexpr double kCut = 36.0;
constexpr double kLogSpan = 8.0;
constexpr double kVMax = 200.0;

double mixture_scale(double v, double beta, double gamma) {
  const double s = beta == 0.0 ? v / gamma : std::log1p(beta * v / gamma) / beta;
  return s >= std::log(kRMax) ? kRMax : std::exp(s);
}

double search_v(int j) { return j == 0 ? 0.0 : 1e-4 * std::pow(2e6, (j - 1) / 22.0); }

int search_points(int n_points) { return std::max(64, ((n_points / 16 + 63) / 64) * 64); }

// Gauss-Legendre nodes t_k (ascending) and weights on [-1, 1]: Newton on P_n from
// t = cos(pi (k + 3/4) / (n + 1/2)), P_n and P_n' by the three-term recurrence
// (j + 1) P_{j+1} = (2j + 1) t P_j - j P_{j-1} and (1 - t^2) P_n' = n (P_{n-1} - t P_n);
// w_k = 2 / ((1 - t_k^2) P_n'(t_k)^2).
void legendre_rule(int n, double* t, double* w) {
  for (int k = 0; k < n; ++k) {
    double x = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 1; j < n; ++j) {
        const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (p0 - x * p1) / (1.0 - x * x);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-16 * std::max(1.0, std::fabs(x))) break;
    }
    {
      double p0 = 1.0, p1 = x;
      for (int j = 1; j < n; ++j) {
        const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (p0 - x * p1) / (1.0 - x * x);
    }
    t[n - 1 - k] = x;
    w[n - 1 - k] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

bool valid_mixture(const vecchia_mixture* m, std::string* why) {
  if (!m) return *why = "mixture is NULL", false;
  if (!(std::isfinite(m->beta) && m->beta >= 0.0)) return *why = "beta must be finite and >= 0", false;
  if (!(std::isfinite(m->gamma) && m->gamma > 0.0)) return *why = "gamma must be finite and > 0", false;
  if (m->n_nodes < 1 || m->n_nodes > kMaxMixNodes) return *why = "n_nodes must be in 1..64", false;
  if (m->reserved != 0) return *why = "reserved must be 0", false;
  return true;
}

// Window of step 2 from the search values log h(v_j); a NaN value gives a NaN window.
void window_for(const double* search_logh, double* lo, double* hi) {
  double ell[kMixSearch];
  int j = 0;
  for (int i = 0; i < kMixSearch; ++i) {
    ell[i] = search_logh[i] - search_v(i);
    if (std::isnan(ell[i])) {
      *lo = *hi = std::nan("");
      return;
    }
    if (ell[i] > ell[j]) j = i;
  }
  const double top = ell[j];
  *lo = 0.0;
  *hi = kVMax;
  for (int i = j - 1; i >= 0; --i)
    if (ell[i] < top - kCut) {
      *lo = search_v(i);
      break;
    }
  for (int i = j + 1; i < kMixSearch; ++i)
    if (ell[i] < top - kCut) {
      *hi = search_v(i);
      break;
    }
}

void rule_for(const vecchia_mixture& m, double lo, double hi, double* v, double* scales, double* logw) {
  double t[kMaxMixNodes], w[kMaxMixNodes];
  legendre_rule(m.n_nodes, t, w);
  const bool logmap = lo > 0.0 && hi / lo > kLogSpan;
  const double a = logmap ? std::log(lo) : lo, b = logmap ? std::log(hi) : hi;
  for (int k = 0; k < m.n_nodes; ++k) {
    const double u = a + (b - a) * (t[k] + 1.0) / 2.0;
    const double vk = logmap ? std::exp(u) : u;
    v[k] = vk;
    scales[k] = mixture_scale(vk, m.beta, m.gamma);
    logw[k] = std::log(w[k] * (b - a) / 2.0) + (logmap ? u : 0.0) - vk;
  }
}

// The plan's cached batch of n instances of itself, rebuilt when the QMC
// settings or the tuned chunk change.
vecchia_status ensure_batch(vecchia_plan_s* P, std::unique_ptr<Batch>* slot, int n, const vecchia_qmc& q) {
  Batch* b = slot->get();
  if (b && b->n() == n && b->qmcs()[0].n_shifts == q.n_shifts && b->qmcs()[0].precision == q.precision &&
      b->qmcs()[0].n_points == q.n_points && b->qmcs()[0].flags == q.flags && b->chunk_points(0) == chunk_points_for(P->m, q.precision, q.n_points))
    return VECCHIA_OK;
  std::unique_ptr<Batch> nb;
  vecchia_status st = Batch::create(std::vector<vecchia_plan_s*>(n, P), std::vector<vecchia_qmc>(n, q), &nb);
  if (st != VECCHIA_OK) return st;
  nb->set_shared_x(true);
  *slot = std::move(nb);
  return VECCHIA_OK;
}

}  // namespace
}  // namespace vecchia

// Scale mixtures of many plans evaluated together (the censored likelihood of
// Section 4 sums log G_{I_t}(x_t) over replicates t): both passes of every
// replicate run as one batch each.
struct vecchia_mixbatch_s {
  std::vector<vecchia_plan_s*> plans;
  int n_nodes = 0;
  vecchia_qmc q{};
  int device = 0;
  std::unique_ptr<vecchia::Batch> search, nodes;
  double* d_search = nullptr;   // n x 24 x {log h, se}
  double* d_nodes = nullptr;    // n x n_nodes x {log h, se}
  double* d_logw = nullptr;     // n x n_nodes
  double* h_search = nullptr;   // pinned copy of d_search
  double* h_logw = nullptr;     // pinned staging of d_logw
  hipEvent_t logw_ev = nullptr; // the last upload of h_logw
  bool logw_used = false;
  std::vector<double> scales1, scales2;
  std::vector<uint64_t> seeds1, seeds2;
};

namespace {
void free_mixbatch(vecchia_mixbatch_s* m) {
  hipFree(m->d_search);
  hipFree(m->d_nodes);
  hipFree(m->d_logw);
  if (m->h_search) hipHostFree(m->h_search);
  if (m->h_logw) hipHostFree(m->h_logw);
  if (m->logw_ev) hipEventDestroy(m->logw_ev);
  delete m;
}
}  // namespace

extern "C" {

vecchia_status vecchia_mixture_search(const vecchia_mixture* mix, double* scales_out) {
  using namespace vecchia;
  std::string why;
  if (!valid_mixture(mix, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (!scales_out) return set_error(VECCHIA_E_INVALID, "scales_out must hold VECCHIA_MIX_SEARCH_NODES values");
  for (int j = 0; j < kMixSearch; ++j) scales_out[j] = mixture_scale(search_v(j), mix->beta, mix->gamma);
  return VECCHIA_OK;
}

vecchia_status vecchia_mixture_rule(const vecchia_mixture* mix, const double* search_logh, double* window_out,
                                    double* v_out, double* scales_out, double* logw_out) {
  using namespace vecchia;
  std::string why;
  if (!valid_mixture(mix, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (!search_logh || !window_out || !v_out || !scales_out || !logw_out)
    return set_error(VECCHIA_E_INVALID, "null pointer");
  double lo, hi;
  window_for(search_logh, &lo, &hi);
  window_out[0] = lo;
  window_out[1] = hi;
  if (std::isnan(lo)) return set_error(VECCHIA_E_INVALID, "a search value is NaN");
  rule_for(*mix, lo, hi, v_out, scales_out, logw_out);
  return VECCHIA_OK;
}

vecchia_status vecchia_mixture_logcdf(vecchia_plan_t plan, const double* x_dev, const vecchia_mixture* mix,
                                      const vecchia_cov* cov_override, const vecchia_qmc* q, double* out_dev,
                                      double* nodes_dev, void* hip_stream) {
  using namespace vecchia;
  if (!plan || !q || !x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::string why;
  if (!valid_mixture(mix, &why) || !valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::lock_guard<std::mutex> lk(plan->mu);
  if (!plan->d_mix) {
    hipError_t e = hipMalloc(&plan->d_mix, sizeof(double) * 2 * (kMixSearch + kMaxMixNodes));
    if (e != hipSuccess) {
      plan->d_mix = nullptr;
      return hip_error(e, "mixture buffer");
    }
  }
  const int n = mix->n_nodes;
  const int nmax = std::max(kMixSearch, n);
  std::vector<vecchia_cov> covs;
  if (cov_override) covs.assign((size_t)nmax, *cov_override);
  std::vector<uint64_t> seeds((size_t)nmax, q->seed);
  // pass 1: the search at n_points / 16
  vecchia_qmc qs = *q;
  qs.n_points = search_points(q->n_points);
  vecchia_status st = ensure_batch(plan, &plan->mix1, kMixSearch, qs);
  if (st != VECCHIA_OK) return st;
  double sc1[kMixSearch];
  for (int j = 0; j < kMixSearch; ++j) sc1[j] = mixture_scale(search_v(j), mix->beta, mix->gamma);
  st = plan->mix1->run(x_dev, sc1, cov_override ? covs.data() : nullptr, plan->d_mix, nullptr, seeds.data(), s);
  if (st != VECCHIA_OK) return st;
  double h[2 * kMixSearch];
  hipError_t e = hipMemcpyAsync(h, plan->d_mix, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "mixture search pass");
  double logh[kMixSearch];
  for (int j = 0; j < kMixSearch; ++j) logh[j] = h[2 * j];
  double lo, hi;
  window_for(logh, &lo, &hi);
  if (std::isnan(lo)) lo = 0.0, hi = kVMax;   // a NaN node value propagates through the combination
  // pass 2: Gauss-Legendre on the window
  double v[kMaxMixNodes], scales[kMaxMixNodes];
  MixWeights mw{};
  mw.n = n;
  rule_for(*mix, lo, hi, v, scales, mw.logw);
  st = ensure_batch(plan, &plan->mix2, n, *q);
  if (st != VECCHIA_OK) return st;
  double* node_out = plan->d_mix + 2 * kMixSearch;
  st = plan->mix2->run(x_dev, scales, cov_override ? covs.data() : nullptr, node_out, nullptr, seeds.data(), s);
  if (st != VECCHIA_OK) return st;
  e = launch_mixture_combine(node_out, mw, out_dev, nodes_dev, s);
  if (e != hipSuccess) return hip_error(e, "mixture combination");
  return VECCHIA_OK;
}

vecchia_status vecchia_mixbatch_create(const vecchia_plan_t* plans, int32_t n, int32_t n_nodes,
                                       const vecchia_qmc* q, vecchia_mixbatch_t* out) {
  using namespace vecchia;
  if (!plans || !q || !out || n < 1) return set_error(VECCHIA_E_INVALID, "bad mixture batch arguments");
  *out = nullptr;
  if (n_nodes < 1 || n_nodes > kMaxMixNodes) return set_error(VECCHIA_E_INVALID, "n_nodes must be in 1..64");
  std::string why;
  if (!valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  if ((int64_t)n * std::max(kMixSearch, n_nodes) > 0x7fffffffLL)
    return set_error(VECCHIA_E_INVALID, "too many plans");
  std::unique_ptr<vecchia_mixbatch_s, void (*)(vecchia_mixbatch_s*)> m(new (std::nothrow) vecchia_mixbatch_s(),
                                                                        free_mixbatch);
  if (!m) return set_error(VECCHIA_E_NOMEM, "host allocation");
  m->plans.assign(plans, plans + n);
  for (auto* P : m->plans)
    if (!P) return set_error(VECCHIA_E_INVALID, "null plan in mixture batch");
  m->n_nodes = n_nodes;
  m->q = *q;
  hipGetDevice(&m->device);
  vecchia_qmc qs = *q;
  qs.n_points = search_points(q->n_points);
  std::vector<vecchia_plan_s*> p1, p2;
  std::vector<vecchia_qmc> q1, q2;
  std::vector<int64_t> off1, off2;
  int64_t xo = 0;
  for (int t = 0; t < n; ++t) {
    for (int k = 0; k < kMixSearch; ++k) {
      p1.push_back(m->plans[t]);
      q1.push_back(qs);
      off1.push_back(xo);
      m->seeds1.push_back(q->seed + (uint64_t)t);
    }
    for (int k = 0; k < n_nodes; ++k) {
      p2.push_back(m->plans[t]);
      q2.push_back(*q);
      off2.push_back(xo);
      m->seeds2.push_back(q->seed + (uint64_t)t);
    }
    xo += m->plans[t]->D;
  }
  vecchia_status st = Batch::create(p1, q1, &m->search);
  if (st == VECCHIA_OK) st = Batch::create(p2, q2, &m->nodes);
  if (st != VECCHIA_OK) return st;
  m->search->set_x_offsets(off1);
  m->nodes->set_x_offsets(off2);
  m->scales1.resize(p1.size());
  m->scales2.resize(p2.size());
  const size_t n1 = (size_t)n * kMixSearch, n2 = (size_t)n * n_nodes;
  hipError_t e = hipMalloc(&m->d_search, sizeof(double) * 2 * n1);
  if (e == hipSuccess) e = hipMalloc(&m->d_nodes, sizeof(double) * 2 * n2);
  if (e == hipSuccess) e = hipMalloc(&m->d_logw, sizeof(double) * n2);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&m->h_search), sizeof(double) * 2 * n1);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&m->h_logw), sizeof(double) * n2);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->logw_ev, hipEventDisableTiming);
  if (e != hipSuccess) return hip_error(e, "mixture batch buffers");
  *out = m.release();
  return VECCHIA_OK;
}

vecchia_status vecchia_mixbatch_logcdf(vecchia_mixbatch_t mb, const double* x_dev, const vecchia_mixture* mix,
                                       const vecchia_cov* cov_override, double* out_dev, double* total_dev,
                                       void* hip_stream) {
  using namespace vecchia;
  if (!mb || !x_dev || !out_dev) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::string why;
  if (!valid_mixture(mix, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (mix->n_nodes != mb->n_nodes) return set_error(VECCHIA_E_INVALID, "n_nodes differs from the batch's");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int n = (int)mb->plans.size();
  const int nn = mb->n_nodes;
  std::vector<vecchia_cov> covs;
  if (cov_override) covs.assign(std::max(mb->scales1.size(), mb->scales2.size()), *cov_override);
  // pass 1: the search of every replicate
  for (int t = 0; t < n; ++t)
    for (int k = 0; k < kMixSearch; ++k)
      mb->scales1[(size_t)t * kMixSearch + k] = mixture_scale(search_v(k), mix->beta, mix->gamma);
  vecchia_status st = mb->search->run(x_dev, mb->scales1.data(), cov_override ? covs.data() : nullptr,
                                      mb->d_search, nullptr, mb->seeds1.data(), s);
  if (st != VECCHIA_OK) return st;
  const size_t n1 = (size_t)n * kMixSearch;
  hipError_t e = hipMemcpyAsync(mb->h_search, mb->d_search, sizeof(double) * 2 * n1, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "mixture batch search pass");
  // the rule of every replicate, once the previous call's weight upload (maybe
  // on another stream) has read the staging buffer
  if (mb->logw_used) e = hipEventSynchronize(mb->logw_ev);
  if (e != hipSuccess) return hip_error(e, "mixture batch staging wait");
  for (int t = 0; t < n; ++t) {
    double logh[kMixSearch];
    for (int k = 0; k < kMixSearch; ++k) logh[k] = mb->h_search[2 * ((size_t)t * kMixSearch + k)];
    double lo, hi;
    window_for(logh, &lo, &hi);
    if (std::isnan(lo)) lo = 0.0, hi = kVMax;
    double v[kMaxMixNodes];
    rule_for(*mix, lo, hi, v, mb->scales2.data() + (size_t)t * nn, mb->h_logw + (size_t)t * nn);
  }
  e = hipMemcpyAsync(mb->d_logw, mb->h_logw, sizeof(double) * (size_t)n * nn, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(mb->logw_ev, s);
  if (e != hipSuccess) return hip_error(e, "mixture batch weights");
  mb->logw_used = true;
  // pass 2: Gauss-Legendre nodes of every replicate, then one wave per replicate
  st = mb->nodes->run(x_dev, mb->scales2.data(), cov_override ? covs.data() : nullptr, mb->d_nodes, nullptr,
                      mb->seeds2.data(), s);
  if (st != VECCHIA_OK) return st;
  e = launch_mixture_combine_many(mb->d_nodes, mb->d_logw, nn, n, out_dev, total_dev, s);
  if (e != hipSuccess) return hip_error(e, "mixture batch combination");
  return VECCHIA_OK;
}

vecchia_status vecchia_mixbatch_status(vecchia_mixbatch_t mb, int64_t* bad_terms_host) {
  using namespace vecchia;
  if (!mb) return set_error(VECCHIA_E_INVALID, "null mixture batch");
  std::vector<int64_t> bad;
  vecchia_status st = mb->nodes->status(&bad);
  if (bad_terms_host) {
    const int n = (int)mb->plans.size();
    for (int t = 0; t < n; ++t) {
      int64_t b = -1;
      for (int k = 0; k < mb->n_nodes; ++k) {
        const int64_t v = bad[(size_t)t * mb->n_nodes + k];
        if (v >= 0 && (b < 0 || v < b)) b = v;
      }
      bad_terms_host[t] = b;
    }
  }
  return st;
}

vecchia_status vecchia_mixbatch_destroy(vecchia_mixbatch_t mb) {
  using namespace vecchia;
  if (!mb) return set_error(VECCHIA_E_INVALID, "null mixture batch");
  if (mb->nodes && mb->nodes->last_stream() != nullptr) hipStreamSynchronize(mb->nodes->last_stream());
  hipDeviceSynchronize();
  free_mixbatch(mb);
  return VECCHIA_OK;
}

}  // extern "C"
