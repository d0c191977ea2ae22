// Gaussian scale mixture, the outer integral over the random scale R
// (Section 4, eqs. (7)-(9)): G(x) = int Phi_D(x / r) f_R(r) dr, with F_R from
// eq. (8) (beta > 0, or beta = 0 read as the Pareto law 1 - r^-gamma), r >= 1.
//
// With v = -log(1 - F_R(R)) ~ Exp(1), G = int_0^inf e^-v h(v) dv where
// h(v) = Phi_D(x / r(v)), r(v) = e^(v/gamma) (beta = 0) or
// (1 + beta v / gamma)^(1/beta), capped at 1e300. The rule has two passes:
//   1. log h at v = 0 and v = 1e-3 (one batched evaluation of the plan at two
//      scales) gives mu = 1 + max(0, -(log h(1e-3) - log h(0)) / 1e-3);
//   2. n-node Gauss-Laguerre in tau = mu v (one batched evaluation at the n
//      scales r(tau_k / mu)), G = sum_k w_k / mu e^(tau_k (1 - 1/mu)) h(tau_k / mu),
//      combined in log space on the device.
// Every node uses the call's seed (common random numbers). The rule is exact
// when log h is linear in v (for instance x = 0, where G = Phi_D(0)).
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

constexpr double kDelta = 1e-3;
constexpr double kRMax = 1e300;

double mixture_scale(double v, double beta, double gamma) {
  const double s = beta == 0.0 ? v / gamma : std::log1p(beta * v / gamma) / beta;
  return s >= std::log(kRMax) ? kRMax : std::exp(s);
}

// L_n(x) and L_n'(x) from the three-term recurrence
// (k + 1) L_{k+1} = (2k + 1 - x) L_k - k L_{k-1} and x L_n' = n (L_n - L_{n-1}).
void laguerre_eval(int n, double x, double* Ln, double* dLn) {
  double p0 = 1.0, p1 = 1.0 - x;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0 - x) * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *Ln = p1;
  *dLn = n * (p1 - p0) / x;
}

// Gauss-Laguerre rule for int_0^inf e^-t g(t) dt. Nodes: eigenvalues of the
// symmetric Jacobi matrix of the Laguerre recurrence (diagonal 2k + 1,
// off-diagonal k + 1; Golub-Welsch) by cyclic Jacobi rotations, then refined by
// Newton steps on L_n. Weights: 1 / (t_k L_n'(t_k)^2).
void laguerre_rule(int n, std::vector<double>* t, std::vector<double>* w) {
  std::vector<double> A((size_t)n * n, 0.0);
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int k = 0; k < n; ++k) {
    a(k, k) = 2.0 * k + 1.0;
    if (k + 1 < n) a(k, k + 1) = a(k + 1, k) = k + 1.0;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
    }
    if (off <= 1e-34 * diag) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = a(p, r) = c * arp - s * arq;
          a(r, q) = a(q, r) = s * arp + c * arq;
        }
        a(p, p) -= tt * apq;
        a(q, q) += tt * apq;
        a(p, q) = a(q, p) = 0.0;
      }
    }
  }
  t->resize(n);
  w->resize(n);
  for (int k = 0; k < n; ++k) (*t)[k] = a(k, k);
  std::sort(t->begin(), t->end());
  for (int k = 0; k < n; ++k) {
    double x = (*t)[k], L = 0.0, dL = 1.0;
    for (int it = 0; it < 4; ++it) {
      laguerre_eval(n, x, &L, &dL);
      x -= L / dL;
    }
    laguerre_eval(n, x, &L, &dL);
    (*t)[k] = x;
    (*w)[k] = 1.0 / (x * dL * dL);
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

void rule_for(const vecchia_mixture& m, double mu, double* scales, double* logw) {
  std::vector<double> t, w;
  laguerre_rule(m.n_nodes, &t, &w);
  for (int k = 0; k < m.n_nodes; ++k) {
    scales[k] = mixture_scale(t[k] / mu, m.beta, m.gamma);
    logw[k] = std::log(w[k]) - std::log(mu) + t[k] * (1.0 - 1.0 / mu);
  }
}

// The plan's cached batch of n instances of itself, rebuilt when the QMC
// settings or the tuned chunk change.
vecchia_status ensure_batch(vecchia_plan_s* P, std::unique_ptr<Batch>* slot, int n, const vecchia_qmc& q) {
  Batch* b = slot->get();
  if (b && b->n() == n && b->qmcs()[0].n_shifts == q.n_shifts && b->qmcs()[0].precision == q.precision &&
      b->qmcs()[0].n_points == q.n_points && b->chunk_points(0) == chunk_points_for(P->m, q.precision, q.n_points))
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

extern "C" {

vecchia_status vecchia_mixture_rule(const vecchia_mixture* mix, double mu, double* scales_out, double* logw_out) {
  using namespace vecchia;
  std::string why;
  if (!valid_mixture(mix, &why)) return set_error(VECCHIA_E_INVALID, why);
  if (!(std::isfinite(mu) && mu >= 1.0) || !scales_out || !logw_out)
    return set_error(VECCHIA_E_INVALID, "mu must be finite and >= 1; outputs must hold n_nodes values");
  rule_for(*mix, mu, scales_out, logw_out);
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
    hipError_t e = hipMalloc(&plan->d_mix, sizeof(double) * 2 * (2 + kMaxMixNodes));
    if (e != hipSuccess) {
      plan->d_mix = nullptr;
      return hip_error(e, "mixture buffer");
    }
  }
  const int n = mix->n_nodes;
  std::vector<vecchia_cov> covs;
  if (cov_override) covs.assign((size_t)std::max(2, n), *cov_override);
  std::vector<uint64_t> seeds((size_t)std::max(2, n), q->seed);
  // pass 1: log h at v = 0 and v = delta
  vecchia_status st = ensure_batch(plan, &plan->mix1, 2, *q);
  if (st != VECCHIA_OK) return st;
  const double sc1[2] = {1.0, mixture_scale(kDelta, mix->beta, mix->gamma)};
  st = plan->mix1->run(x_dev, sc1, cov_override ? covs.data() : nullptr, plan->d_mix, nullptr, seeds.data(), s);
  if (st != VECCHIA_OK) return st;
  double h[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(h, plan->d_mix, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "mixture first pass");
  double mu = 1.0 + std::max(0.0, -(h[2] - h[0]) / kDelta);
  if (!std::isfinite(mu)) mu = 1.0;   // a non-finite node value propagates through the combination
  // pass 2: the Laguerre nodes
  std::vector<double> scales(n);
  MixWeights mw{};
  mw.n = n;
  rule_for(*mix, mu, scales.data(), mw.logw);
  st = ensure_batch(plan, &plan->mix2, n, *q);
  if (st != VECCHIA_OK) return st;
  double* node_out = plan->d_mix + 4;
  st = plan->mix2->run(x_dev, scales.data(), cov_override ? covs.data() : nullptr, node_out, nullptr, seeds.data(),
                       s);
  if (st != VECCHIA_OK) return st;
  e = launch_mixture_combine(node_out, mw, out_dev, nodes_dev, s);
  if (e != hipSuccess) return hip_error(e, "mixture combination");
  return VECCHIA_OK;
}

}  // extern "C"
