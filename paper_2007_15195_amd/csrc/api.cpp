// C ABI entry points (include/vecchia.h): argument checks, plan construction
// (host ordering + GPU nearest-neighbour kernel) and the evaluation calls.
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host_order.h"
#include "runtime.h"

using namespace vecchia;

namespace vecchia {
const char* last_error_message();
}

namespace {

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
}

void free_plan_buffers(vecchia_plan_s* P) {
  for (int k = 0; k < 2; ++k) {
    if (P->replan_ev[k]) hipEventDestroy(P->replan_ev[k]);
    if (P->h_replan[k]) hipHostFree(P->h_replan[k]);
  }
  if (P->d_geo) {
    hipFree(P->d_geo);   // holds d_xs, d_ys and d_perm
  } else {
    hipFree(P->d_xs);
    hipFree(P->d_ys);
    hipFree(P->d_perm);
  }
  hipFree(P->d_cov);
  hipFree(P->d_nbr);
  hipFree(P->d_kcnt);
  hipFree(P->d_sovk);
  hipFree(P->d_bvar_off);
  hipFree(P->d_bvars);
  hipFree(P->d_split);
  hipFree(P->d_mix);
  hipFree(P->d_full);
  if (P->has_grid) {
    hipFree(P->grid.cell);
    hipFree(P->grid.start);
    hipFree(P->grid.cursor);
    hipFree(P->grid.gx);
    hipFree(P->grid.gy);
    hipFree(P->grid.gid);
  }
}

// Grid geometry over the bounding box of the plan-order points: about two
// points per cell, and a margin covering rounding in cell bounds.
void grid_geometry(const double* xs, const double* ys, int64_t D, KnnGrid* g) {
  double x0 = xs[0], x1 = xs[0], y0 = ys[0], y1 = ys[0];
  for (int64_t i = 1; i < D; ++i) {
    x0 = std::min(x0, xs[i]);
    x1 = std::max(x1, xs[i]);
    y0 = std::min(y0, ys[i]);
    y1 = std::max(y1, ys[i]);
  }
  g->G = (int32_t)std::max<int64_t>(1, (int64_t)std::sqrt((double)D / 2.0));
  g->x0 = x0;
  g->y0 = y0;
  g->wx = x1 > x0 ? (x1 - x0) / g->G : 1.0;
  g->wy = y1 > y0 ? (y1 - y0) / g->G : 1.0;
  const double mag = std::max(std::max(std::fabs(x0), std::fabs(x1)), std::max(std::fabs(y0), std::fabs(y1))) +
                     g->G * std::max(g->wx, g->wy);
  g->margin = 16.0 * std::numeric_limits<double>::epsilon() * mag;
}

hipError_t alloc_grid(vecchia_plan_s* P) {
  const int64_t D = P->D;
  KnnGrid& g = P->grid;
  g.G = (int32_t)std::max<int64_t>(1, (int64_t)std::sqrt((double)D / 2.0));
  const int64_t cells = (int64_t)g.G * g.G;
  P->has_grid = true;
  hipError_t e = dev_alloc(&g.cell, D);
  if (e == hipSuccess) e = dev_alloc(&g.start, cells + 1);
  if (e == hipSuccess) e = dev_alloc(&g.cursor, cells);
  if (e == hipSuccess) e = dev_alloc(&g.gx, D);
  if (e == hipSuccess) e = dev_alloc(&g.gy, D);
  if (e == hipSuccess) e = dev_alloc(&g.gid, D);
  return e;
}

// SOV dimension of each term of a censored plan: 0 for an uncensored site (its
// term is a conditional density), else the number of censored neighbours (the
// uncensored ones are conditioned on by equality and add no dimension).
void set_sov_dims(vecchia_plan_s* P, const std::vector<int32_t>& nbr) {
  P->sovk.assign(P->D, 0);
  for (int64_t i = P->n_obs; i < P->D; ++i) {
    int c = 0;
    for (int a = 0; a < P->kcnt[i]; ++a) c += nbr[(size_t)i * P->m + a] >= P->n_obs;
    P->sovk[i] = c;
  }
}

// Joint terms of a block plan (groups of p consecutive plan positions): the
// conditioning set of group g is the union of its members' neighbour rows (each
// already limited to positions before the group), in member order, first
// occurrence kept; the term's variables are that set then the group.
void set_block_terms(vecchia_plan_s* P, int32_t p, const std::vector<int32_t>& nbr) {
  const int64_t D = P->D;
  P->block = p;
  P->n_terms = (D + p - 1) / p;
  P->bvar_off.assign(1, 0);
  P->bvars.clear();
  P->split.clear();
  P->sovk.clear();
  P->block_nv = 0;
  for (int64_t g0 = 0; g0 < D; g0 += p) {
    const int64_t g1 = std::min<int64_t>(D, g0 + p);
    std::vector<int32_t> cond;
    for (int64_t i = g0; i < g1; ++i)
      for (int a = 0; a < P->kcnt[i]; ++a) {
        const int32_t j = nbr[(size_t)i * P->m + a];
        if (std::find(cond.begin(), cond.end(), j) == cond.end()) cond.push_back(j);
      }
    const int nv = (int)(cond.size() + (g1 - g0));
    for (int32_t j : cond) P->bvars.push_back(j);
    for (int64_t i = g0; i < g1; ++i) P->bvars.push_back((int32_t)i);
    P->bvar_off.push_back((int32_t)P->bvars.size());
    P->split.push_back((int32_t)cond.size());
    P->sovk.push_back(nv - 1);
    P->block_nv = std::max(P->block_nv, nv);
  }
}

hipError_t upload_block_terms(vecchia_plan_s* P, hipStream_t s) {
  const int64_t T = P->n_terms;
  hipError_t e = dev_alloc(&P->d_bvar_off, T + 1);
  if (e == hipSuccess) e = dev_alloc(&P->d_bvars, P->bvars.size());
  if (e == hipSuccess) e = dev_alloc(&P->d_split, T);
  if (e == hipSuccess) e = dev_alloc(&P->d_sovk, T);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->d_bvar_off, P->bvar_off.data(), sizeof(int32_t) * (T + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->d_bvars, P->bvars.data(), sizeof(int32_t) * P->bvars.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->d_split, P->split.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_sovk, P->sovk.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

vecchia_status order_impl(const double* locs, int64_t D, int32_t ordering, const int64_t* perm_in,
                          int64_t* perm_out) {
  if (!locs || !perm_out) return set_error(VECCHIA_E_INVALID, "null pointer");
  if (D < 1 || D > 0x7fffffffLL) return set_error(VECCHIA_E_INVALID, "D must be in 1..2^31-1");
  for (int64_t j = 0; j < 2 * D; ++j)
    if (!std::isfinite(locs[j])) return set_error(VECCHIA_E_INVALID, "non-finite location");
  switch (ordering) {
    case VECCHIA_ORDER_COORD:
      order_coord(locs, D, perm_out);
      return VECCHIA_OK;
    case VECCHIA_ORDER_MAXMIN:
      order_maxmin(locs, D, perm_out);
      return VECCHIA_OK;
    case VECCHIA_ORDER_GIVEN: {
      if (!perm_in) return set_error(VECCHIA_E_INVALID, "VECCHIA_ORDER_GIVEN needs a permutation");
      std::vector<char> seen(D, 0);
      for (int64_t i = 0; i < D; ++i) {
        const int64_t v = perm_in[i];
        if (v < 0 || v >= D || seen[v]) return set_error(VECCHIA_E_INVALID, "given ordering is not a permutation");
        seen[v] = 1;
        perm_out[i] = v;
      }
      return VECCHIA_OK;
    }
    default:
      return set_error(VECCHIA_E_INVALID, "unknown ordering");
  }
}

}  // namespace

extern "C" {

const char* vecchia_last_error(void) { return last_error_message(); }

vecchia_status vecchia_order(const double* locs_host, int64_t D, int32_t ordering,
                             const int64_t* perm_in_host, int64_t* perm_out_host) {
  return order_impl(locs_host, D, ordering, perm_in_host, perm_out_host);
}

}  // extern "C"

namespace {

// Geometry plan for the plan-order permutation perm (D entries) whose first
// n_obs positions are uncensored sites (0 for a plain plan): copies the
// locations, finds the neighbours on the device and records the host copies of
// k_i and of the SOV dimension of each term.
vecchia_status build_geometry_plan(const double* locs_host, int64_t D, std::vector<int64_t> perm, int64_t n_obs,
                                   int32_t m, const vecchia_cov* cov, void* hip_stream, vecchia_plan_t* out,
                                   int32_t group = 1) {
  auto* P = new (std::nothrow) vecchia_plan_s();
  if (!P) return set_error(VECCHIA_E_NOMEM, "host allocation");
  hipGetDevice(&P->device);
  P->D = D;
  P->m = m;
  P->cov = *cov;
  P->perm = std::move(perm);
  P->n_obs = n_obs;
  P->n_terms = D;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // {xs, ys, perm} packed as the device block (and the replan staging)
  const size_t geo_bytes = (sizeof(double) * 2 + sizeof(int32_t)) * (size_t)D;
  std::vector<char> geo(geo_bytes);
  double* hx = reinterpret_cast<double*>(geo.data());
  double* hy = hx + D;
  int32_t* hp = reinterpret_cast<int32_t*>(hy + D);
  for (int64_t i = 0; i < D; ++i) {
    hx[i] = locs_host[2 * P->perm[i]];
    hy[i] = locs_host[2 * P->perm[i] + 1];
    hp[i] = (int32_t)P->perm[i];
  }
  hipError_t e = hipMalloc(&P->d_geo, geo_bytes);
  if (e == hipSuccess) {
    P->d_xs = static_cast<double*>(P->d_geo);
    P->d_ys = P->d_xs + D;
    P->d_perm = reinterpret_cast<int32_t*>(P->d_ys + D);
  }
  if (e == hipSuccess) e = dev_alloc(&P->d_kcnt, D);
  if (e == hipSuccess && n_obs > 0) e = dev_alloc(&P->d_sovk, D);
  if (e == hipSuccess && m > 0) e = dev_alloc(&P->d_nbr, (size_t)D * m);
  if (e == hipSuccess && m > 0 && D > kKnnGridMinD && group == 1) {
    e = alloc_grid(P);
    grid_geometry(hx, hy, D, &P->grid);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_geo, geo.data(), geo_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_knn(P->d_xs, P->d_ys, D, m, P->d_nbr, P->d_kcnt, P->has_grid ? &P->grid : nullptr, s, group);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    P->kcnt.resize(D);
    e = hipMemcpy(P->kcnt.data(), P->d_kcnt, sizeof(int32_t) * D, hipMemcpyDeviceToHost);
  }
  if (e == hipSuccess && group > 1) {
    std::vector<int32_t> nbr((size_t)D * m);
    if (m > 0) e = hipMemcpy(nbr.data(), P->d_nbr, sizeof(int32_t) * D * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      set_block_terms(P, group, nbr);
      e = upload_block_terms(P, s);
    }
  }
  if (e == hipSuccess && n_obs > 0) {
    std::vector<int32_t> nbr((size_t)D * m);
    if (m > 0) e = hipMemcpy(nbr.data(), P->d_nbr, sizeof(int32_t) * D * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      set_sov_dims(P, nbr);
      e = hipMemcpy(P->d_sovk, P->sovk.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice);
    }
  }
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipHostMalloc(reinterpret_cast<void**>(&P->h_replan[k]), (2 * sizeof(double) + sizeof(int32_t)) * D,
                      hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->replan_ev[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    free_plan_buffers(P);
    delete P;
    return hip_error(e, "plan construction");
  }
  *out = P;
  return VECCHIA_OK;
}

vecchia_status check_plan_args(int32_t dim, int32_t m, const vecchia_cov* cov, vecchia_plan_t* out) {
  if (!out || !cov) return set_error(VECCHIA_E_INVALID, "null pointer");
  *out = nullptr;
  if (dim != 2) return set_error(VECCHIA_E_INVALID, "only 2-D locations are supported (dim must be 2)");
  if (m < 0 || m > VECCHIA_MAX_M) return set_error(VECCHIA_E_INVALID, "m must be in 0..63");
  std::string why;
  if (!valid_cov(*cov, &why)) return set_error(VECCHIA_E_INVALID, why);
  return VECCHIA_OK;
}

}  // namespace

extern "C" {

vecchia_status vecchia_plan(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                            const int64_t* perm_in_host, int32_t m, const vecchia_cov* cov,
                            void* hip_stream, vecchia_plan_t* out) {
  vecchia_status st = check_plan_args(dim, m, cov, out);
  if (st != VECCHIA_OK) return st;
  std::vector<int64_t> perm(D > 0 && D <= 0x7fffffffLL ? D : 0);
  st = order_impl(locs_host, D, ordering, perm_in_host, perm.data());
  if (st != VECCHIA_OK) return st;
  return build_geometry_plan(locs_host, D, std::move(perm), 0, m, cov, hip_stream, out);
}

vecchia_status vecchia_plan_censored(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                                     const int64_t* perm_in_host, const uint8_t* observed_host, int32_t m,
                                     const vecchia_cov* cov, void* hip_stream, vecchia_plan_t* out) {
  vecchia_status st = check_plan_args(dim, m, cov, out);
  if (st != VECCHIA_OK) return st;
  if (!observed_host) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::vector<int64_t> base(D > 0 && D <= 0x7fffffffLL ? D : 0);
  st = order_impl(locs_host, D, ordering, perm_in_host, base.data());
  if (st != VECCHIA_OK) return st;
  for (int64_t u = 0; u < D; ++u)
    if (observed_host[u] > 1) return set_error(VECCHIA_E_INVALID, "observed flags must be 0 or 1");
  std::vector<int64_t> perm;
  perm.reserve(D);
  for (int64_t i = 0; i < D; ++i)
    if (observed_host[base[i]]) perm.push_back(base[i]);
  const int64_t n_obs = (int64_t)perm.size();
  for (int64_t i = 0; i < D; ++i)
    if (!observed_host[base[i]]) perm.push_back(base[i]);
  return build_geometry_plan(locs_host, D, std::move(perm), n_obs, m, cov, hip_stream, out);
}

static vecchia_status plan_from_cov_impl(const double* cov_host, int64_t D, const int32_t* nbr_host, int32_t m,
                                         int64_t n_obs, void* hip_stream, vecchia_plan_t* out) {
  if (!out || !cov_host) return set_error(VECCHIA_E_INVALID, "null pointer");
  *out = nullptr;
  if (D < 1 || D > 4096) return set_error(VECCHIA_E_INVALID, "D must be in 1..4096");
  if (n_obs < 0 || n_obs > D) return set_error(VECCHIA_E_INVALID, "n_observed must be in 0..D");
  if (m < 0 || m > VECCHIA_MAX_M) return set_error(VECCHIA_E_INVALID, "m must be in 0..63");
  for (int64_t a = 0; a < D; ++a)
    for (int64_t b = 0; b < D; ++b) {
      const double v = cov_host[a * D + b];
      if (!std::isfinite(v)) return set_error(VECCHIA_E_INVALID, "non-finite covariance entry");
      if (v != cov_host[b * D + a]) return set_error(VECCHIA_E_INVALID, "covariance matrix is not symmetric");
    }
  std::vector<int32_t> nbr((size_t)D * m, -1), kc(D, 0);
  for (int64_t i = 0; i < D; ++i) {
    if (nbr_host) {
      int k = 0;
      while (k < m && nbr_host[i * m + k] >= 0) ++k;
      for (int c = k; c < m; ++c)
        if (nbr_host[i * m + c] != -1) return set_error(VECCHIA_E_INVALID, "neighbour rows must be -1 padded at the end");
      for (int c = 0; c < k; ++c) {
        const int32_t v = nbr_host[i * m + c];
        if (v >= i) return set_error(VECCHIA_E_INVALID, "neighbour " + std::to_string(v) + " of row " + std::to_string(i) + " does not precede it");
        for (int c2 = 0; c2 < c; ++c2)
          if (nbr_host[i * m + c2] == v) return set_error(VECCHIA_E_INVALID, "repeated neighbour");
        nbr[i * m + c] = v;
      }
      kc[i] = k;
    } else {
      const int k = (int)(i < m ? i : m);
      for (int c = 0; c < k; ++c) nbr[i * m + c] = (int32_t)(i - k + c);
      kc[i] = k;
    }
  }
  auto* P = new (std::nothrow) vecchia_plan_s();
  if (!P) return set_error(VECCHIA_E_NOMEM, "host allocation");
  hipGetDevice(&P->device);
  P->D = D;
  P->m = m;
  P->matrix = true;
  P->n_obs = n_obs;
  P->cov = vecchia_cov{VECCHIA_COV_EXPONENTIAL, 0, 0.5, 1.0, 1.0, 0.0};
  P->perm.resize(D);
  P->kcnt = kc;
  if (n_obs > 0) set_sov_dims(P, nbr);   // reads kcnt
  std::vector<int32_t> hp(D);
  for (int64_t i = 0; i < D; ++i) {
    P->perm[i] = i;
    hp[i] = (int32_t)i;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = dev_alloc(&P->d_cov, (size_t)D * D);
  if (e == hipSuccess) e = dev_alloc(&P->d_perm, D);
  if (e == hipSuccess) e = dev_alloc(&P->d_kcnt, D);
  if (e == hipSuccess && m > 0) e = dev_alloc(&P->d_nbr, (size_t)D * m);
  if (e == hipSuccess && n_obs > 0) e = dev_alloc(&P->d_sovk, D);
  if (e == hipSuccess && n_obs > 0)
    e = hipMemcpyAsync(P->d_sovk, P->sovk.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_cov, cov_host, sizeof(double) * D * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_perm, hp.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_kcnt, kc.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m > 0)
    e = hipMemcpyAsync(P->d_nbr, nbr.data(), sizeof(int32_t) * D * m, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_plan_buffers(P);
    delete P;
    return hip_error(e, "plan construction");
  }
  *out = P;
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_from_cov(const double* cov_host, int64_t D, const int32_t* nbr_host,
                                     int32_t m, void* hip_stream, vecchia_plan_t* out) {
  return plan_from_cov_impl(cov_host, D, nbr_host, m, 0, hip_stream, out);
}

vecchia_status vecchia_plan_block(const double* locs_host, int64_t D, int32_t dim, int32_t ordering,
                                  const int64_t* perm_in_host, int32_t m, int32_t p, const vecchia_cov* cov,
                                  void* hip_stream, vecchia_plan_t* out) {
  vecchia_status st = check_plan_args(dim, m, cov, out);
  if (st != VECCHIA_OK) return st;
  if (p < 1 || (int64_t)p * (m + 1) > kMaxVars)
    return set_error(VECCHIA_E_INVALID, "groups need 1 <= p and p (m + 1) <= 64 variables per term");
  std::vector<int64_t> perm(D > 0 && D <= 0x7fffffffLL ? D : 0);
  st = order_impl(locs_host, D, ordering, perm_in_host, perm.data());
  if (st != VECCHIA_OK) return st;
  return build_geometry_plan(locs_host, D, std::move(perm), 0, m, cov, hip_stream, out, p);
}

vecchia_status vecchia_plan_block_terms(vecchia_plan_t plan, int64_t* n_terms, int32_t* var_off_host,
                                        int32_t* vars_host, int32_t* split_host) {
  if (!plan || !n_terms) return set_error(VECCHIA_E_INVALID, "null pointer");
  if (plan->block <= 0) return set_error(VECCHIA_E_INVALID, "not a block plan");
  *n_terms = plan->n_terms;
  if (var_off_host) std::memcpy(var_off_host, plan->bvar_off.data(), sizeof(int32_t) * (plan->n_terms + 1));
  if (vars_host) std::memcpy(vars_host, plan->bvars.data(), sizeof(int32_t) * plan->bvars.size());
  if (split_host) std::memcpy(split_host, plan->split.data(), sizeof(int32_t) * plan->n_terms);
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_from_cov_block(const double* cov_host, int64_t D, const int32_t* var_off_host,
                                           const int32_t* vars_host, const int32_t* split_host, int64_t n_terms,
                                           void* hip_stream, vecchia_plan_t* out) {
  if (!out || !cov_host || !var_off_host || !vars_host || !split_host)
    return set_error(VECCHIA_E_INVALID, "null pointer");
  *out = nullptr;
  if (D < 1 || D > 4096) return set_error(VECCHIA_E_INVALID, "D must be in 1..4096");
  if (n_terms < 1 || n_terms > 1000000) return set_error(VECCHIA_E_INVALID, "n_terms must be in 1..10^6");
  for (int64_t a = 0; a < D; ++a)
    for (int64_t b = 0; b < D; ++b) {
      const double v = cov_host[a * D + b];
      if (!std::isfinite(v)) return set_error(VECCHIA_E_INVALID, "non-finite covariance entry");
      if (v != cov_host[b * D + a]) return set_error(VECCHIA_E_INVALID, "covariance matrix is not symmetric");
    }
  if (var_off_host[0] != 0) return set_error(VECCHIA_E_INVALID, "var_off[0] must be 0");
  int nv_max = 0;
  for (int64_t g = 0; g < n_terms; ++g) {
    const int nv = var_off_host[g + 1] - var_off_host[g];
    if (nv < 1 || nv > kMaxVars) return set_error(VECCHIA_E_INVALID, "every term needs 1..64 variables");
    if (split_host[g] < 0 || split_host[g] >= nv)
      return set_error(VECCHIA_E_INVALID, "split must be in 0..(variables - 1)");
    for (int c = 0; c < nv; ++c) {
      const int32_t v = vars_host[var_off_host[g] + c];
      if (v < 0 || v >= D) return set_error(VECCHIA_E_INVALID, "variable index out of range");
      for (int c2 = 0; c2 < c; ++c2)
        if (vars_host[var_off_host[g] + c2] == v) return set_error(VECCHIA_E_INVALID, "repeated variable in a term");
    }
    nv_max = std::max(nv_max, nv);
  }
  auto* P = new (std::nothrow) vecchia_plan_s();
  if (!P) return set_error(VECCHIA_E_NOMEM, "host allocation");
  hipGetDevice(&P->device);
  P->D = D;
  P->m = 0;
  P->matrix = true;
  P->cov = vecchia_cov{VECCHIA_COV_EXPONENTIAL, 0, 0.5, 1.0, 1.0, 0.0};
  P->perm.resize(D);
  P->kcnt.assign(D, 0);
  P->block = 1 << 30;   // explicit terms: no group size
  P->n_terms = n_terms;
  P->bvar_off.assign(var_off_host, var_off_host + n_terms + 1);
  P->bvars.assign(vars_host, vars_host + var_off_host[n_terms]);
  P->split.assign(split_host, split_host + n_terms);
  P->sovk.resize(n_terms);
  for (int64_t g = 0; g < n_terms; ++g) P->sovk[g] = var_off_host[g + 1] - var_off_host[g] - 1;
  P->block_nv = nv_max;
  std::vector<int32_t> hp(D);
  for (int64_t i = 0; i < D; ++i) {
    P->perm[i] = i;
    hp[i] = (int32_t)i;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = dev_alloc(&P->d_cov, (size_t)D * D);
  if (e == hipSuccess) e = dev_alloc(&P->d_perm, D);
  if (e == hipSuccess) e = dev_alloc(&P->d_kcnt, D);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_cov, cov_host, sizeof(double) * D * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_perm, hp.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->d_kcnt, P->kcnt.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = upload_block_terms(P, s);
  if (e != hipSuccess) {
    free_plan_buffers(P);
    delete P;
    return hip_error(e, "plan construction");
  }
  *out = P;
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_from_cov_censored(const double* cov_host, int64_t D, const int32_t* nbr_host,
                                              int32_t m, int64_t n_observed, void* hip_stream,
                                              vecchia_plan_t* out) {
  return plan_from_cov_impl(cov_host, D, nbr_host, m, n_observed, hip_stream, out);
}

vecchia_status vecchia_plan_censoring(vecchia_plan_t plan, int64_t* n_observed) {
  if (!plan || !n_observed) return set_error(VECCHIA_E_INVALID, "null pointer");
  *n_observed = plan->n_obs;
  return VECCHIA_OK;
}

vecchia_status vecchia_replan(vecchia_plan_t plan, const double* locs_host, int32_t ordering,
                              const int64_t* perm_in_host, void* hip_stream) {
  if (!plan) return set_error(VECCHIA_E_INVALID, "null plan");
  if (plan->matrix) return set_error(VECCHIA_E_INVALID, "a matrix plan has no locations to re-plan");
  if (plan->n_obs > 0)
    return set_error(VECCHIA_E_INVALID, "a censored plan belongs to one replicate; build a new one");
  if (plan->block > 0) return set_error(VECCHIA_E_INVALID, "a block plan is not re-planned in place; build a new one");
  std::lock_guard<std::mutex> lk(plan->mu);
  if (plan->inflight.load() > 0) return set_error(VECCHIA_E_BUSY, "plan has requests in flight");
  const int64_t D = plan->D;
  std::vector<int64_t> perm(D);
  vecchia_status st = order_impl(locs_host, D, ordering, perm_in_host, perm.data());
  if (st != VECCHIA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int k = plan->replan_next;
  plan->replan_next ^= 1;
  hipError_t e = hipSuccess;
  if (plan->replan_used[k]) e = hipEventSynchronize(plan->replan_ev[k]);
  if (e != hipSuccess) return hip_error(e, "replan staging wait");
  double* hx = reinterpret_cast<double*>(plan->h_replan[k]);
  double* hy = hx + D;
  int32_t* hp = reinterpret_cast<int32_t*>(hy + D);
  for (int64_t i = 0; i < D; ++i) {
    hx[i] = locs_host[2 * perm[i]];
    hy[i] = locs_host[2 * perm[i] + 1];
    hp[i] = (int32_t)perm[i];
  }
  // the staging block has the device block's layout: one copy
  e = hipMemcpyAsync(plan->d_geo, hx, (sizeof(double) * 2 + sizeof(int32_t)) * (size_t)D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(plan->replan_ev[k], s);
  if (plan->has_grid) grid_geometry(hx, hy, D, &plan->grid);
  if (e == hipSuccess)
    e = launch_knn(plan->d_xs, plan->d_ys, D, plan->m, plan->d_nbr, plan->d_kcnt,
                   plan->has_grid ? &plan->grid : nullptr, s);
  if (e != hipSuccess) return hip_error(e, "replan");
  plan->replan_used[k] = true;
  plan->perm = std::move(perm);   // k_i = min(m, i) is unchanged
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_info(vecchia_plan_t plan, int64_t* D, int32_t* m) {
  if (!plan) return set_error(VECCHIA_E_INVALID, "null plan");
  if (D) *D = plan->D;
  if (m) *m = plan->m;
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_neighbours(vecchia_plan_t plan, int64_t* perm_host, int32_t* nbr_host) {
  if (!plan) return set_error(VECCHIA_E_INVALID, "null plan");
  if (perm_host) std::memcpy(perm_host, plan->perm.data(), sizeof(int64_t) * plan->D);
  if (nbr_host && plan->m > 0) {
    hipError_t e = hipMemcpy(nbr_host, plan->d_nbr, sizeof(int32_t) * plan->D * plan->m, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_error(e, "neighbour copy");
  }
  return VECCHIA_OK;
}

vecchia_status vecchia_logcdf(vecchia_plan_t plan, const double* x_dev, double scale,
                              const vecchia_cov* cov_override, const vecchia_qmc* q,
                              double* out_dev, double* terms_dev, void* hip_stream) {
  if (!plan || !q) return set_error(VECCHIA_E_INVALID, "null pointer");
  std::string why;
  if (!valid_qmc(*q, &why)) return set_error(VECCHIA_E_INVALID, why);
  std::lock_guard<std::mutex> lk(plan->mu);
  Batch* b = plan->single.get();
  if (!b || b->qmcs()[0].n_shifts != q->n_shifts || b->qmcs()[0].precision != q->precision ||
      b->qmcs()[0].n_points != q->n_points || b->qmcs()[0].flags != q->flags ||
      b->chunk_points(0) != chunk_points_for(plan->m, q->precision, q->n_points)) {
    std::unique_ptr<Batch> nb;
    vecchia_status st = Batch::create({plan}, {*q}, &nb);
    if (st != VECCHIA_OK) return st;
    plan->single = std::move(nb);
    b = plan->single.get();
  }
  const uint64_t seed = q->seed;
  return b->run(x_dev, &scale, cov_override, out_dev, terms_dev, &seed, static_cast<hipStream_t>(hip_stream));
}

vecchia_status vecchia_plan_status(vecchia_plan_t plan, int64_t* bad_term) {
  if (!plan) return set_error(VECCHIA_E_INVALID, "null plan");
  if (bad_term) *bad_term = -1;
  std::lock_guard<std::mutex> lk(plan->mu);
  // the first NOT_PD report of the plan's evaluation batches (single call, then
  // the scale-mixture passes)
  for (Batch* b : {plan->single.get(), plan->mix1.get(), plan->mix2.get()}) {
    if (!b) continue;
    std::vector<int64_t> bad;
    vecchia_status st = b->status(&bad);
    if (st == VECCHIA_E_NOT_PD) {
      for (int64_t v : bad)
        if (v >= 0) {
          if (bad_term) *bad_term = v;
          break;
        }
      return st;
    }
    if (st != VECCHIA_OK) return st;
  }
  return VECCHIA_OK;
}

vecchia_status vecchia_plan_destroy(vecchia_plan_t plan) {
  if (!plan) return set_error(VECCHIA_E_INVALID, "null plan");
  if (plan->inflight.load() > 0) return set_error(VECCHIA_E_BUSY, "plan has requests in flight");
  if (plan->single && plan->single->last_stream() != nullptr) hipStreamSynchronize(plan->single->last_stream());
  hipDeviceSynchronize();
  plan->single.reset();
  plan->mix1.reset();
  plan->mix2.reset();
  free_plan_buffers(plan);
  delete plan;
  return VECCHIA_OK;
}

vecchia_status vecchia_batch_create(const vecchia_plan_t* plans, int32_t n, const vecchia_qmc* qmcs,
                                    vecchia_batch_t* out) {
  if (!plans || !qmcs || !out || n < 1) return set_error(VECCHIA_E_INVALID, "bad batch arguments");
  *out = nullptr;
  std::vector<vecchia_plan_s*> ps(plans, plans + n);
  std::vector<vecchia_qmc> qs(qmcs, qmcs + n);
  std::unique_ptr<Batch> b;
  vecchia_status st = Batch::create(ps, qs, &b);
  if (st != VECCHIA_OK) return st;
  auto* h = new (std::nothrow) vecchia_batch_s();
  if (!h) return set_error(VECCHIA_E_NOMEM, "host allocation");
  h->b = std::move(b);
  *out = h;
  return VECCHIA_OK;
}

vecchia_status vecchia_batch_logcdf(vecchia_batch_t batch, const double* x_dev, const double* scales_host,
                                    const vecchia_cov* covs_host, double* out_dev, void* hip_stream) {
  if (!batch) return set_error(VECCHIA_E_INVALID, "null batch");
  return batch->b->run(x_dev, scales_host, covs_host, out_dev, nullptr, nullptr,
                       static_cast<hipStream_t>(hip_stream));
}

vecchia_status vecchia_batch_status(vecchia_batch_t batch, int64_t* bad_terms_host) {
  if (!batch) return set_error(VECCHIA_E_INVALID, "null batch");
  std::vector<int64_t> bad;
  vecchia_status st = batch->b->status(&bad);
  if (bad_terms_host) std::memcpy(bad_terms_host, bad.data(), sizeof(int64_t) * bad.size());
  return st;
}

vecchia_status vecchia_batch_destroy(vecchia_batch_t batch) {
  if (!batch) return set_error(VECCHIA_E_INVALID, "null batch");
  if (batch->b && batch->b->last_stream() != nullptr) hipStreamSynchronize(batch->b->last_stream());
  hipDeviceSynchronize();
  delete batch;
  return VECCHIA_OK;
}

vecchia_status vecchia_map_anisotropic(const double* locs_host, int64_t D, double phi, double A,
                                       double* out_host) {
  if (!locs_host || !out_host) return set_error(VECCHIA_E_INVALID, "null pointer");
  if (D < 0) return set_error(VECCHIA_E_INVALID, "D must be >= 0");
  if (!std::isfinite(phi) || !(std::isfinite(A) && A > 0.0))
    return set_error(VECCHIA_E_INVALID, "phi must be finite and A finite and > 0");
  const double c = std::cos(phi), sn = std::sin(phi);
  for (int64_t i = 0; i < D; ++i) {
    const double x = locs_host[2 * i], y = locs_host[2 * i + 1];
    out_host[2 * i] = c * x - sn * y;
    out_host[2 * i + 1] = A * (sn * x + c * y);
  }
  return VECCHIA_OK;
}

}  // extern "C"
