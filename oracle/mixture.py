"""Gaussian scale mixture: the outer integral over the random scale R
(Section 4, eqs. (7)-(9), (11)). Test infrastructure only, like the rest of oracle/.

Model: X = R W with W a Gaussian process and R ~ F_R independent of W, eq. (8):
    beta > 0:  F_R(r) = 1 - exp{-gamma (r^beta - 1) / beta},   r >= 1
    beta = 0:  F_R(r) = 1 - r^(-gamma),                         r >= 1
(the beta = 0 case is printed as 1 - r^gamma, which is negative for r > 1; it is
read as the Pareto law 1 - r^(-gamma)). The marginal CDF is eq. (9),
    G(x) = int_1^inf Phi_D(x / r) f_R(r) dr,
and the censored likelihood, eq. (11), has the same form with Phi_D(x / r)
replaced by the integrand L_r(x) of oracle.censored.

Quadrature (the paper asks for a numerical rule and names none). With
v = -log(1 - F_R(R)), which is Exp(1) whatever F_R is,
    G = int_0^inf e^-v h(v) dv,   h(v) = Phi_D(x / r(v))  (or L_r(x)),
    r(v) = e^(v / gamma) (beta = 0)  or  (1 + beta v / gamma)^(1 / beta) (beta > 0),
capped at 1e300 (x / r is then zero to double precision). The bulk of
l(v) = log h(v) - v sits at v = 0 for a plain CDF with positive thresholds
(steeply so for large D) and inside (0, inf) for a censored likelihood (the
density factors grow with r before the r^-|I| Jacobian wins), so the rule first
finds it:
  1. search: l at the 24 points v = 0 and v_j = 1e-4 (2e6)^((j-1)/22), j = 1..23
     (1e-4 to 200), with n_points / 16 lattice points (at least 64, a multiple
     of 64) and the call's shifts and seed;
  2. window: with j* the search maximum, lo = the nearest search point left of
     j* whose l is more than 36 below the maximum (else 0) and hi = the nearest
     one right of it (else 200); e^-36 < 3e-16 of the peak is left outside;
     (the window covers the mode holding the search maximum: all of the mass
     when l is unimodal, as for log-concave integrands);
  3. n-point Gauss-Legendre on [lo, hi], in s = log v when lo > 0 and
     hi / lo > 8, else in v, at the full lattice size:
        G = sum_k w_k e^(-v_k) h(v_k)   (w_k including the map's Jacobian),
     summed in log space.
The standard error propagates each node's log-CDF SE (first order):
    se(log G)^2 = sum_k (c_k / G)^2 se_k^2,  c_k the k-th summand of G.
The same seed is used at every node (common random numbers), so G is a smooth
function of the thresholds.
"""
from __future__ import annotations

import math

import numpy as np

R_MAX = 1e300          # r is capped here: x / r is then zero to double precision
N_SEARCH = 24
V_SEARCH_MAX = 200.0
CUT = 36.0
LOG_SPAN = 8.0


def scale_at(v: float, beta: float, gamma: float) -> float:
    """r(v) = F_R^{-1}(1 - e^-v), eq. (8), capped at R_MAX."""
    s = v / gamma if beta == 0.0 else math.log1p(beta * v / gamma) / beta
    return R_MAX if s >= math.log(R_MAX) else math.exp(s)


def search_v():
    return [0.0] + [1e-4 * 2e6 ** ((j - 1) / 22) for j in range(1, N_SEARCH)]


def search_n_points(n_points: int) -> int:
    return max(64, ((n_points // 16 + 63) // 64) * 64)


def window(search_logF):
    """[lo, hi] from the search values log h(v_j) (step 2)."""
    v = search_v()
    ell = [float(h) - vj for h, vj in zip(search_logF, v)]
    j = int(np.argmax(ell))
    top = ell[j]
    lo, hi = 0.0, V_SEARCH_MAX
    for i in range(j - 1, -1, -1):
        if ell[i] < top - CUT:
            lo = v[i]
            break
    for i in range(j + 1, N_SEARCH):
        if ell[i] < top - CUT:
            hi = v[i]
            break
    return lo, hi


def legendre_rule(lo: float, hi: float, n: int):
    """Nodes v_k and log weights log w_k - v_k of step 3 (leggauss: library routine)."""
    t, w = np.polynomial.legendre.leggauss(n)
    if lo > 0.0 and hi / lo > LOG_SPAN:
        a, b = math.log(lo), math.log(hi)
        s = a + (b - a) * (t + 1.0) / 2.0
        v = np.exp(s)
        logw = np.log(w * (b - a) / 2.0) + s - v
    else:
        v = lo + (hi - lo) * (t + 1.0) / 2.0
        logw = np.log(w * (hi - lo) / 2.0) - v
    return v, logw


def logsumexp(v) -> float:
    v = np.asarray(v, dtype=np.float64)
    mx = float(np.max(v))
    if mx == -math.inf:
        return -math.inf
    return mx + math.log(math.fsum(np.exp(v - mx)))


def logcdf_mixture(eval_logF, beta: float, gamma: float, n_nodes: int, eval_search=None):
    """eval_logF(scale) -> (log h at scale, se), at the full lattice size;
    eval_search(scale) -> the same at the search size (default eval_logF).
    Returns dict(logG, se, window, v, scales, node_logF, search_logF)."""
    if not (gamma > 0.0 and beta >= 0.0 and n_nodes >= 1):
        raise ValueError("need gamma > 0, beta >= 0, n_nodes >= 1")
    ev_s = eval_logF if eval_search is None else eval_search
    search = [ev_s(scale_at(v, beta, gamma))[0] for v in search_v()]
    lo, hi = window(search)
    v, logw = legendre_rule(lo, hi, n_nodes)
    scales = np.array([scale_at(float(vk), beta, gamma) for vk in v])
    node = [eval_logF(float(r)) for r in scales]
    logF = np.array([p[0] for p in node])
    se = np.array([p[1] for p in node])
    summand = logw + logF
    logG = logsumexp(summand)
    # G = 0 (every node 0, e.g. a -inf threshold) is exact: SE 0
    frac = np.exp(summand - logG) if logG > -math.inf else np.zeros_like(summand)
    se_G = math.sqrt(math.fsum((frac * se) ** 2))
    return dict(logG=logG, se=se_G, window=(lo, hi), v=v, scales=scales, node_logF=logF,
                search_logF=np.array(search))
