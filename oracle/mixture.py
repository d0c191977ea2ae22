"""Gaussian scale mixture: the outer integral over the random scale R
(Section 4, eqs. (7)-(9)). Test infrastructure only, like the rest of oracle/.

Model: X = R W with W a Gaussian process and R ~ F_R independent of W, eq. (8):
    beta > 0:  F_R(r) = 1 - exp{-gamma (r^beta - 1) / beta},   r >= 1
    beta = 0:  F_R(r) = 1 - r^(-gamma),                         r >= 1
(the beta = 0 case is printed as 1 - r^gamma, which is negative for r > 1; it is
read as the Pareto law 1 - r^(-gamma)). The marginal CDF is eq. (9):
    G(x) = int_1^inf Phi_D(x / r) f_R(r) dr.

Quadrature (the paper asks for a numerical rule and names none). With
v = -log(1 - F_R(R)), which is Exp(1) whatever F_R is, eq. (9) becomes
    G = int_0^inf e^-v h(v) dv,   h(v) = Phi_D(x / r(v)),
    r(v) = e^(v / gamma) (beta = 0)  or  (1 + beta v / gamma)^(1 / beta) (beta > 0),
capped at 1e300 (x / r is then zero to double precision).
For large D, h falls steeply from v = 0 (its log-slope grows with D), so the
rule follows that decay:
  1. pass 1 evaluates log h at v = 0 and v = delta (delta = 1e-3) and takes
     mu = 1 + max(0, -(log h(delta) - log h(0)) / delta);
  2. pass 2 is n-node Gauss-Laguerre in tau = mu v:
        G = (1 / mu) sum_k w_k exp(tau_k (1 - 1/mu)) h(tau_k / mu),
     summed in log space. It is exact whenever log h is linear in v, in
     particular for h constant (x = 0, where Phi_D(x / r) = Phi_D(0) for every r,
     so G = Phi_D(0)), and for any F_R the mixing law itself is integrated by
     the Laguerre weight exactly.
The standard error propagates each node's log-CDF SE (first order):
    se(log G)^2 = sum_k (c_k / G)^2 se_k^2,  c_k the k-th summand of G.
The same seed is used at every node (common random numbers), so G is a smooth
function of the thresholds.
"""
from __future__ import annotations

import math

import numpy as np

DELTA = 1e-3


R_MAX = 1e300   # r is capped here: x / r is then zero to double precision


def scale_at(v: float, beta: float, gamma: float) -> float:
    """r(v) = F_R^{-1}(1 - e^-v), eq. (8), capped at R_MAX."""
    s = v / gamma if beta == 0.0 else math.log1p(beta * v / gamma) / beta
    return R_MAX if s >= math.log(R_MAX) else math.exp(s)


def laguerre_nodes(n: int):
    """Gauss-Laguerre nodes and weights for int_0^inf e^-t g(t) dt (library routine)."""
    t, w = np.polynomial.laguerre.laggauss(n)
    return t, w


def pass2(mu: float, n: int, beta: float, gamma: float):
    """Pass-2 scales r_k = r(tau_k / mu) and log weights log(w_k / mu) + tau_k (1 - 1/mu)."""
    t, w = laguerre_nodes(n)
    scales = np.array([scale_at(float(tk) / mu, beta, gamma) for tk in t])
    return scales, np.log(w) - math.log(mu) + t * (1.0 - 1.0 / mu)


def logsumexp(v) -> float:
    v = np.asarray(v, dtype=np.float64)
    mx = float(np.max(v))
    return mx + math.log(math.fsum(np.exp(v - mx)))


def logcdf_mixture(eval_logF, beta: float, gamma: float, n_nodes: int):
    """eval_logF(scale) -> (log Phi_D(x / scale), se). Returns dict(logG, se, mu,
    scales, node_logF)."""
    if not (gamma > 0.0 and beta >= 0.0 and n_nodes >= 1):
        raise ValueError("need gamma > 0, beta >= 0, n_nodes >= 1")
    h0, _ = eval_logF(1.0)
    h1, _ = eval_logF(scale_at(DELTA, beta, gamma))
    mu = 1.0 + max(0.0, -(h1 - h0) / DELTA)
    scales, logw = pass2(mu, n_nodes, beta, gamma)
    node = [eval_logF(float(r)) for r in scales]
    logF = np.array([v[0] for v in node])
    se = np.array([v[1] for v in node])
    summand = logw + logF
    logG = logsumexp(summand)
    frac = np.exp(summand - logG)
    se_G = math.sqrt(math.fsum((frac * se) ** 2))
    return dict(logG=logG, se=se_G, mu=mu, scales=scales, node_logF=logF)
