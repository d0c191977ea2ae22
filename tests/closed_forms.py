"""Gaussian CDFs with closed forms or 1-D integral forms, used as pins.

These are textbook results, independent of the SOV/QMC estimator:
* Sheppard (1899): P(X1 < 0, X2 < 0) = 1/4 + asin(rho) / (2 pi).
* Trivariate orthant: P(X < 0) = 1/8 + (asin r12 + asin r13 + asin r23) / (4 pi).
* Equicorrelated normal (Dunnett & Sobel 1955; Tong 1990): with unit variances
  and common correlation rho >= 0, X_i = sqrt(rho) Z + sqrt(1-rho) E_i, so
  P(X < b) = int phi(z) prod_i Phi((b_i - sqrt(rho) z) / sqrt(1 - rho)) dz;
  for rho = 1/2 and b = 0 this is 1 / (D + 1).
* Bivariate normal by conditioning on X1:
  P(X1 < b1, X2 < b2) = int_{-inf}^{b1} phi(z) Phi((b2 - rho z) / sqrt(1 - rho^2)) dz.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import ndtr
from scipy.stats import norm


def sheppard(rho: float) -> float:
    return 0.25 + math.asin(rho) / (2.0 * math.pi)


def orthant3(r12: float, r13: float, r23: float) -> float:
    return 0.125 + (math.asin(r12) + math.asin(r13) + math.asin(r23)) / (4.0 * math.pi)


def bivariate_cdf(b1: float, b2: float, rho: float) -> float:
    s = math.sqrt(1.0 - rho * rho)
    f = lambda z: norm.pdf(z) * ndtr((b2 - rho * z) / s)
    val, _ = integrate.quad(f, -np.inf, b1, epsabs=1e-14, epsrel=1e-12, limit=200)
    return val


def equicorrelated_cdf(b, rho: float) -> float:
    b = np.asarray(b, dtype=np.float64)
    sr, sq = math.sqrt(rho), math.sqrt(1.0 - rho)
    f = lambda z: norm.pdf(z) * float(np.prod(ndtr((b - sr * z) / sq)))
    val, _ = integrate.quad(f, -np.inf, np.inf, epsabs=1e-15, epsrel=1e-12, limit=400)
    return val


def monte_carlo_cdf(Sigma, b, n: int, seed: int, batch: int = 1_000_000):
    """Brute-force Monte Carlo P(X < b), X ~ N(0, Sigma); returns (p, se)."""
    Sigma = np.asarray(Sigma, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    L = np.linalg.cholesky(Sigma)
    rng = np.random.Generator(np.random.PCG64(seed))
    hits = 0
    done = 0
    while done < n:
        nb = min(batch, n - done)
        X = rng.standard_normal((nb, len(b))) @ L.T
        hits += int(np.count_nonzero(np.all(X < b, axis=1)))
        done += nb
    p = hits / n
    return p, math.sqrt(p * (1.0 - p) / n)


def bivariate_owen(h: float, k: float, rho: float) -> float:
    """P(X1 < h, X2 < k), unit variances, correlation rho, by Owen's (1956)
    T-function identity (h, k != 0):
      1/2 [Phi(h) + Phi(k)] - T(h, a_h) - T(k, a_k) - delta,
      a_h = (k - rho h) / (h sqrt(1 - rho^2)), a_k = (h - rho k) / (k sqrt(1 - rho^2)),
      delta = 0 if h k > 0 else 1/2."""
    from scipy.special import owens_t
    s = math.sqrt(1.0 - rho * rho)
    ah = (k - rho * h) / (h * s)
    ak = (h - rho * k) / (k * s)
    delta = 0.0 if h * k > 0.0 else 0.5
    return 0.5 * (float(ndtr(h)) + float(ndtr(k))) - float(owens_t(h, ah)) - float(owens_t(k, ak)) - delta


def one_factor_cdf(y, a: float, c: float) -> float:
    """P(Y < y) for Y_j = sqrt(a) Z + sqrt(c) E_j (Z, E_j iid N(0, 1)), i.e.
    covariance c I + a 1 1^T: int phi(z) prod_j Phi((y_j - sqrt(a) z) / sqrt(c)) dz."""
    y = np.asarray(y, dtype=np.float64)
    sa, sc = math.sqrt(a), math.sqrt(c)
    f = lambda z: norm.pdf(z) * float(np.prod(ndtr((y - sa * z) / sc)))
    val, _ = integrate.quad(f, -np.inf, np.inf, epsabs=1e-15, epsrel=1e-12, limit=400)
    return val
