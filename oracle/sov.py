"""One Vecchia term Phi_{k+1}(b) / Phi_k(b[:k]) by separation of variables + QMC.

Section 2.2, eq. (6): the term of component i is the ratio of the CDF of
(X_{N_i}, X_i) at (x_{N_i}, x_i) to the CDF of X_{N_i} at x_{N_i}; the paper asks
for a Genz-type QM estimate of numerator and denominator.

Variables are ordered neighbours first, component i last. With C = L L^T,
Genz's transform writes the (k+1)-dimensional CDF as an integral over [0,1]^k:
    e_1     = Phi(b_1 / L_11)
    y_{a-1} = Phi^{-1}(w_{a-1} e_{a-1})                         a = 2..k+1
    e_a     = Phi((b_a - sum_{b<a} L_ab y_b) / L_aa)
    Phi_{k+1}(b) = E_w[ prod_{a=1}^{k+1} e_a ],   Phi_k(b[:k]) = E_w[ prod_{a=1}^{k} e_a ]
(the prefix product does not depend on w_k, so one point set serves both).
Per shift r the means over the N lattice points are n_r and d_r; the estimate is
log(mean_r n_r) - log(mean_r d_r) and its standard error is the delta-method
one from the R shift replicates:
    se^2 = sum_r (n_r / n - d_r / d)^2 / (R (R - 1)).
When a factor e_a is exactly 0 the sample's products are 0 and its later
coordinates are not used; u = w e is clamped below at the smallest normal double.

Infinite limits (the paper is silent; reading): b_a = +inf leaves variable a
unconstrained (e_a = 1, so it only shapes the later conditional means), and a
term any of whose limits is -inf is 0 (log-term -inf, SE 0). Its numerator
vanishes; when the -inf limit is a conditioning one the ratio is 0 / 0, and
taking it as 0 keeps the product of eq. (6) equal to Phi_D = 0.
"""
from __future__ import annotations

import math
import sys

import numpy as np
from scipy.special import ndtr, ndtri

from . import lattice

DBL_MIN = sys.float_info.min


class NotPositiveDefinite(Exception):
    pass


def term_sums(C: np.ndarray, b: np.ndarray, n_points: int, n_shifts: int, seed: int,
              term: int, Z: list | None = None, split: int | None = None, second: bool = False):
    """Return (L, num[R], den[R]): per-shift lattice means of the numerator and
    denominator integrands of the term with covariance C and limits b.

    split (default n - 1): the denominator is the CDF of the first `split`
    variables, E[prod_{a<split} e_a] (a joint block term of Section 3.2 has its
    conditioning variables first and its group last); split = 0 gives 1.
    second: use the term's second lattice (lattice.shift(..., second=True))."""
    n = len(b)
    try:
        L = np.linalg.cholesky(C)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    k = n - 1
    split = k if split is None else split
    Z = lattice.richtmyer_generator() if Z is None else Z
    num = np.empty(n_shifts)
    den = np.empty(n_shifts)
    e1 = ndtr(b[0] / L[0, 0])
    for r in range(n_shifts):
        e = np.full(n_points, e1)
        prod = e.copy()                    # running product e_1 ... e_{a-1}
        head = np.ones(n_points) if split == 0 else (prod.copy() if split == 1 else None)
        ys = np.zeros((k, n_points))
        for a in range(1, n):              # 0-based variable a = 1..k
            w = lattice.points(n_points, a - 1, lattice.shift(seed, term, r, a - 1, second), Z)
            alive = e > 0.0
            u = np.maximum(w * e, DBL_MIN)
            y = np.where(alive, ndtri(u), 0.0)
            ys[a - 1] = y
            acc = np.full(n_points, b[a])
            for c in range(a):
                acc = acc - L[a, c] * ys[c]
            e = np.where(alive, ndtr(acc / L[a, a]), 0.0)
            if a < k:
                prod = prod * e
                if a + 1 == split:
                    head = prod.copy()
        den[r] = np.mean(head)
        num[r] = np.mean(prod * e)
    return L, num, den


def term_estimate(C: np.ndarray, b: np.ndarray, n_points: int, n_shifts: int, seed: int,
                  term: int, Z: list | None = None, split: int | None = None,
                  independent: bool = False):
    """Return (log_term, se) of one Vecchia term (split: as term_sums).

    independent: the paper-literal form that estimates the numerator and the
    denominator from separate point sets: the numerator from the term's lattice,
    the denominator from its second lattice; the two estimates are independent,
    so their relative variances add:
        se^2 = [sum_r (n_r / n - 1)^2 + sum_r (d_r / d - 1)^2] / (R (R - 1))."""
    if np.any(np.asarray(b) == -np.inf):
        # a covariance that is not positive definite is reported first
        try:
            np.linalg.cholesky(C)
        except np.linalg.LinAlgError as exc:
            raise NotPositiveDefinite(str(exc)) from exc
        return -math.inf, 0.0
    if len(b) == 1:
        if not C[0, 0] > 0.0:
            raise NotPositiveDefinite("variance <= 0")
        with np.errstate(divide="ignore"):
            return float(np.log(ndtr(b[0] / math.sqrt(C[0, 0])))), 0.0
    _, num, den = term_sums(C, b, n_points, n_shifts, seed, term, Z, split)
    if independent:
        _, _, den = term_sums(C, b, n_points, n_shifts, seed, term, Z, split, second=True)
    nh = np.mean(num)
    dh = np.mean(den)
    with np.errstate(divide="ignore", invalid="ignore"):
        log_term = float(np.log(nh) - np.log(dh))
    R = n_shifts
    if R < 2:
        return log_term, float("nan")
    if independent:
        se2 = (np.sum((num / nh - 1.0) ** 2) + np.sum((den / dh - 1.0) ** 2)) / (R * (R - 1))
    else:
        se2 = np.sum((num / nh - den / dh) ** 2) / (R * (R - 1))
    return log_term, float(math.sqrt(se2))
