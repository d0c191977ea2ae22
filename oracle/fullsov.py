"""Full-dimension SOV estimate of log Phi_D(b) (Genz's method over all D
variables), the comparator the paper checks the Vecchia approximation against
(Section 3.1, Figures 1-4). Test infrastructure only, like the rest of oracle/.

With C = L L^T, separation of variables writes Phi_D(b) = E_w[prod_{a<D} e_a]
over w in [0,1]^(D-1) with
    e_0 = Phi(b_0 / L_00),  y_{a-1} = Phi^-1(w_{a-1} e_{a-1}),
    e_a = Phi((b_a - sum_{c<a} L_ac y_c) / L_aa),   a = 1..D-1,
the same recursion as one Vecchia term with every preceding variable in its
conditioning set. The lattice is oracle.lattice's rule in D - 1 dimensions
(Z_j from the first D - 1 primes) and the shift of dimension j in replicate r
is lattice.full_shift(seed, r, j). For large D the product underflows, so each
sample carries log prod e_a = sum_a log Phi(t_a) (scipy's log_ndtr), u = w e is
clamped below at the smallest normal double, and the per-replicate mean of the
products is taken in log space:
    l_r = log((1/N) sum_p exp(sum_a log e_a(p))),
    log F = log((1/R) sum_r exp(l_r)),
    se(log F) = sqrt(sum_r (exp(l_r - log F) - 1)^2 / (R (R - 1)))   (delta method).
"""
from __future__ import annotations

import math
import sys

import numpy as np
from scipy.special import log_ndtr, ndtr, ndtri

from . import lattice
from .mixture import logsumexp

DBL_MIN = sys.float_info.min


def logcdf_full(C: np.ndarray, b: np.ndarray, n_points: int, n_shifts: int, seed: int,
                Z: list | None = None):
    """Return (log F, se, l_r[R]) for X ~ N(0, C) at thresholds b."""
    C = np.asarray(C, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    D = len(b)
    L = np.linalg.cholesky(C)
    Z = lattice.richtmyer_generator(max(1, D - 1)) if Z is None else Z
    lr = np.empty(n_shifts)
    for r in range(n_shifts):
        t = np.full(n_points, b[0] / L[0, 0])
        e = ndtr(t)
        lp = log_ndtr(t)
        ys = np.zeros((max(0, D - 1), n_points))
        for a in range(1, D):
            w = lattice.points(n_points, a - 1, lattice.full_shift(seed, r, a - 1), Z)
            ys[a - 1] = ndtri(np.maximum(w * e, DBL_MIN))
            acc = np.full(n_points, b[a])
            acc = acc - L[a, :a] @ ys[:a]
            t = acc / L[a, a]
            e = ndtr(t)
            lp = lp + log_ndtr(t)
        lr[r] = logsumexp(lp) - math.log(n_points)
    logF = logsumexp(lr) - math.log(n_shifts)
    R = n_shifts
    if R < 2:
        return logF, float("nan"), lr
    se = math.sqrt(math.fsum((math.exp(v - logF) - 1.0) ** 2 for v in lr) / (R * (R - 1)))
    return logF, se, lr
