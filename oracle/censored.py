"""Censored likelihood of one replicate (Section 4, eq. (11)) in Vecchia form.
Test infrastructure only, like the rest of oracle/.

A replicate observes D sites. I holds the sites above the censoring threshold
(their value x_i is known exactly); I^c holds the censored sites (only
X_i <= x_i is known, x_i being the threshold). At scale r, eq. (11)'s integrand
is the |I|-th partial derivative of Phi_D(x / r) in x_I:
    L_r(x) = phi_{|I|}(x_I / r; S_II) r^-|I|
             * Phi_{|I^c|}((x_{I^c} - S_{I^c,I} S_II^-1 x_I) / r; S_{I^c|I}).

Reading (the paper states eq. (11) and no Vecchia form of it): sort the sites
so that every uncensored site precedes every censored one, each group keeping
its order under the base ordering. In that order L_1 factorises exactly as
    prod_{i in I} f(x_i | x_{I before i})
    * prod_{i in I^c} P(X_i <= x_i | X_{I^c before i} <= x_{I^c before i}, X_I = x_I),
and every factor conditions on N_i, the m nearest preceding sites, instead:
  * i in I: N_i holds uncensored sites only and the factor is the univariate
    Gaussian density with the conditional mean and variance stated after
    eq. (3) (the Vecchia density, eq. (4));
  * i in I^c: N_i splits into E (uncensored, conditioned on by equality) and C
    (censored, by inequality). With A = (C, i), the factor is the Vecchia term
    of eq. (6) for the conditional Gaussian of X_A given X_E = b_E:
        mean mu_A = S_AE S_EE^-1 b_E,   covariance S_A|E = S_AA - S_AE S_EE^-1 S_EA,
        factor = Phi_{|C|+1}(b_A - mu_A; S_A|E) / Phi_{|C|}(b_C - mu_C; S_C|E),
    estimated like every other term (sov.term_estimate) with the plan index i
    as its shift key.
With m = D - 1 every N_i is every preceding site and the product is L_1
exactly. At scale r the limits are b = x / r and each density factor gains the
Jacobian 1 / r.

Infinite values (reading, as in sov): a factor any of whose variables is an
uncensored site with an infinite value, or has the limit -inf, is 0 (the
density vanishes at infinity; a probability of X <= -inf is 0).
"""
from __future__ import annotations

import math

import numpy as np

from . import covariance, neighbours, ordering, sov
from .vecchia import _run_terms

LOG_2PI = math.log(2.0 * math.pi)


def censored_plan(locs, observed, rule: int, m: int, perm=None):
    """Return (perm, nbrs, n_obs): the base ordering with the observed sites
    moved first (stable), the neighbour lists in that order, and |I|."""
    locs = np.asarray(locs, dtype=np.float64)
    obs = np.asarray(observed, dtype=bool)
    base = ordering.order(locs, rule, perm)
    first = base[obs[base]]
    rest = base[~obs[base]]
    perm2 = np.concatenate([first, rest]).astype(np.int64)
    nbrs = neighbours.knn_preceding(locs[perm2], m)
    return perm2, nbrs, int(first.size)


def conditional(C: np.ndarray, b: np.ndarray, eq: np.ndarray):
    """Gaussian of the variables not in eq given those in eq at b[eq]:
    returns (index of the others, mean, covariance) from plain solves."""
    E = np.flatnonzero(eq)
    A = np.flatnonzero(~eq)
    if E.size == 0:
        return A, np.zeros(A.size), C[np.ix_(A, A)]
    CEE = C[np.ix_(E, E)]
    CAE = C[np.ix_(A, E)]
    mu = CAE @ np.linalg.solve(CEE, b[E])
    S = C[np.ix_(A, A)] - CAE @ np.linalg.solve(CEE, CAE.T)
    return A, mu, 0.5 * (S + S.T)


def _terms(get_C, b_all, nbrs, n_obs, n_points, n_shifts, seed, scale, idx, processes, independent=False):
    """Evaluate the terms idx; returns {plan index: (log term, se)}."""
    out = {}
    jobs = []
    for i in idx:
        v = np.concatenate([nbrs[i], [i]]).astype(np.int64)
        C = get_C(v)
        b = b_all[v]
        eq = v < n_obs
        if np.any(b == -np.inf) or np.any(np.isinf(b[eq])):
            out[int(i)] = (-math.inf, 0.0)
            continue
        if i < n_obs:
            # density factor: every neighbour precedes i, so every one is observed
            _, mu, S = conditional(C, b, np.append(eq[:-1], False))
            var = float(S[0, 0])
            if not var > 0.0:
                raise sov.NotPositiveDefinite("conditional variance <= 0")
            z = (b[-1] - mu[0]) / math.sqrt(var)
            out[int(i)] = (-0.5 * (LOG_2PI + math.log(var)) - 0.5 * z * z - math.log(scale), 0.0)
        else:
            A, mu, S = conditional(C, b, eq)
            jobs.append((int(i), S, b[A] - mu, n_points, n_shifts, seed, independent))
    for (i, *_), r in zip(jobs, _run_terms(jobs, processes)):
        out[i] = r
    return out


def _assemble(res, perm, D):
    terms = np.full((D, 2), np.nan)
    for i, (lt, se) in res.items():
        terms[perm[i]] = (lt, se)
    lts = [v[0] for v in res.values()]
    ses = [v[1] for v in res.values()]
    return math.fsum(lts), math.sqrt(math.fsum(s * s for s in ses)), terms


def loglik(locs, x, observed, m, family, nu, sigma2, rho, nugget, rule, n_points, n_shifts,
           seed, scale: float = 1.0, perm=None, terms_subset=None, processes: int = 1,
           plan_cache=None, independent: bool = False):
    """Vecchia log L_r(x) of one replicate (r = scale). observed: D flags in
    user order (True = uncensored). Returns dict(logL, se, terms (D x 2, user
    order), perm, nbrs, n_obs); terms_subset restricts the terms (plan indices)."""
    locs = np.asarray(locs, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    D = locs.shape[0]
    if plan_cache is not None:
        perm2, nbrs, n_obs = plan_cache
    else:
        perm2, nbrs, n_obs = censored_plan(locs, observed, rule, m, perm)
    s = locs[perm2]
    b_all = x[perm2] / scale
    get_C = lambda v: covariance.cov_matrix(s[v], family, nu, sigma2, rho, nugget)
    idx = range(D) if terms_subset is None else terms_subset
    res = _terms(get_C, b_all, nbrs, n_obs, n_points, n_shifts, seed, scale, idx, processes, independent)
    logL, se, terms = _assemble(res, perm2, D)
    return dict(logL=logL, se=se, terms=terms, perm=perm2, nbrs=nbrs, n_obs=n_obs)


def loglik_from_cov(Sigma, x, n_obs: int, nbrs, n_points, n_shifts, seed, scale: float = 1.0,
                    processes: int = 1):
    """Vecchia log L_r(x) for an explicit covariance in identity order whose
    first n_obs variables are the uncensored ones; nbrs[i] holds indices < i."""
    Sigma = np.asarray(Sigma, dtype=np.float64)
    b_all = np.asarray(x, dtype=np.float64) / scale
    D = Sigma.shape[0]
    nb = [np.asarray(v, dtype=np.int64) for v in nbrs]
    get_C = lambda v: Sigma[np.ix_(v, v)]
    res = _terms(get_C, b_all, nb, n_obs, n_points, n_shifts, seed, scale, range(D), processes)
    logL, se, terms = _assemble(res, np.arange(D), D)
    return dict(logL=logL, se=se, terms=terms)
