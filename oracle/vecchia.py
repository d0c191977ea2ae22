"""The Vecchia log-CDF, assembled term by term (Section 2.2, eq. (6); Section 3.1).

logcdf():
  1. order the locations (ordering.order) and relabel: s_i = locs[perm[i]],
     b_i = x[perm[i]] / scale (scale-mixture thresholds x / r, eq. (9));
  2. N_i = nearest preceding neighbours (neighbours.knn_preceding);
  3. term i: variables (N_i[0], ..., N_i[k-1], i), covariance of those
     locations, SOV/QMC estimate with shifts keyed by the plan index i;
  4. log F = exactly rounded sum of the log terms (math.fsum), SE = sqrt(sum se^2).

Results per term are also returned in user index order: terms[perm[i]] = term i.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import covariance, lattice, neighbours, ordering, sov


def plan(locs: np.ndarray, rule: int, m: int, perm: np.ndarray | None = None):
    """Return (perm, nbrs): the ordering and the neighbour lists in plan indices."""
    locs = np.asarray(locs, dtype=np.float64)
    perm = ordering.order(locs, rule, perm)
    nbrs = neighbours.knn_preceding(locs[perm], m)
    return perm, nbrs


def _term_job(args):
    (i, C, b, n_points, n_shifts, seed, *rest) = args
    independent = bool(rest[0]) if rest else False
    return sov.term_estimate(C, b, n_points, n_shifts, seed, i, independent=independent)


def _run_terms(jobs, processes: int):
    if processes <= 1 or len(jobs) < 2:
        return [_term_job(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=processes) as ex:
        return list(ex.map(_term_job, jobs, chunksize=max(1, len(jobs) // (8 * processes))))


def logcdf(locs, x, m, family, nu, sigma2, rho, nugget, rule, n_points, n_shifts, seed,
           scale: float = 1.0, perm=None, terms_subset=None, processes: int = 1,
           plan_cache=None, independent: bool = False):
    """Vecchia log-CDF of a zero-mean GP at thresholds x / scale.

    Returns dict(logF, se, terms (D x 2, user order; NaN outside terms_subset),
    perm, nbrs). terms_subset: plan indices to evaluate (default all); logF and
    se then cover only those terms. independent: separate point sets for each
    term's numerator and denominator (sov.term_estimate).
    """
    locs = np.asarray(locs, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    D = locs.shape[0]
    if plan_cache is not None:
        perm, nbrs = plan_cache
    else:
        perm, nbrs = plan(locs, rule, m, perm)
    s = locs[perm]
    b_all = x[perm] / scale
    idx = range(D) if terms_subset is None else terms_subset
    jobs = []
    for i in idx:
        v = np.concatenate([nbrs[i], [i]]).astype(np.int64)
        C = covariance.cov_matrix(s[v], family, nu, sigma2, rho, nugget)
        jobs.append((int(i), C, b_all[v], n_points, n_shifts, seed, independent))
    res = _run_terms(jobs, processes)
    terms = np.full((D, 2), np.nan)
    for (i, *_), (lt, se) in zip(jobs, res):
        terms[perm[i]] = (lt, se)
    lts = [r[0] for r in res]
    ses = [r[1] for r in res]
    return dict(logF=math.fsum(lts), se=math.sqrt(math.fsum(v * v for v in ses)),
                terms=terms, perm=perm, nbrs=nbrs)


def logcdf_from_cov(Sigma, x, nbrs, n_points, n_shifts, seed, scale: float = 1.0,
                    processes: int = 1, independent: bool = False):
    """Vecchia log-CDF for an explicit covariance, identity ordering and given
    neighbour lists (nbrs[i] must hold indices < i, in the order to use)."""
    Sigma = np.asarray(Sigma, dtype=np.float64)
    b_all = np.asarray(x, dtype=np.float64) / scale
    D = Sigma.shape[0]
    jobs = []
    for i in range(D):
        v = np.concatenate([np.asarray(nbrs[i], dtype=np.int64), [i]])
        jobs.append((i, Sigma[np.ix_(v, v)], b_all[v], n_points, n_shifts, seed, independent))
    res = _run_terms(jobs, processes)
    terms = np.array(res, dtype=np.float64).reshape(D, 2)
    return dict(logF=math.fsum(terms[:, 0]), se=math.sqrt(math.fsum(terms[:, 1] ** 2)),
                terms=terms)


def default_processes() -> int:
    return max(1, min(16, os.cpu_count() or 1))
