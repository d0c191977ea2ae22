"""Joint (block) conditional Vecchia log-CDF (Section 3.2). Test infrastructure
only, like the rest of oracle/.

The telescoping product of eq. (5) can also run over groups: the D components
(in plan order) are cut into consecutive groups of p, G_1, G_2, ..., and
    P(X <= x) = prod_g P(X_{G_g} <= x_{G_g} | X_{earlier groups} <= x).
Each factor conditions on a smaller set instead: C_g, the union over the
members of G_g of their m nearest neighbours among the components of earlier
groups (the paper's first construction: the m most correlated per member, a
set of at most p m). Each term is then a ratio of Gaussian CDFs of dimension
|C_g| + |G_g| and |C_g|, from one SOV chain over the variables (C_g, G_g) whose
denominator is the prefix of its first |C_g| factors (sov.term_sums with
split = |C_g|).

Readings: groups are consecutive plan positions [g p, (g + 1) p) (the last one
ragged); C_g lists the members' neighbour lists in member order, each in the
(d^2, index) order of neighbours.knn_preceding restricted to positions before
the group, keeping the first occurrence of a repeated index; the shift key of
term g is g. With p = 1 this is the plain Vecchia log-CDF (eq. (6)).
"""
from __future__ import annotations

import math

import numpy as np

from . import covariance, ordering, sov


def nearest_before(s: np.ndarray, i: int, limit: int, m: int) -> np.ndarray:
    """The min(m, limit) positions j < limit nearest to s[i] under (d^2, j)."""
    if limit <= 0 or m <= 0:
        return np.zeros(0, dtype=np.int64)
    dx = s[:limit, 0] - s[i, 0]
    dy = s[:limit, 1] - s[i, 1]
    d2 = dx * dx + dy * dy
    idx = np.arange(limit)
    order = np.lexsort((idx, d2))
    return order[:min(m, limit)].astype(np.int64)


def block_plan(locs, rule: int, m: int, p: int, perm=None):
    """Return (perm, groups, conds): plan-index arrays of every group and its
    conditioning set."""
    locs = np.asarray(locs, dtype=np.float64)
    D = locs.shape[0]
    perm = ordering.order(locs, rule, perm)
    s = locs[perm]
    groups, conds = [], []
    for g0 in range(0, D, p):
        members = np.arange(g0, min(D, g0 + p), dtype=np.int64)
        cond = []
        for i in members:
            for j in nearest_before(s, int(i), g0, m):
                if int(j) not in cond:
                    cond.append(int(j))
        groups.append(members)
        conds.append(np.array(cond, dtype=np.int64))
    return perm, groups, conds


def _job(args):
    g, C, b, split, n_points, n_shifts, seed, independent = args
    return sov.term_estimate(C, b, n_points, n_shifts, seed, g, split=split, independent=independent)


def logcdf_block(locs, x, m, p, family, nu, sigma2, rho, nugget, rule, n_points, n_shifts, seed,
                 scale: float = 1.0, perm=None, processes: int = 1, plan_cache=None,
                 independent: bool = False):
    """Block Vecchia log-CDF. Returns dict(logF, se, terms (one row per group,
    group order), perm, groups, conds). independent: as sov.term_estimate."""
    locs = np.asarray(locs, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if plan_cache is not None:
        perm, groups, conds = plan_cache
    else:
        perm, groups, conds = block_plan(locs, rule, m, p, perm)
    s = locs[perm]
    b_all = x[perm] / scale
    jobs = []
    for g, (G, Cg) in enumerate(zip(groups, conds)):
        v = np.concatenate([Cg, G])
        C = covariance.cov_matrix(s[v], family, nu, sigma2, rho, nugget)
        jobs.append((g, C, b_all[v], len(Cg), n_points, n_shifts, seed, independent))
    from concurrent.futures import ProcessPoolExecutor
    if processes <= 1 or len(jobs) < 2:
        res = [_job(j) for j in jobs]
    else:
        with ProcessPoolExecutor(max_workers=processes) as ex:
            res = list(ex.map(_job, jobs, chunksize=max(1, len(jobs) // (8 * processes))))
    terms = np.array(res, dtype=np.float64).reshape(len(jobs), 2)
    return dict(logF=math.fsum(terms[:, 0]), se=math.sqrt(math.fsum(terms[:, 1] ** 2)), terms=terms,
                perm=perm, groups=groups, conds=conds)


def logcdf_block_from_cov(Sigma, x, groups, conds, n_points, n_shifts, seed, scale: float = 1.0):
    """Block terms over an explicit covariance in identity order."""
    Sigma = np.asarray(Sigma, dtype=np.float64)
    b_all = np.asarray(x, dtype=np.float64) / scale
    res = []
    for g, (G, Cg) in enumerate(zip(groups, conds)):
        v = np.concatenate([np.asarray(Cg, dtype=np.int64), np.asarray(G, dtype=np.int64)])
        res.append(sov.term_estimate(Sigma[np.ix_(v, v)], b_all[v], n_points, n_shifts, seed, g,
                                     split=len(Cg)))
    terms = np.array(res, dtype=np.float64).reshape(len(res), 2)
    return dict(logF=math.fsum(terms[:, 0]), se=math.sqrt(math.fsum(terms[:, 1] ** 2)), terms=terms)
