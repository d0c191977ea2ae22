"""Pins of the oracle for infinite thresholds. The paper is silent on them; the
reading is that a limit of +inf leaves its component unconstrained and a limit
of -inf makes the probability 0. Checked against the marginalisation identity
P(X_A <= x_A, X_B <= +inf) = P(X_A <= x_A) with closed forms for the right-hand
side (Owen's T-function identity, the one-factor integral), the exact zero of a
term whose own limit is +inf, and log F = -inf for a -inf limit, in the plain,
joint (block) and censored forms.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import block, censored, covariance, sov
from tests import closed_forms as cf

EXP = covariance.COV_EXPONENTIAL
MAT = covariance.COV_MATERN


def test_own_limit_plus_inf_gives_an_exact_zero_term():
    rng = np.random.default_rng(3)
    pts = rng.random((5, 2))
    C = covariance.cov_matrix(pts, MAT, 1.5, 1.3, 0.3, 1e-8)
    b = np.append(rng.normal(0.2, 1.0, size=4), np.inf)
    assert sov.term_estimate(C, b, 512, 6, 7, 3) == (0.0, 0.0)
    assert sov.term_estimate(C[:1, :1], np.array([np.inf]), 512, 6, 7, 0) == (0.0, 0.0)


def test_unconstrained_component_marginalises_out_exactly():
    # m = D - 1: the Vecchia product is exact, so log F equals log P(X_0 <= h, X_2 <= k)
    pts = np.array([[0.0, 0.0], [0.15, 0.05], [0.1, 0.25]])
    C = covariance.cov_matrix(pts, EXP, 0.5, 1.0, 0.5, 0.0)
    for (h, k) in ((0.4, -0.3), (-1.1, 0.8), (1.5, 1.2)):
        r = oracle.logcdf_from_cov(C, np.array([h, np.inf, k]), [[], [0], [0, 1]], 4096, 10, 11)
        want = math.log(cf.bivariate_owen(h, k, C[0, 2]))
        assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-9, (h, k, r["logF"], want, r["se"])
        assert r["terms"][1, 0] == 0.0 and r["terms"][1, 1] == 0.0


def test_one_factor_covariance_with_unbounded_components():
    # covariance c I + a 1 1^T: dropping components leaves the same family, so
    # Phi_D with some limits at +inf is the one-factor integral over the rest
    D, a, c = 8, 0.35, 0.65
    Sigma = c * np.eye(D) + a
    x = np.array([0.3, np.inf, -0.4, 0.9, np.inf, 0.1, 1.2, np.inf])
    nbrs = [list(range(i)) for i in range(D)]
    r = oracle.logcdf_from_cov(Sigma, x, nbrs, 4096, 10, 13)
    want = math.log(cf.one_factor_cdf(x[np.isfinite(x)], a, c))
    assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-9, (r["logF"], want, r["se"])


def test_minus_inf_limit_gives_minus_inf_and_leaves_other_terms_alone():
    rng = np.random.default_rng(5)
    locs = rng.random((40, 2))
    x = rng.normal(1.0, 0.5, size=40)
    args = (4, MAT, 1.5, 1.0, 0.2, 1e-8, 2, 256, 4, 17)
    base = oracle.logcdf(locs, x, *args)
    j = 7
    x2 = x.copy()
    x2[j] = -np.inf
    r = oracle.logcdf(locs, x2, *args)
    assert r["logF"] == -math.inf
    perm, nbrs = r["perm"], r["nbrs"]
    pj = int(np.flatnonzero(perm == j)[0])
    for i in range(40):
        involved = i == pj or pj in set(int(v) for v in nbrs[i])
        lt, se = r["terms"][perm[i]]
        if involved:
            assert lt == -math.inf and se == 0.0
        else:
            assert (lt, se) == tuple(base["terms"][perm[i]])


def test_block_terms_with_infinite_limits():
    rng = np.random.default_rng(8)
    locs = rng.random((30, 2))
    x = rng.normal(0.8, 0.6, size=30)
    x[[3, 11]] = np.inf
    r = block.logcdf_block(locs, x, 3, 3, MAT, 1.5, 1.0, 0.25, 1e-8, 2, 256, 4, 19)
    assert np.all(np.isfinite(r["terms"][:, 0]))
    x[20] = -np.inf
    r = block.logcdf_block(locs, x, 3, 3, MAT, 1.5, 1.0, 0.25, 1e-8, 2, 256, 4, 19)
    assert r["logF"] == -math.inf


def test_censored_infinite_values():
    # an observed site at +-inf has zero density; a censored limit of +inf is no constraint
    rng = np.random.default_rng(9)
    locs = rng.random((25, 2))
    x = rng.normal(0.5, 0.7, size=25)
    obs = np.zeros(25, dtype=bool)
    obs[[1, 4, 9, 16]] = True
    args = (3, MAT, 1.5, 1.0, 0.2, 1e-8, 2, 256, 4, 23)
    x1 = x.copy()
    x1[4] = np.inf
    assert censored.loglik(locs, x1, obs, *args)["logL"] == -math.inf
    x2 = x.copy()
    x2[12] = np.inf
    r = censored.loglik(locs, x2, obs, *args)
    assert np.isfinite(r["logL"])
    assert r["terms"][12, 0] == 0.0 and r["terms"][12, 1] == 0.0
    x3 = x.copy()
    x3[12] = -np.inf
    assert censored.loglik(locs, x3, obs, *args)["logL"] == -math.inf


def test_not_positive_definite_is_reported_before_minus_inf():
    C = np.array([[1.0, 1.2], [1.2, 1.0]])
    with pytest.raises(sov.NotPositiveDefinite):
        sov.term_estimate(C, np.array([-np.inf, 0.3]), 64, 2, 1, 1)
