"""Pins of the oracle's Vecchia log-CDF estimator against values fixed by the
mathematics: the 1-D case, diagonal covariances, Sheppard's and the trivariate
orthant formulas, equicorrelated normals (1-D integral form and the exact
1/(D+1) orthant), the bivariate conditioning integral, the exact case m = D-1
against brute-force Monte Carlo (telescoping identity, eq. (5)), and SE coverage.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtr

import oracle
from oracle import covariance, sov
from tests import closed_forms as cf

EXP = covariance.COV_EXPONENTIAL


def _exp_cov(pts, rho, sigma2=1.0):
    return covariance.cov_matrix(pts, EXP, 0.5, sigma2, rho, 0.0)


def test_single_location_is_exact():
    r = oracle.logcdf(np.array([[0.3, 0.4]]), np.array([0.7]), 5, EXP, 0.5, 2.0, 0.2, 0.0,
                      1, 64, 4, 1)
    assert r["logF"] == pytest.approx(math.log(ndtr(0.7 / math.sqrt(2.0))), abs=1e-15)
    assert r["se"] == 0.0


def test_diagonal_covariance_gives_product_of_marginals():
    # range 1e-9 on points >= 0.05 apart: off-diagonal exp(-h/rho) underflows to 0
    from workloads import grid_locations
    locs = grid_locations(5, 4)
    rng = np.random.default_rng(2)
    x = rng.normal(0.5, 1.0, size=20)
    r = oracle.logcdf(locs, x, 4, EXP, 0.5, 1.5, 1e-9, 0.0, 2, 256, 3, 9)
    want = np.log(ndtr(x / math.sqrt(1.5)))
    np.testing.assert_allclose(r["terms"][:, 0], want, rtol=0, atol=1e-13)   # user order
    assert r["logF"] == pytest.approx(math.fsum(want), abs=1e-12)


def test_bivariate_terms_match_conditioning_integral():
    # m = 1: every term is Phi_2(b_nbr, b_i; rho) / Phi(b_nbr)
    rng = np.random.default_rng(8)
    locs = rng.random((25, 2))
    x = rng.normal(0.3, 0.8, size=25)
    rho_cov = 0.3
    r = oracle.logcdf(locs, x, 1, EXP, 0.5, 1.0, rho_cov, 0.0, 2, 2048, 8, 21)
    perm, nbrs = r["perm"], r["nbrs"]
    s = locs[perm]
    for i in range(1, 25):
        j = int(nbrs[i][0])
        h = math.hypot(*(s[i] - s[j]))
        corr = math.exp(-h / rho_cov)
        b1, b2 = x[perm[j]], x[perm[i]]
        want = math.log(cf.bivariate_cdf(b1, b2, corr) / ndtr(b1))
        lt, se = r["terms"][perm[i]]
        assert abs(lt - want) <= 4 * se + 1e-9, (i, lt, want, se)


def test_sheppard_orthant():
    for corr in (-0.6, 0.2, 0.9):
        C = np.array([[1.0, corr], [corr, 1.0]])
        lt, se = sov.term_estimate(C, np.zeros(2), 4096, 8, 5, 0)
        want = math.log(cf.sheppard(corr) / 0.5)
        assert abs(lt - want) <= 4 * se + 1e-9


def test_trivariate_orthant_exact_vecchia():
    # D = 3, m = 2 = D - 1: the Vecchia product is the exact telescoping product
    pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
    C = _exp_cov(pts, 0.4)
    nbrs = [[], [0], [0, 1]]
    r = oracle.logcdf_from_cov(C, np.zeros(3), nbrs, 8192, 10, 3)
    want = math.log(cf.orthant3(C[0, 1], C[0, 2], C[1, 2]))
    assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-9
    assert abs(r["logF"] - want) < 1e-4


@pytest.mark.parametrize("D,m", [(6, 5), (12, 3), (20, 8)])
def test_equicorrelated_half_orthant(D, m):
    # rho = 1/2, b = 0: Phi_n(0) = 1/(n+1), so term i = (k_i+1)/(k_i+2)
    Sigma = 0.5 * np.eye(D) + 0.5
    nbrs = [list(range(max(0, i - m), i))[::-1] for i in range(D)]
    r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 4096, 8, 17)
    for i in range(D):
        k = min(m, i)
        want = math.log((k + 1) / (k + 2))
        lt, se = r["terms"][i]
        assert abs(lt - want) <= 4 * se + 1e-9, (i, lt, want, se)
    if m == D - 1:
        assert abs(r["logF"] + math.log(D + 1)) <= 4 * r["se"] + 1e-9


def test_equicorrelated_general_thresholds():
    D, m, rho = 10, 4, 0.3
    Sigma = (1 - rho) * np.eye(D) + rho
    x = np.random.default_rng(4).normal(0.5, 1.0, size=D)
    nbrs = [list(range(max(0, i - m), i)) for i in range(D)]
    r = oracle.logcdf_from_cov(Sigma, x, nbrs, 4096, 8, 23)
    for i in range(1, D):
        v = nbrs[i] + [i]
        want = math.log(cf.equicorrelated_cdf(x[v], rho) / cf.equicorrelated_cdf(x[v[:-1]], rho))
        lt, se = r["terms"][i]
        assert abs(lt - want) <= 4 * se + 1e-9, (i, lt, want, se)


def test_scale_divides_thresholds():
    Sigma = 0.6 * np.eye(4) + 0.4
    nbrs = [[], [0], [1, 0], [2, 1]]
    x = np.array([1.0, 0.5, 2.0, -0.3])
    a = oracle.logcdf_from_cov(Sigma, x, nbrs, 512, 4, 3, scale=2.5)
    b = oracle.logcdf_from_cov(Sigma, x / 2.5, nbrs, 512, 4, 3)
    assert a["logF"] == b["logF"]


@pytest.mark.slow
def test_exact_case_against_brute_force_monte_carlo():
    # m = D - 1 makes eq. (6) the exact telescoping product of eq. (5)
    rng = np.random.default_rng(12)
    pts = rng.random((5, 2))
    C = covariance.cov_matrix(pts, covariance.COV_MATERN, 1.5, 1.0, 0.3, 0.0)
    x = rng.normal(0.2, 0.6, size=5)
    nbrs = [list(range(i)) for i in range(5)]
    r = oracle.logcdf_from_cov(C, x, nbrs, 8192, 10, 31)
    p, se_p = cf.monte_carlo_cdf(C, x, 4_000_000, 77)
    tol = 4.0 * math.hypot(r["se"], se_p / p)
    assert abs(r["logF"] - math.log(p)) <= tol, (r["logF"], math.log(p), tol)


def test_se_coverage_over_seeds():
    # the delta-method SE is an honest error bar: ~95% of seeds land within 2 SE
    D, m, rho = 5, 4, 0.5
    Sigma = (1 - rho) * np.eye(D) + rho
    nbrs = [list(range(i)) for i in range(D)]
    want = -math.log(D + 1)
    inside = 0
    n_seeds = 60
    for seed in range(n_seeds):
        r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 1000 + seed)
        inside += abs(r["logF"] - want) <= 2 * r["se"]
    assert inside >= 0.8 * n_seeds
    assert inside <= n_seeds            # (and the SE is not absurdly wide:)
    r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 5)
    assert r["se"] < 0.05


def test_not_positive_definite_is_reported():
    C = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(sov.NotPositiveDefinite):
        sov.term_estimate(C, np.zeros(2), 64, 2, 1, 0)


def test_single_shift_has_no_se():
    C = np.array([[1.0, 0.5], [0.5, 1.0]])
    lt, se = sov.term_estimate(C, np.zeros(2), 256, 1, 1, 0)
    assert math.isfinite(lt) and math.isnan(se)
