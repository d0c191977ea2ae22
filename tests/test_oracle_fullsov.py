"""Pins of the full-dimension SOV oracle (the paper's comparator, Section 3.1)
against closed forms, brute force and the Vecchia oracle at m = D - 1."""
import importlib.util
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import log_ndtr, ndtr
from scipy.stats import norm

import oracle
from oracle import covariance
from oracle import fullsov as FS
from tests import closed_forms as cf


def _log_one_factor(b, rho):
    """log int phi(z) prod Phi((b - sqrt(rho) z) / sqrt(1 - rho)) dz, in log space
    around the integrand's peak (no underflow for large D)."""
    b = np.asarray(b, dtype=np.float64)
    sr, sq = math.sqrt(rho), math.sqrt(1.0 - rho)
    lf = lambda z: float(norm.logpdf(z) + np.sum(log_ndtr((b - sr * z) / sq)))
    zs = np.linspace(-12.0, 12.0, 4801)
    vals = np.array([lf(z) for z in zs])
    top = vals.max()
    val, _ = integrate.quad(lambda z: math.exp(lf(z) - top), -14.0, 14.0, epsabs=0.0, epsrel=1e-12, limit=500,
                            points=[float(zs[np.argmax(vals)])])
    return top + math.log(val)


def test_one_dimension_is_exact():
    lf, se, _ = FS.logcdf_full(np.array([[2.0]]), np.array([0.7]), 64, 4, 1)
    assert abs(lf - float(log_ndtr(0.7 / math.sqrt(2.0)))) <= 1e-15 and se == 0.0


def test_diagonal_covariance_is_exact():
    b = np.linspace(-2.0, 2.5, 30)
    lf, se, _ = FS.logcdf_full(np.diag(np.linspace(0.5, 2.0, 30)), b, 128, 4, 3)
    want = float(np.sum(log_ndtr(b / np.sqrt(np.linspace(0.5, 2.0, 30)))))
    assert abs(lf - want) <= 1e-12 * abs(want) and se <= 1e-13


def test_trivariate_orthant():
    pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
    S = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 1.0, 0.4, 0.0)
    lf, se, _ = FS.logcdf_full(S, np.zeros(3), 8192, 8, 5)
    want = math.log(cf.orthant3(S[0, 1], S[0, 2], S[1, 2]))
    assert abs(lf - want) <= 4 * se + 1e-12 and se < 1e-4


@pytest.mark.parametrize("D,rho,x0", [(12, 0.4, 0.3), (200, 0.5, -1.0)])
def test_equicorrelated_one_factor_form(D, rho, x0):
    # D = 200 at negative thresholds: log F about -100, the products would
    # underflow without the log-space accumulation
    rng = np.random.default_rng(D)
    b = x0 + rng.normal(0.0, 0.3, D)
    lf, se, _ = FS.logcdf_full((1 - rho) * np.eye(D) + rho, b, 2048, 8, 7)
    want = _log_one_factor(b, rho)
    assert abs(lf - want) <= 4 * se + 1e-9 * abs(want), (lf, want, se)


def test_brute_force_monte_carlo():
    rng = np.random.default_rng(4)
    pts = rng.random((4, 2))
    S = covariance.cov_matrix(pts, covariance.COV_MATERN, 1.5, 1.0, 0.3, 0.0)
    b = np.array([0.4, -0.2, 1.0, 0.1])
    lf, se, _ = FS.logcdf_full(S, b, 4096, 8, 9)
    p, pse = cf.monte_carlo_cdf(S, b, 4_000_000, 17)
    assert abs(math.exp(lf) - p) <= 4 * math.sqrt((se * math.exp(lf)) ** 2 + pse ** 2)


def test_agrees_with_the_vecchia_oracle_at_m_d_minus_1():
    # two different estimators of the same exact CDF
    rng = np.random.default_rng(6)
    pts = rng.random((25, 2))
    S = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 1.0, 0.3, 1e-8)
    b = rng.normal(1.0, 0.5, 25)
    lf, se, _ = FS.logcdf_full(S, b, 4096, 8, 2)
    v = oracle.logcdf_from_cov(S, b, [list(range(i)) for i in range(25)], 4096, 8, 2)
    assert abs(lf - v["logF"]) <= 4 * math.sqrt(se ** 2 + v["se"] ** 2), (lf, v["logF"], se, v["se"])


def test_full_shift_keys():
    from oracle import lattice
    a = {lattice.full_shift(5, r, d) for r in range(4) for d in range(300)}
    assert len(a) == 1200
    assert lattice.full_shift(5, 0, 0) == lattice.splitmix64_output(5, 1 << 63)
    assert lattice.full_shift(5, 3, 7) == lattice.splitmix64_output(5, (1 << 63) | (3 << 32) | 7)


FULL_MUTATIONS = {
    "no_diagonal_scaling": ("t = acc / L[a, a]", "t = acc"),
    "first_factor_dropped": ("lp = log_ndtr(t)\n", "lp = 0.0 * log_ndtr(t)\n"),
    "quantile_without_e": ("ndtri(np.maximum(w * e, DBL_MIN))", "ndtri(np.maximum(w, DBL_MIN))"),
    "sum_not_mean": ("lr[r] = logsumexp(lp) - math.log(n_points)", "lr[r] = logsumexp(lp)"),
    "transposed_factor": ("acc = acc - L[a, :a] @ ys[:a]", "acc = acc - L[:a, a] @ ys[:a]"),
}


@pytest.mark.parametrize("name", ["none"] + sorted(FULL_MUTATIONS))
def test_planted_fullsov_mistakes_fail_a_pin(name):
    path = os.path.join(os.path.dirname(FS.__file__), "fullsov.py")
    src = open(path).read()
    if name != "none":
        old, new = FULL_MUTATIONS[name]
        assert old in src
        src = src.replace(old, new)
    spec = importlib.util.spec_from_loader("oracle._mutant_fullsov", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src, path, "exec"), mod.__dict__)
    ok = True
    pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
    S = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 2.0, 0.4, 0.0)
    lf, se, _ = mod.logcdf_full(S, np.zeros(3), 4096, 8, 5)
    ok = ok and abs(lf - math.log(cf.orthant3(S[0, 1] / 2, S[0, 2] / 2, S[1, 2] / 2))) <= 4 * se + 1e-12
    rng = np.random.default_rng(12)
    b = 0.3 + rng.normal(0.0, 0.3, 12)
    lf, se, _ = mod.logcdf_full(0.6 * np.eye(12) + 0.4, b, 2048, 8, 7)
    ok = ok and abs(lf - _log_one_factor(b, 0.4)) <= 4 * se + 1e-9
    lf, se, _ = mod.logcdf_full(np.diag([2.0, 0.5, 1.0]), np.array([0.3, -0.4, 1.2]), 64, 4, 1)
    ok = ok and abs(lf - float(np.sum(log_ndtr(np.array([0.3, -0.4, 1.2]) / np.sqrt([2.0, 0.5, 1.0]))))) <= 1e-12
    assert ok == (name == "none"), name
