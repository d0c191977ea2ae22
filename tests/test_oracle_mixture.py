"""Pins of the scale-mixture oracle (Section 4, eqs. (8)-(9)): the quadrature
rule against closed forms, an adaptive library integrator and limits."""
import math
import warnings

import numpy as np
import pytest
from scipy import integrate
from scipy.special import log_ndtr

import oracle
from oracle import mixture as M

FAMILIES = [(0.0, 2.0), (0.0, 0.7), (0.5, 1.0), (1.0, 3.0), (2.0, 0.5)]


def _reference_logG(logF_of_r, beta, gamma, mu):
    """int_0^inf e^-v Phi_D(x / r(v)) dv by adaptive quadrature (scipy quad)."""
    def f(v):
        val = -v + logF_of_r(M.scale_at(v, beta, gamma))
        return math.exp(val) if val > -745.0 else 0.0
    b = 30.0 / mu
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        a1 = integrate.quad(f, 0.0, b, epsabs=0.0, epsrel=1e-13, limit=1000)[0]
        a2 = integrate.quad(f, b, 800.0, epsabs=0.0, epsrel=1e-13, limit=1000)[0]
    return math.log(a1 + a2)


def test_scale_map_is_the_inverse_cdf_of_eq8():
    # v = -log(1 - F_R(r)) for the two branches of eq. (8) (beta = 0 read as Pareto)
    for beta, gamma in FAMILIES:
        for v in (0.0, 1e-3, 0.7, 3.0, 20.0):
            r = M.scale_at(v, beta, gamma)
            assert r >= 1.0
            # log of the survival function 1 - F_R(r), written without cancellation
            if beta == 0.0:
                log_surv = -gamma * math.log(r)
            else:
                log_surv = -gamma * math.expm1(beta * math.log(r)) / beta
            assert abs(-log_surv - v) <= 1e-12 * max(1.0, v)


@pytest.mark.parametrize("beta,gamma", FAMILIES)
def test_zero_thresholds_give_the_unmixed_orthant_exactly(beta, gamma):
    # Phi_D(0 / r) does not depend on r, so G(0) = Phi_D(0) for every F_R and the
    # rule (mu = 1, weights summing to 1) returns the node value to rounding
    c = math.log(1.0 / 8.0 + (math.asin(0.3) + math.asin(0.5) + math.asin(0.2)) / (4.0 * math.pi))
    res = M.logcdf_mixture(lambda r: (c, 0.01), beta, gamma, 32)
    assert res["mu"] == 1.0
    assert abs(res["logG"] - c) <= 1e-14
    assert abs(res["se"] - 0.01 * math.sqrt(np.sum(np.polynomial.laguerre.laggauss(32)[1] ** 2))) < 1e-15


def test_zero_thresholds_through_the_vecchia_oracle():
    # trivariate orthant, m = D-1 (Vecchia exact): G(0) equals the estimator's
    # Phi_3(0), which is within a few SE of 1/8 + sum asin(rho) / (4 pi)
    S = np.array([[1.0, 0.3, 0.5], [0.3, 1.0, 0.2], [0.5, 0.2, 1.0]])
    nb = [[], [0], [0, 1]]
    x = np.zeros(3)
    ev = lambda r: (lambda d: (d["logF"], d["se"]))(oracle.vecchia.logcdf_from_cov(S, x, nb, 4096, 8, 5, scale=r))
    res = M.logcdf_mixture(ev, 0.0, 2.0, 16)
    base = oracle.vecchia.logcdf_from_cov(S, x, nb, 4096, 8, 5)
    assert abs(res["logG"] - base["logF"]) <= 1e-14
    exact = math.log(1.0 / 8.0 + (math.asin(0.3) + math.asin(0.5) + math.asin(0.2)) / (4.0 * math.pi))
    assert abs(res["logG"] - exact) <= 4.0 * res["se"] + 1e-12


@pytest.mark.parametrize("beta,gamma", FAMILIES)
@pytest.mark.parametrize("D,tol", [(1, 1e-7), (50, 1e-9), (2000, 1e-11)])
def test_independent_components_against_adaptive_quadrature(beta, gamma, D, tol):
    # diagonal covariance: Phi_D(x / r) = prod Phi(x_i / r) exactly, so eq. (9) is a
    # one-dimensional integral that scipy's adaptive rule evaluates independently
    x = np.random.default_rng(D).normal(1.5, 0.5, D)
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 32)
    ref = _reference_logG(logF, beta, gamma, res["mu"])
    assert abs(res["logG"] - ref) <= tol * max(1.0, abs(ref)), (res["logG"], ref)


def test_negative_thresholds_rising_integrand():
    # x < 0: Phi_D(x / r) grows with r, mu stays 1 and the rule still converges
    x = np.array([-1.0, -0.4, -2.0])
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    for beta, gamma in FAMILIES:
        res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 32)
        assert res["mu"] == 1.0
        ref = _reference_logG(logF, beta, gamma, 1.0)
        assert abs(res["logG"] - ref) <= 1e-5 * abs(ref)


def test_point_mass_limit():
    # gamma -> infinity puts R at 1: G -> Phi_D(x)
    x = np.array([0.5, 1.2, 2.0, -0.3])
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    for beta in (0.0, 1.0):
        res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, 1e8, 32)
        assert abs(res["logG"] - logF(1.0)) <= 1e-6


def test_se_propagation_first_order():
    # a single dominant node passes its SE through; equal nodes combine in quadrature
    x = np.full(2000, 1.5)
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    res = M.logcdf_mixture(lambda r: (logF(r), 0.02), 0.0, 2.0, 32)
    t, w = np.polynomial.laguerre.laggauss(32)
    assert 0.0 < res["se"] <= 0.02 + 1e-15
    assert res["se"] >= 0.02 * math.sqrt(np.sum(w ** 2)) - 1e-15


MIXTURE_MUTATIONS = {
    "pareto_exponent_inverted": ("s = v / gamma if beta == 0.0", "s = v * gamma if beta == 0.0"),
    "missing_jacobian_1_over_mu": ("np.log(w) - math.log(mu) + t", "np.log(w) + t"),
    "missing_weight_correction": ("+ t * (1.0 - 1.0 / mu)", "+ 0.0 * t"),
    "nodes_not_rescaled": ("scale_at(float(tk) / mu, beta, gamma)", "scale_at(float(tk), beta, gamma)"),
    "slope_sign": ("-(h1 - h0) / DELTA", "(h1 - h0) / DELTA"),
}


@pytest.mark.parametrize("name", ["none"] + sorted(MIXTURE_MUTATIONS))
def test_planted_mixture_mistakes_fail_a_pin(name):
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(M.__file__), "mixture.py")
    src = open(path).read()
    if name != "none":
        old, new = MIXTURE_MUTATIONS[name]
        assert old in src
        src = src.replace(old, new)
    spec = importlib.util.spec_from_loader("oracle._mutant_mixture", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src, path, "exec"), mod.__dict__)
    ok = True
    for beta, gamma in ((0.0, 2.0), (1.0, 3.0)):
        for D in (1, 50, 2000):
            x = np.random.default_rng(D).normal(1.5, 0.5, D)
            logF = lambda r: float(np.sum(log_ndtr(x / r)))
            res = mod.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 32)
            ref = _reference_logG(logF, beta, gamma, max(1.0, res["mu"]))
            ok = ok and abs(res["logG"] - ref) <= 1e-7 * max(1.0, abs(ref))
    assert ok == (name == "none"), name
