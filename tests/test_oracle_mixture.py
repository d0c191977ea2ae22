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


BREAKS = [0.0, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 0.1, 1.0, 3.0, 10.0, 30.0, 2000.0]


def _reference_logG(logF_of_r, beta, gamma):
    """int_0^inf e^-v Phi_D(x / r(v)) dv by adaptive quadrature (scipy quad) over
    fixed pieces from 1e-6 to 2000, scaled by the integrand's largest sampled value."""
    ell = lambda v: -v + logF_of_r(M.scale_at(v, beta, gamma))
    peak = max(ell(v) for v in np.concatenate([[0.0], np.geomspace(1e-7, 2000.0, 400)]))

    def f(v):
        val = ell(v) - peak
        return math.exp(val) if val > -745.0 else 0.0
    total = 0.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for a, b in zip(BREAKS[:-1], BREAKS[1:]):
            total += integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=2000)[0]
    return peak + math.log(total)


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
    # Phi_D(0 / r) does not depend on r, so G(0) = Phi_D(0) for every F_R; the
    # window is [0, v] with e^-v < e^-36, and 48-point Gauss-Legendre integrates
    # e^-v over it to 1e-13; equal node SEs combine to at most that SE
    c = math.log(1.0 / 8.0 + (math.asin(0.3) + math.asin(0.5) + math.asin(0.2)) / (4.0 * math.pi))
    res = M.logcdf_mixture(lambda r: (c, 0.01), beta, gamma, 48)
    assert res["window"][0] == 0.0 and res["window"][1] >= 36.0
    assert abs(res["logG"] - c) <= 1e-12
    assert 0.01 / math.sqrt(48) <= res["se"] <= 0.01


def test_zero_thresholds_through_the_vecchia_oracle():
    # trivariate orthant, m = D-1 (Vecchia exact): G(0) equals the estimator's
    # Phi_3(0), which is within a few SE of 1/8 + sum asin(rho) / (4 pi)
    S = np.array([[1.0, 0.3, 0.5], [0.3, 1.0, 0.2], [0.5, 0.2, 1.0]])
    nb = [[], [0], [0, 1]]
    x = np.zeros(3)
    ev = lambda r: (lambda d: (d["logF"], d["se"]))(oracle.vecchia.logcdf_from_cov(S, x, nb, 4096, 8, 5, scale=r))
    res = M.logcdf_mixture(ev, 0.0, 2.0, 48)
    base = oracle.vecchia.logcdf_from_cov(S, x, nb, 4096, 8, 5)
    assert abs(res["logG"] - base["logF"]) <= 1e-12
    exact = math.log(1.0 / 8.0 + (math.asin(0.3) + math.asin(0.5) + math.asin(0.2)) / (4.0 * math.pi))
    assert abs(res["logG"] - exact) <= 4.0 * res["se"] + 1e-12


@pytest.mark.parametrize("beta,gamma", FAMILIES)
@pytest.mark.parametrize("D,tol", [(1, 1e-7), (50, 1e-7), (2000, 1e-11)])
def test_independent_components_against_adaptive_quadrature(beta, gamma, D, tol):
    # diagonal covariance: Phi_D(x / r) = prod Phi(x_i / r) exactly, so eq. (9) is a
    # one-dimensional integral that scipy's adaptive rule evaluates independently
    x = np.random.default_rng(D).normal(1.5, 0.5, D)
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 48)
    ref = _reference_logG(logF, beta, gamma)
    assert abs(res["logG"] - ref) <= tol * max(1.0, abs(ref)), (res["logG"], ref)


def test_negative_thresholds_rising_integrand():
    # x < 0: Phi_D(x / r) grows with r, mu stays 1 and the rule still converges
    x = np.array([-1.0, -0.4, -2.0])
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    for beta, gamma in FAMILIES:
        res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 48)
        ref = _reference_logG(logF, beta, gamma)
        assert abs(res["logG"] - ref) <= 1e-7 * abs(ref)


def test_point_mass_limit():
    # gamma -> infinity puts R at 1: G -> Phi_D(x)
    x = np.array([0.5, 1.2, 2.0, -0.3])
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    for beta in (0.0, 1.0):
        res = M.logcdf_mixture(lambda r: (logF(r), 0.0), beta, 1e8, 48)
        assert abs(res["logG"] - logF(1.0)) <= 1e-6


def test_se_propagation_first_order():
    # a single dominant node passes its SE through; equal nodes combine in quadrature
    x = np.full(2000, 1.5)
    logF = lambda r: float(np.sum(log_ndtr(x / r)))
    res = M.logcdf_mixture(lambda r: (logF(r), 0.02), 0.0, 2.0, 48)
    assert 0.0 < res["se"] <= 0.02 + 1e-15
    assert res["se"] >= 0.02 / math.sqrt(48) - 1e-15


def test_search_grid_and_window_rule():
    # the search points span 1e-4 .. 200 geometrically after v = 0, and for a
    # unimodal l the window brackets every point within 36 of the search maximum
    v = M.search_v()
    assert len(v) == 24 and v[0] == 0.0 and abs(v[1] - 1e-4) < 1e-19 and abs(v[-1] - 200.0) < 1e-12
    ratios = np.array(v[2:]) / np.array(v[1:-1])
    assert np.allclose(ratios, ratios[0], rtol=1e-13)
    rng = np.random.default_rng(4)
    for _ in range(200):
        j0, c, p = rng.integers(0, 24), rng.uniform(0.5, 40.0), rng.uniform(0.5, 2.5)
        ell = -c * np.abs(np.arange(24) - j0) ** p + rng.normal(0.0, 50.0)
        lo, hi = M.window(ell + np.array(v))
        top = ell.max()
        inside = [vj for vj, e in zip(v, ell) if e >= top - M.CUT]
        assert lo <= min(inside) and hi >= max(inside)
    assert M.search_n_points(10000) == 640 and M.search_n_points(100) == 64 and M.search_n_points(1024) == 64


def test_censored_shape_against_adaptive_quadrature():
    # an interior bulk (a censored likelihood: density factors rising with r, then
    # the r^-|I| Jacobian): l(v) peaks inside (0, inf)
    xI = np.array([2.3, 3.1, 2.7, 3.4])
    from scipy.stats import norm
    logh = lambda r: float(np.sum(norm.logpdf(xI / r)) - 4 * math.log(r) + 26 * log_ndtr(1.64 / r))
    xJ = np.random.default_rng(26).uniform(3.0, 8.0, 26)
    narrow = lambda r: float(np.sum(norm.logpdf(xJ / r)) - 26 * math.log(r) + 330 * log_ndtr(3.0 / r))
    for beta, gamma in FAMILIES:
        for f in (logh, narrow):
            res = M.logcdf_mixture(lambda r: (f(r), 0.0), beta, gamma, 48)
            ref = _reference_logG(f, beta, gamma)
            assert abs(res["logG"] - ref) <= 1e-5 * abs(ref), (beta, gamma, res["logG"], ref)
    # the narrow bulk sits away from v = 0; for some families its window spans
    # more than a factor 8 and the rule uses the log map there
    wins = [M.logcdf_mixture(lambda r: (narrow(r), 0.0), b, g, 48)["window"] for b, g in FAMILIES]
    assert all(lo > 0.0 for lo, hi in wins)
    assert any(hi / lo > M.LOG_SPAN for lo, hi in wins) and any(hi / lo <= M.LOG_SPAN for lo, hi in wins)


MIXTURE_MUTATIONS = {
    "pareto_exponent_inverted": ("s = v / gamma if beta == 0.0", "s = v * gamma if beta == 0.0"),
    "missing_exp_minus_v": ("logw = np.log(w * (hi - lo) / 2.0) - v", "logw = np.log(w * (hi - lo) / 2.0)"),
    "log_map_jacobian_dropped": ("np.log(w * (b - a) / 2.0) + s - v", "np.log(w * (b - a) / 2.0) - v"),
    "half_length_dropped": ("np.log(w * (hi - lo) / 2.0) - v", "np.log(w * (hi - lo)) - v"),
    "cut_too_tight": ("CUT = 36.0", "CUT = 3.0"),
    "window_from_log_h_only": ("ell = [float(h) - vj for", "ell = [float(h) + 0.0 * vj for"),
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
    from scipy.stats import norm
    xI = np.array([2.3, 3.1, 2.7, 3.4])
    cens = lambda r: float(np.sum(norm.logpdf(xI / r)) - 4 * math.log(r) + 26 * log_ndtr(1.64 / r))
    xJ = np.random.default_rng(26).uniform(3.0, 8.0, 26)
    narrow = lambda r: float(np.sum(norm.logpdf(xJ / r)) - 26 * math.log(r) + 330 * log_ndtr(3.0 / r))
    ok = True
    for beta, gamma in ((0.0, 2.0), (1.0, 3.0), (2.0, 0.5)):
        cases = []
        for D in (1, 50, 2000):
            x = np.random.default_rng(D).normal(1.5, 0.5, D)
            cases.append(lambda r, x=x: float(np.sum(log_ndtr(x / r))))
        cases += [cens, narrow]
        for logF in cases:
            res = mod.logcdf_mixture(lambda r: (logF(r), 0.0), beta, gamma, 48)
            ref = _reference_logG(logF, beta, gamma)
            ok = ok and abs(res["logG"] - ref) <= 1e-5 * max(1.0, abs(ref))
    assert ok == (name == "none"), name
