"""Pins of the censored-likelihood oracle (Section 4, eq. (11)) against closed
forms, library routines, an integral identity and a Markov special case."""
import importlib.util
import math
import os
import warnings

import numpy as np
import pytest
from scipy import integrate
from scipy.special import log_ndtr
from scipy.stats import multivariate_normal, norm

import oracle
from oracle import censored as CZ
from oracle import covariance
from oracle import mixture as M
from tests import closed_forms as cf


def _all_preceding(D):
    return [list(range(i)) for i in range(D)]


def _geometry_cov(pts, rho=0.4, sigma2=1.0):
    return covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, sigma2, rho, 0.0)


# ---------------------------------------------------------------- plan -----

def test_plan_puts_observed_sites_first_in_base_order():
    rng = np.random.default_rng(11)
    locs = rng.random((60, 2))
    obs = rng.random(60) < 0.2
    perm, nbrs, n_obs = CZ.censored_plan(locs, obs, oracle.ordering.ORDER_MAXMIN, 5)
    base = oracle.ordering.maxmin_order(locs)
    assert n_obs == int(obs.sum())
    assert np.array_equal(perm[:n_obs], [v for v in base if obs[v]])
    assert np.array_equal(perm[n_obs:], [v for v in base if not obs[v]])
    for i in range(n_obs):
        assert np.all(nbrs[i] < n_obs)   # an observed site conditions on observed sites only


# ------------------------------------------------------- special cases -----

def test_no_observed_sites_is_the_plain_logcdf():
    rng = np.random.default_rng(3)
    locs = rng.random((40, 2))
    x = rng.normal(1.0, 0.4, 40)
    args = (locs, x)
    kw = dict(m=6, family=1, nu=1.5, sigma2=1.0, rho=0.15, nugget=0.0, rule=2, n_points=512,
              n_shifts=4, seed=9)
    a = CZ.loglik(*args, np.zeros(40, bool), **kw)
    b = oracle.logcdf(*args, **kw)
    assert a["logL"] == b["logF"] and a["se"] == b["se"]
    assert np.array_equal(a["terms"], b["terms"])


@pytest.mark.parametrize("scale", [1.0, 1.7])
def test_all_observed_exact_vecchia_is_the_gaussian_logpdf(scale):
    # m = D - 1: the Vecchia density is the joint density (eq. (3)); at scale r
    # the integrand is phi_D(x / r) r^-D (library logpdf)
    rng = np.random.default_rng(5)
    pts = rng.random((7, 2))
    x = rng.normal(0.5, 1.0, 7)
    res = CZ.loglik(pts, x, np.ones(7, bool), 6, 0, 0.5, 1.3, 0.5, 0.01, 1, 64, 2, 1, scale=scale)
    S = covariance.cov_matrix(pts, 0, 0.5, 1.3, 0.5, 0.01)
    want = multivariate_normal(np.zeros(7), S).logpdf(x / scale) - 7 * math.log(scale)
    assert abs(res["logL"] - want) <= 1e-11 * abs(want)
    assert res["se"] == 0.0


@pytest.mark.parametrize("m", [1, 3])
def test_markov_transect_density_is_exact_at_small_m(m):
    # exponential covariance on a line is Markov (Ornstein-Uhlenbeck): ordered by
    # position, conditioning on the previous site only is exact, so the Vecchia
    # density with m >= 1 equals the joint density
    rng = np.random.default_rng(7)
    xs = np.sort(rng.random(40)) * 4.0
    pts = np.stack([xs, np.zeros(40)], axis=1)
    x = rng.normal(0.0, 1.2, 40)
    res = CZ.loglik(pts, x, np.ones(40, bool), m, 0, 0.5, 2.0, 0.7, 0.0, 1, 64, 2, 1)
    want = multivariate_normal(np.zeros(40), _geometry_cov(pts, 0.7, 2.0)).logpdf(x)
    assert abs(res["logL"] - want) <= 1e-10 * abs(want)


def test_equicorrelated_exact_vecchia_matches_one_factor_form():
    # Sigma = (1-rho) I + rho 1 1^T with the first n_I variables observed. Given
    # X_I = x_I the censored ones have mean rho / (1 + (n_I - 1) rho) sum x_I and
    # covariance (1-rho) I + rho (1-rho) / (1 + (n_I - 1) rho) 1 1^T, so eq. (11)'s
    # integrand is a library logpdf times a one-factor 1-D integral
    D, n_I, rho = 8, 3, 0.4
    Sigma = (1 - rho) * np.eye(D) + rho
    x = np.array([1.9, 2.4, 1.7, 0.9, 1.2, 0.4, 1.0, 1.5])
    res = CZ.loglik_from_cov(Sigma, x, n_I, _all_preceding(D), 4096, 8, 13)
    den = 1.0 + (n_I - 1) * rho
    mu = rho / den * x[:n_I].sum()
    a = rho * (1.0 - rho) / den
    logcdf = math.log(cf.one_factor_cdf(x[n_I:] - mu, a, 1.0 - rho))
    want = multivariate_normal(np.zeros(n_I), Sigma[:n_I, :n_I]).logpdf(x[:n_I]) + logcdf
    assert abs(res["logL"] - want) <= 4.0 * res["se"] + 1e-10, (res["logL"], want, res["se"])
    assert res["se"] < 1e-3


def test_bivariate_integral_identity():
    # int_{-inf}^{x0} dPhi_2(t, x1) / dt dt = Phi_2(x0, x1): the one-observed
    # likelihood of D = 2 integrated over the observed value is the CDF (Owen's T)
    for x0, x1, rho in [(0.8, -0.3, 0.6), (-0.4, 1.1, -0.5), (1.5, 0.7, 0.9)]:
        S = np.array([[1.0, rho], [rho, 1.0]])
        f = lambda t: math.exp(CZ.loglik_from_cov(S, [t, x1], 1, [[], [0]], 64, 2, 1)["logL"])
        val, _ = integrate.quad(f, -np.inf, x0, epsabs=1e-14, epsrel=1e-12, limit=200)
        assert abs(val - cf.bivariate_owen(x0, x1, rho)) <= 1e-11


def test_trivariate_integral_identity_at_the_orthant():
    # int_{-inf}^0 dPhi_3(t, 0, 0) / dt dt = 1/8 + sum asin / (4 pi); the last
    # censored term is a QMC estimate (common random numbers in t), so the bar is
    # its relative SE
    pts = np.array([[0.0, 0.0], [0.3, 0.1], [0.1, 0.35]])
    S = _geometry_cov(pts, 0.6)
    ses = []

    def f(t):
        r = CZ.loglik_from_cov(S, [t, 0.0, 0.0], 1, _all_preceding(3), 8192, 8, 21)
        ses.append(r["se"])
        return math.exp(r["logL"])

    val, _ = integrate.quad(f, -np.inf, 0.0, epsabs=1e-12, epsrel=1e-10, limit=200)
    want = cf.orthant3(S[0, 1], S[0, 2], S[1, 2])
    assert abs(val / want - 1.0) <= 4.0 * max(ses) + 1e-9, (val, want, max(ses))


def test_mixed_sites_exact_vecchia_any_ordering():
    # m = D - 1 makes L exact whatever the ordering (up to the QMC error of the
    # one censored term with a censored neighbour); observed sites 1 and 3 (not a
    # prefix): logpdf of the observed pair plus Owen's bivariate CDF of the
    # textbook conditional Gaussian of the censored pair
    pts = np.array([[0.0, 0.0], [0.25, 0.05], [0.1, 0.3], [0.4, 0.35]])
    S = _geometry_cov(pts, 0.5)
    x = np.array([0.7, 1.8, -0.2, 2.1])
    obs = np.array([False, True, False, True])
    I, C = [1, 3], [0, 2]
    mu = S[np.ix_(C, I)] @ np.linalg.inv(S[np.ix_(I, I)]) @ x[I]
    Sc = S[np.ix_(C, C)] - S[np.ix_(C, I)] @ np.linalg.inv(S[np.ix_(I, I)]) @ S[np.ix_(I, C)]
    sd = np.sqrt(np.diag(Sc))
    y = (x[C] - mu) / sd
    want = (multivariate_normal(np.zeros(2), S[np.ix_(I, I)]).logpdf(x[I])
            + math.log(cf.bivariate_owen(y[0], y[1], Sc[0, 1] / (sd[0] * sd[1]))))
    for rule, perm in ((1, None), (2, None), (0, np.array([2, 0, 3, 1]))):
        res = CZ.loglik(pts, x, obs, 3, 0, 0.5, 1.0, 0.5, 0.0, rule, 4096, 8, 1, perm=perm)
        assert res["n_obs"] == 2
        assert 0.0 < res["se"] < 1e-4
        assert abs(res["logL"] - want) <= 4.0 * res["se"] + 1e-12, (rule, res["logL"], want, res["se"])


# --------------------------------------------------------- scale mixture ---

def _reference_logG(logL_of_r, beta, gamma):
    from tests.test_oracle_mixture import _reference_logG as ref
    return ref(logL_of_r, beta, gamma)


@pytest.mark.parametrize("beta,gamma", [(0.0, 2.0), (0.82, 1.0), (2.0, 0.5)])
def test_censored_mixture_with_independent_sites(beta, gamma):
    # diagonal covariance: L_r = prod_I phi(x_i / r) / r * prod_c Phi(x_c / r), so
    # G_I = int L_r f_R(r) dr is a 1-D integral for an adaptive library rule
    D, n_I = 30, 4
    rng = np.random.default_rng(17)
    x = np.concatenate([rng.uniform(2.0, 3.5, n_I), np.full(D - n_I, 1.64)])
    ev = lambda r: (lambda d: (d["logL"], d["se"]))(
        CZ.loglik_from_cov(np.eye(D), x, n_I, [list(range(max(0, i - 3), i)) for i in range(D)], 64, 2, 1,
                           scale=r))
    res = M.logcdf_mixture(ev, beta, gamma, 48)
    exact = lambda r: float(np.sum(norm.logpdf(x[:n_I] / r)) - n_I * math.log(r) + np.sum(log_ndtr(x[n_I:] / r)))
    assert abs(ev(1.3)[0] - exact(1.3)) <= 1e-12 * abs(exact(1.3))
    ref = _reference_logG(exact, beta, gamma)
    # 48-node rule: ~5e-7 relative at worst over these families (beta = 2, a bulk
    # near v = 0 with a long tail), far below the QMC error of a node
    assert abs(res["logG"] - ref) <= 1e-6 * abs(ref), (res["logG"], ref)


# ------------------------------------------------------ planted mistakes ---

CENSORED_MUTATIONS = {
    "mean_shift_dropped": ("mu = CAE @ np.linalg.solve(CEE, b[E])", "mu = 0.0 * (CAE @ np.linalg.solve(CEE, b[E]))"),
    "mean_shift_sign": ("b[A] - mu, n_points", "b[A] + mu, n_points"),
    "unconditioned_covariance": ("S = C[np.ix_(A, A)] - CAE", "S = C[np.ix_(A, A)] + 0.0 * CAE"),
    "missing_jacobian": ("- 0.5 * z * z - math.log(scale), 0.0)", "- 0.5 * z * z, 0.0)"),
    "sd_for_variance": ("-0.5 * (LOG_2PI + math.log(var))", "-0.5 * LOG_2PI - math.log(var)"),
    "censored_sites_first": ("np.concatenate([first, rest])", "np.concatenate([rest, first])"),
    "density_conditions_on_nothing": ("np.append(eq[:-1], False)", "np.zeros(len(eq), bool)"),
}


def _pins_pass(mod) -> bool:
    checks = []
    try:
        # reuse the pins above on the edited module
        g = globals()
        g["CZ"] = mod
        for fn, args in ((test_all_observed_exact_vecchia_is_the_gaussian_logpdf, (1.7,)),
                         (test_markov_transect_density_is_exact_at_small_m, (1,)),
                         (test_equicorrelated_exact_vecchia_matches_one_factor_form, ()),
                         (test_bivariate_integral_identity, ()),
                         (test_mixed_sites_exact_vecchia_any_ordering, ()),
                         (test_censored_mixture_with_independent_sites, (0.0, 2.0))):
            try:
                fn(*args)
                checks.append(True)
            except (AssertionError, ValueError, FloatingPointError, np.linalg.LinAlgError,
                    oracle.sov.NotPositiveDefinite):
                checks.append(False)
    finally:
        globals()["CZ"] = CZ_REAL
    return all(checks)


CZ_REAL = CZ


@pytest.mark.parametrize("name", ["none"] + sorted(CENSORED_MUTATIONS))
def test_planted_censored_mistakes_fail_a_pin(name):
    path = os.path.join(os.path.dirname(CZ_REAL.__file__), "censored.py")
    src = open(path).read()
    if name != "none":
        old, new = CENSORED_MUTATIONS[name]
        assert old in src, old
        src = src.replace(old, new)
    spec = importlib.util.spec_from_loader("oracle._mutant_censored", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src, path, "exec"), mod.__dict__)
    with np.errstate(all="ignore"):
        assert _pins_pass(mod) == (name == "none"), name
