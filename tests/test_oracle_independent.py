"""Pins of the oracle's independent-points estimator (the paper-literal reading
of Section 2.2, where the numerator and the denominator of each term get their
own QM estimate): closed forms within the SE (trivariate orthant, equicorrelated
orthant ratios, the bivariate conditioning integral), SE coverage over seeds,
the exact terms unchanged, the second lattice's points distinct from the
first's, and the shared-points estimator's smaller error bar (the reason it is
the default)."""
import math

import numpy as np
import pytest
from scipy.special import ndtr

import oracle
from oracle import covariance, lattice, sov
from tests import closed_forms as cf

EXP = covariance.COV_EXPONENTIAL


def test_trivariate_orthant_exact_product():
    pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
    C = covariance.cov_matrix(pts, EXP, 0.5, 1.0, 0.4, 0.0)
    r = oracle.logcdf_from_cov(C, np.zeros(3), [[], [0], [0, 1]], 8192, 10, 3, independent=True)
    want = math.log(cf.orthant3(C[0, 1], C[0, 2], C[1, 2]))
    assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-9


@pytest.mark.parametrize("D,m", [(6, 5), (12, 3)])
def test_equicorrelated_half_orthant_terms(D, m):
    Sigma = 0.5 * np.eye(D) + 0.5
    nbrs = [list(range(max(0, i - m), i))[::-1] for i in range(D)]
    r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 4096, 8, 17, independent=True)
    for i in range(D):
        k = min(m, i)
        lt, se = r["terms"][i]
        assert abs(lt - math.log((k + 1) / (k + 2))) <= 4 * se + 1e-9, (i, lt, se)
    assert r["terms"][0, 1] == 0.0       # the exact first term is unchanged


def test_bivariate_conditioning_integral():
    rng = np.random.default_rng(8)
    locs = rng.random((25, 2))
    x = rng.normal(0.3, 0.8, size=25)
    r = oracle.logcdf(locs, x, 1, EXP, 0.5, 1.0, 0.3, 0.0, 2, 2048, 8, 21, independent=True)
    perm, nbrs = r["perm"], r["nbrs"]
    s = locs[perm]
    for i in range(1, 25):
        j = int(nbrs[i][0])
        corr = math.exp(-math.hypot(*(s[i] - s[j])) / 0.3)
        b1, b2 = x[perm[j]], x[perm[i]]
        want = math.log(cf.bivariate_cdf(b1, b2, corr) / ndtr(b1))
        lt, se = r["terms"][perm[i]]
        assert abs(lt - want) <= 4 * se + 1e-9, (i, lt, want, se)


def test_se_coverage_over_seeds():
    D, rho = 5, 0.5
    Sigma = (1 - rho) * np.eye(D) + rho
    nbrs = [list(range(i)) for i in range(D)]
    want = -math.log(D + 1)
    inside = 0
    n_seeds = 60
    for seed in range(n_seeds):
        r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 1000 + seed, independent=True)
        inside += abs(r["logF"] - want) <= 2 * r["se"]
    assert inside >= 0.8 * n_seeds


def test_second_lattice_differs_and_shared_points_have_the_smaller_error_bar():
    # the denominator's points come from other shifts; with shared points the
    # numerator and denominator errors are positively correlated and cancel in
    # the ratio, so the shared estimator's SE is smaller on typical terms
    assert lattice.shift(7, 3, 2, 1) != lattice.shift(7, 3, 2, 1, second=True)
    rng = np.random.default_rng(4)
    locs = rng.random((200, 2))
    x = rng.normal(1.2, 0.3, size=200)
    args = (10, covariance.COV_MATERN, 1.5, 1.0, 0.1, 1e-8, 2, 256, 8, 9)
    a = oracle.logcdf(locs, x, *args)
    b = oracle.logcdf(locs, x, *args, independent=True)
    assert not np.array_equal(a["terms"][:, 0], b["terms"][:, 0])
    ratio = b["terms"][:, 1] / np.where(a["terms"][:, 1] > 0, a["terms"][:, 1], np.nan)
    assert np.nanmedian(ratio) > 1.5
    assert abs(a["logF"] - b["logF"]) <= 4 * math.hypot(a["se"], b["se"])


MUTATIONS = {
    "denominator_from_the_first_lattice": (
        "_, _, den = term_sums(C, b, n_points, n_shifts, seed, term, Z, split, second=True)",
        "_, _, den = term_sums(C, b, n_points, n_shifts, seed, term, Z, split)"),
    "uncentred_relative_variance": ("np.sum((den / dh - 1.0) ** 2)", "np.sum((den / dh) ** 2)"),
    "numerator_variance_dropped": (
        "se2 = (np.sum((num / nh - 1.0) ** 2) + np.sum((den / dh - 1.0) ** 2)) / (R * (R - 1))",
        "se2 = np.sum((den / dh - 1.0) ** 2) / (R * (R - 1))"),
}


def _battery(sov_mod) -> bool:
    orig = oracle.vecchia.sov
    oracle.vecchia.sov = sov_mod
    try:
        D, rho = 5, 0.5
        Sigma = (1 - rho) * np.eye(D) + rho
        nbrs = [list(range(i)) for i in range(D)]
        want = -math.log(D + 1)
        inside = 0
        for seed in range(40):
            r = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 1000 + seed, independent=True)
            if not r["se"] < 0.1:
                return False
            inside += abs(r["logF"] - want) <= 2 * r["se"]
        if inside < 32:
            return False
        a = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 5)
        b = oracle.logcdf_from_cov(Sigma, np.zeros(D), nbrs, 64, 8, 5, independent=True)
        return not np.array_equal(a["terms"][:, 0], b["terms"][:, 0])
    finally:
        oracle.vecchia.sov = orig


def _load(src):
    import importlib.util
    spec = importlib.util.spec_from_loader("oracle._mutant_sov_ind", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src, sov.__file__, "exec"), mod.__dict__)
    return mod


def test_unedited_oracle_passes_the_battery():
    with open(sov.__file__) as f:
        assert _battery(_load(f.read()))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    with open(sov.__file__) as f:
        src = f.read()
    assert src.count(old) == 1, name
    assert not _battery(_load(src.replace(old, new)))
