"""Planted mistakes in the oracle (on the CPU) must be caught by the pins.

Each case edits the oracle's SOV source text, loads the edited copy as a module
and runs a small battery of the closed-form pins against it; every plausible
mistake below must make at least one pin fail, and the unedited source must pass.
"""
import importlib.util
import math
import os
import types

import numpy as np
import pytest
from scipy.special import ndtr

import oracle
from oracle import covariance
from tests import closed_forms as cf

SOV_PATH = os.path.join(os.path.dirname(oracle.__file__), "sov.py")

MUTATIONS = {
    "sign_of_conditioning_sum": ("acc = acc - L[a, c] * ys[c]", "acc = acc + L[a, c] * ys[c]"),
    "transposed_cholesky": ("acc = acc - L[a, c] * ys[c]", "acc = acc - L[c, a] * ys[c]"),
    "wrong_y_index": ("acc = acc - L[a, c] * ys[c]", "acc = acc - L[a, c] * ys[a - 1]"),
    "dropped_last_factor": ("num[r] = np.mean(prod * e)", "num[r] = np.mean(prod)"),
    "last_factor_in_denominator": ("if a < k:", "if a <= k:"),
    "missing_diagonal_scaling": ("ndtr(acc / L[a, a])", "ndtr(acc)"),
    "first_factor_unscaled": ("e1 = ndtr(b[0] / L[0, 0])", "e1 = ndtr(b[0])"),
    "inverse_of_w_without_e": ("u = np.maximum(w * e, DBL_MIN)", "u = np.maximum(w, DBL_MIN)"),
    "minus_inf_rule_dropped": ("if np.any(np.asarray(b) == -np.inf):", "if False:"),
    "plus_inf_taken_as_minus_inf": ("if np.any(np.asarray(b) == -np.inf):",
                                    "if np.any(np.isinf(np.asarray(b))):"),
}


def _load_sov(src: str) -> types.ModuleType:
    spec = importlib.util.spec_from_loader("oracle._mutant_sov", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src, SOV_PATH, "exec"), mod.__dict__)
    return mod


def _pins_pass(sov_mod) -> bool:
    orig = oracle.vecchia.sov
    oracle.vecchia.sov = sov_mod
    try:
        # equicorrelated, general thresholds (1-D integral form)
        D, m, rho = 7, 3, 0.4
        Sigma = (1 - rho) * np.eye(D) + rho
        x = np.array([0.3, -0.2, 1.1, 0.5, -0.6, 0.9, 0.1])
        nbrs = [list(range(max(0, i - m), i)) for i in range(D)]
        r = oracle.logcdf_from_cov(Sigma, x, nbrs, 1024, 8, 3)
        for i in range(1, D):
            v = nbrs[i] + [i]
            want = math.log(cf.equicorrelated_cdf(x[v], rho) / cf.equicorrelated_cdf(x[v[:-1]], rho))
            lt, se = r["terms"][i]
            if not abs(lt - want) <= 4 * se + 1e-9:
                return False
        # trivariate orthant, unequal correlations, non-unit variance
        pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
        C = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 2.0, 0.4, 0.0)
        r = oracle.logcdf_from_cov(C, np.zeros(3), [[], [0], [0, 1]], 2048, 8, 3)
        R = C / 2.0
        if not abs(r["logF"] - math.log(cf.orthant3(R[0, 1], R[0, 2], R[1, 2]))) <= 4 * r["se"] + 1e-9:
            return False
        # bivariate, non-unit variance, non-zero thresholds
        C = np.array([[2.0, 1.2], [1.2, 1.5]])
        b = np.array([0.7, -0.4])
        r = oracle.logcdf_from_cov(C, b, [[], [0]], 2048, 8, 5)
        corr = 1.2 / math.sqrt(3.0)
        b1, b2 = b[0] / math.sqrt(2.0), b[1] / math.sqrt(1.5)
        want = math.log(cf.bivariate_cdf(b1, b2, corr) / ndtr(b1))
        if not abs(r["terms"][1, 0] - want) <= 4 * r["terms"][1, 1] + 1e-9:
            return False
        # infinite limits: +inf leaves a component unconstrained (here the exact
        # m = D - 1 product then is the bivariate CDF of the other two), and a
        # -inf limit gives log F = -inf
        C = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 1.0, 0.4, 0.0)
        with np.errstate(all="ignore"):
            r = oracle.logcdf_from_cov(C, np.array([0.4, np.inf, -0.3]), [[], [0], [0, 1]], 2048, 8, 5)
            want = math.log(cf.bivariate_owen(0.4, -0.3, C[0, 2]))
            if not abs(r["logF"] - want) <= 4 * r["se"] + 1e-9:
                return False
            r = oracle.logcdf_from_cov(C, np.array([0.4, -np.inf, -0.3]), [[], [0], [0, 1]], 256, 4, 5)
        if r["logF"] != -math.inf:
            return False
        return True
    finally:
        oracle.vecchia.sov = orig


def test_unedited_oracle_passes_battery():
    with open(SOV_PATH) as f:
        assert _pins_pass(_load_sov(f.read()))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    with open(SOV_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    assert not _pins_pass(_load_sov(src.replace(old, new)))
