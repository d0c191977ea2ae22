"""Pins of the joint (block) conditional Vecchia oracle (Section 3.2) and of
the SOV split it uses, against closed forms and the plain form."""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle
from oracle import block as B
from oracle import covariance, sov
from tests import closed_forms as cf


def _equi(D, rho):
    return (1 - rho) * np.eye(D) + rho


def test_split_zero_is_the_joint_cdf():
    # split = 0: the denominator is 1 and the term is Phi_2 itself (Owen's T)
    S = np.array([[1.0, 0.55], [0.55, 1.0]])
    lt, se = sov.term_estimate(S, np.array([0.4, -0.3]), 4096, 8, 3, 0, split=0)
    assert abs(lt - math.log(cf.bivariate_owen(0.4, -0.3, 0.55))) <= 4 * se + 1e-12
    # default split = n - 1: unchanged arithmetic
    a = sov.term_estimate(S, np.array([0.4, -0.3]), 512, 4, 3, 7)
    b = sov.term_estimate(S, np.array([0.4, -0.3]), 512, 4, 3, 7, split=1)
    assert a == b


@pytest.mark.parametrize("split", [0, 1, 2, 3])
def test_split_terms_against_the_equicorrelated_form(split):
    # Phi_5(b) / Phi_split(b[:split]) for an equicorrelated covariance
    rho, b = 0.35, np.array([0.3, 1.1, -0.2, 0.7, 0.5])
    lt, se = sov.term_estimate(_equi(5, rho), b, 8192, 8, 11, 2, split=split)
    den = 1.0 if split == 0 else cf.equicorrelated_cdf(b[:split], rho)
    want = math.log(cf.equicorrelated_cdf(b, rho) / den)
    assert abs(lt - want) <= 4 * se + 1e-10, (split, lt, want, se)


def test_group_size_one_is_the_plain_vecchia():
    rng = np.random.default_rng(2)
    locs = rng.random((80, 2))
    x = rng.normal(1.0, 0.5, 80)
    a = B.logcdf_block(locs, x, 6, 1, 1, 1.5, 1.0, 0.15, 1e-8, 2, 256, 4, 5)
    b = oracle.logcdf(locs, x, 6, 1, 1.5, 1.0, 0.15, 1e-8, 2, 256, 4, 5)
    assert a["logF"] == b["logF"] and a["se"] == b["se"]
    assert np.array_equal(a["terms"], b["terms"][a["perm"]])


def test_block_plan_conditioning_sets():
    rng = np.random.default_rng(9)
    locs = rng.random((50, 2))
    perm, groups, conds = B.block_plan(locs, 2, 4, 3)
    s = locs[perm]
    assert [len(g) for g in groups] == [3] * 16 + [2]
    for g, (G, C) in enumerate(zip(groups, conds)):
        assert np.array_equal(G, np.arange(3 * g, min(50, 3 * g + 3)))
        assert np.all(C < 3 * g) and len(set(C.tolist())) == len(C) and len(C) <= 12
        # every member's 4 nearest earlier-group positions are in C, by brute force
        for i in G:
            d2 = ((s[:3 * g] - s[i]) ** 2).sum(axis=1)
            near = set(np.lexsort((np.arange(3 * g), d2))[:min(4, 3 * g)].tolist())
            assert near <= set(C.tolist())


@pytest.mark.parametrize("p", [2, 3, 7])
def test_all_earlier_components_give_the_exact_cdf(p):
    # m = D - 1: every group conditions on all earlier components, the product
    # telescopes to Phi_D; equicorrelated closed form, D = 7
    D, rho = 7, 0.4
    x = np.array([0.3, -0.2, 1.1, 0.5, -0.6, 0.9, 0.1])
    groups = [np.arange(g, min(D, g + p)) for g in range(0, D, p)]
    conds = [np.arange(0, g) for g in range(0, D, p)]
    r = B.logcdf_block_from_cov(_equi(D, rho), x, groups, conds, 8192, 8, 4)
    want = math.log(cf.equicorrelated_cdf(x, rho))
    assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-10, (p, r["logF"], want, r["se"])


def test_one_group_is_the_full_cdf():
    # p = D: a single term Phi_3(0) = trivariate orthant
    pts = np.array([[0.0, 0.0], [0.2, 0.1], [0.05, 0.3]])
    S = covariance.cov_matrix(pts, covariance.COV_EXPONENTIAL, 0.5, 1.0, 0.4, 0.0)
    r = B.logcdf_block_from_cov(S, np.zeros(3), [np.arange(3)], [np.zeros(0, np.int64)], 8192, 8, 6)
    want = math.log(cf.orthant3(S[0, 1], S[0, 2], S[1, 2]))
    assert abs(r["logF"] - want) <= 4 * r["se"] + 1e-12


def test_equicorrelated_block_terms_with_small_sets():
    # per-term pin: each term is a ratio of equicorrelated CDFs whatever the sets
    D, rho = 9, 0.3
    x = np.array([0.8, 0.1, -0.4, 1.3, 0.6, -0.1, 0.9, 0.2, 0.4])
    groups = [np.arange(0, 3), np.arange(3, 6), np.arange(6, 9)]
    conds = [np.zeros(0, np.int64), np.array([2, 0]), np.array([5, 1, 3, 4])]
    r = B.logcdf_block_from_cov(_equi(D, rho), x, groups, conds, 4096, 8, 12)
    for g, (G, C) in enumerate(zip(groups, conds)):
        v = np.concatenate([C, G])
        den = 1.0 if len(C) == 0 else cf.equicorrelated_cdf(x[C], rho)
        want = math.log(cf.equicorrelated_cdf(x[v], rho) / den)
        lt, se = r["terms"][g]
        assert abs(lt - want) <= 4 * se + 1e-10, (g, lt, want, se)


def test_independent_components_are_exact_products():
    # a diagonal covariance: every term is prod_{i in G} Phi(x_i) exactly
    from scipy.special import log_ndtr
    D = 12
    x = np.linspace(-1.0, 2.0, D)
    groups = [np.arange(g, min(D, g + 5)) for g in range(0, D, 5)]
    conds = [np.arange(max(0, g - 3), g) for g in range(0, D, 5)]
    r = B.logcdf_block_from_cov(np.eye(D), x, groups, conds, 256, 4, 1)
    for g, G in enumerate(groups):
        assert abs(r["terms"][g, 0] - float(np.sum(log_ndtr(x[G])))) <= 1e-12


BLOCK_MUTATIONS = {
    "sets_from_all_preceding": ("for j in nearest_before(s, int(i), g0, m):",
                                "for j in nearest_before(s, int(i), int(i), m):"),
    "group_before_conditioning": ("v = np.concatenate([np.asarray(Cg, dtype=np.int64), np.asarray(G, dtype=np.int64)])",
                                  "v = np.concatenate([np.asarray(G, dtype=np.int64), np.asarray(Cg, dtype=np.int64)])"),
    "split_short_by_one": ("split=len(Cg)))", "split=max(0, len(Cg) - 1)))"),
}
SOV_SPLIT_MUTATIONS = {
    "head_one_factor_late": ("if a + 1 == split:", "if a == split:"),
}


def _load(path, name, src):
    spec = importlib.util.spec_from_loader(name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src, path, "exec"), mod.__dict__)
    return mod


def _block_pins_pass(Bm) -> bool:
    try:
        D, rho = 7, 0.4
        x = np.array([0.3, -0.2, 1.1, 0.5, -0.6, 0.9, 0.1])
        for p in (2, 3):
            groups = [np.arange(g, min(D, g + p)) for g in range(0, D, p)]
            conds = [np.arange(0, g) for g in range(0, D, p)]
            r = Bm.logcdf_block_from_cov(_equi(D, rho), x, groups, conds, 4096, 8, 4)
            if not abs(r["logF"] - math.log(cf.equicorrelated_cdf(x, rho))) <= 4 * r["se"] + 1e-10:
                return False
        x9 = np.array([0.8, 0.1, -0.4, 1.3, 0.6, -0.1, 0.9, 0.2, 0.4])
        groups = [np.arange(0, 3), np.arange(3, 6), np.arange(6, 9)]
        conds = [np.zeros(0, np.int64), np.array([2, 0]), np.array([5, 1, 3, 4])]
        r = Bm.logcdf_block_from_cov(_equi(9, 0.3), x9, groups, conds, 4096, 8, 12)
        for g, (G, C) in enumerate(zip(groups, conds)):
            v = np.concatenate([C, G])
            den = 1.0 if len(C) == 0 else cf.equicorrelated_cdf(x9[C], 0.3)
            lt, se = r["terms"][g]
            if not abs(lt - math.log(cf.equicorrelated_cdf(x9[v], 0.3) / den)) <= 4 * se + 1e-10:
                return False
        rng = np.random.default_rng(9)
        locs = rng.random((50, 2))
        perm, groups, conds = Bm.block_plan(locs, 2, 4, 3)
        s = locs[perm]
        for g, (G, C) in enumerate(zip(groups, conds)):
            if not np.all(C < 3 * g):
                return False
            for i in G:
                d2 = ((s[:3 * g] - s[i]) ** 2).sum(axis=1)
                if not set(np.lexsort((np.arange(3 * g), d2))[:min(4, 3 * g)].tolist()) <= set(C.tolist()):
                    return False
        return True
    except (ValueError, IndexError, TypeError, sov.NotPositiveDefinite, np.linalg.LinAlgError):
        return False


@pytest.mark.parametrize("name", ["none"] + sorted(BLOCK_MUTATIONS) + sorted(SOV_SPLIT_MUTATIONS))
def test_planted_block_mistakes_fail_a_pin(name):
    bpath = os.path.join(os.path.dirname(B.__file__), "block.py")
    spath = os.path.join(os.path.dirname(B.__file__), "sov.py")
    bsrc, ssrc = open(bpath).read(), open(spath).read()
    if name in BLOCK_MUTATIONS:
        old, new = BLOCK_MUTATIONS[name]
        assert old in bsrc
        bsrc = bsrc.replace(old, new)
    if name in SOV_SPLIT_MUTATIONS:
        old, new = SOV_SPLIT_MUTATIONS[name]
        assert old in ssrc
        ssrc = ssrc.replace(old, new)
    sov_m = _load(spath, "oracle._mutant_sov_split", ssrc)
    Bm = _load(bpath, "oracle._mutant_block", bsrc)
    Bm.sov = sov_m
    with np.errstate(all="ignore"):
        assert _block_pins_pass(Bm) == (name == "none"), name
