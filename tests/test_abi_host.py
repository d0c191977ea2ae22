"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, orders locations on the host exactly as the oracle does, and
rejects bad arguments before touching a GPU."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import ordering as oracle_ordering
from paper_2007_15195_amd import vecchia as V

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vecchia.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:vecchia_status|const char\*)\s+(vecchia_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_entry_point():
    L = V.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(V.EXPORTED) == names


def test_struct_layouts_match_header():
    assert ctypes.sizeof(V.vecchia_cov) == 40
    assert ctypes.sizeof(V.vecchia_qmc) == 24


@pytest.mark.parametrize("rule", [W.ORDER_COORD, W.ORDER_MAXMIN])
@pytest.mark.parametrize("case", ["grid", "uniform", "dupes", "line", "repeated", "thin_offset"])
def test_host_ordering_matches_oracle(rule, case):
    rng = np.random.default_rng(11)
    if case == "grid":
        locs = W.grid_locations(17, 13)
    elif case == "uniform":
        locs = rng.random((3000, 2))
    elif case == "dupes":
        locs = np.round(rng.random((500, 2)) * 6) / 6.0
    elif case == "repeated":           # every location three times
        locs = np.repeat(rng.random((40, 2)), 3, axis=0)
    elif case == "thin_offset":        # a strip far from the origin (cell bounds at large magnitude)
        locs = rng.random((500, 2)) * np.array([1e-6, 1.0]) + 1e3
    else:
        locs = np.stack([np.linspace(0, 1, 300), np.full(300, 0.25)], axis=1)
    got = V.vecchia_order(locs, rule)
    want = oracle_ordering.order(locs, rule)
    assert np.array_equal(got, want)


def test_host_maxmin_on_the_2500_point_workload():
    inst = W.uniform2500_matern15()
    assert np.array_equal(V.vecchia_order(inst.locs, W.ORDER_MAXMIN),
                          oracle_ordering.maxmin_order(inst.locs))


def test_given_ordering_and_validation():
    locs = np.random.default_rng(1).random((5, 2))
    assert list(V.vecchia_order(locs, W.ORDER_GIVEN, [4, 3, 2, 1, 0])) == [4, 3, 2, 1, 0]
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_order(locs, W.ORDER_GIVEN, [0, 0, 1, 2, 3])
    assert e.value.status == 1
    bad = locs.copy()
    bad[2, 1] = np.nan
    with pytest.raises(V.VecchiaError):
        V.vecchia_order(bad, W.ORDER_COORD)
    with pytest.raises(V.VecchiaError):
        V.vecchia_order(locs, 7)


def test_plan_rejects_bad_arguments_before_gpu_work():
    locs = np.random.default_rng(1).random((5, 2))
    cov = V.make_cov(V.VECCHIA_COV_MATERN, 1.5, 1.0, 0.1, 0.0)
    for kwargs in (dict(m=64), dict(m=-1)):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_plan(locs, W.ORDER_COORD, kwargs["m"], cov, stream=0)
        assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan(np.random.default_rng(1).random((5, 3)), W.ORDER_COORD, 2, cov, stream=0)
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan(locs, W.ORDER_COORD, 2, V.make_cov(V.VECCHIA_COV_MATERN, 0.7, 1.0, 0.1), stream=0)
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan(locs, W.ORDER_COORD, 2, V.make_cov(V.VECCHIA_COV_MATERN, 1.5, -1.0, 0.1), stream=0)
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_from_cov(np.array([[1.0, 0.5], [0.4, 1.0]]), 1, stream=0)   # not symmetric
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_from_cov(np.eye(3), 2, nbr=[[], [0], [2]], stream=0)      # not preceding
    assert e.value.status == 1
    obs = np.array([1, 0, 0, 1, 0], dtype=bool)
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_censored(locs, obs, W.ORDER_COORD, 64, cov, stream=0)
    assert e.value.status == 1
    with pytest.raises(ValueError):
        V.vecchia_plan_censored(locs, obs[:4], W.ORDER_COORD, 2, cov, stream=0)
    bad = np.array([1, 0, 2, 0, 0], dtype=np.uint8)
    with pytest.raises(V.VecchiaError) as e:
        V._check(V.lib().vecchia_plan_censored(locs.ctypes.data, 5, 2, W.ORDER_COORD, None, bad.ctypes.data, 2,
                                               V.byref(cov), None, V.byref(V.c_void_p())))
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_from_cov_censored(np.eye(3), 2, 4, stream=0)              # n_observed > D
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_from_cov_censored(np.eye(3), 2, -1, stream=0)
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_server_create(0, 4)
    assert e.value.status == 1
    assert "budget" in V.vecchia_last_error()


def test_tuning_table_and_autotune_validation():
    # the tuning table is host state: default 0, settable per (precision, m)
    assert V.vecchia_tuning_get(V.VECCHIA_FP32_LOOP, 10) == 0
    V.vecchia_tuning_set(V.VECCHIA_FP32_LOOP, 10, 1024)
    try:
        assert V.vecchia_tuning_get(V.VECCHIA_FP32_LOOP, 10) == 1024
        assert V.vecchia_tuning_get(V.VECCHIA_FP64, 10) == 0
    finally:
        V.vecchia_tuning_set(V.VECCHIA_FP32_LOOP, 10, 0)
    assert V.vecchia_tuning_get(V.VECCHIA_FP32_LOOP, 10) == 0
    for bad in ((2, 10, 1024), (1, 64, 1024), (1, -1, 1024), (1, 10, 100), (1, 10, 32), (1, 10, 1 << 25)):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_tuning_set(*bad)
        assert e.value.status == 1
    # the autotuner rejects bad arguments before any device work
    for bad in ((2, 1000, 4, [3]), (1, 0, 4, [3]), (1, 1000, 0, [3]), (1, 1000, 4, []), (1, 1000, 4, [0]),
                (1, 1000, 4, [5, 64])):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_autotune(*bad, stream=0)
        assert e.value.status == 1


def test_calibration_hook_rejects_missing_output():
    with pytest.raises(V.VecchiaError) as e:
        V._check(V.lib().vecchia_calibrate_valu(None, None))
    assert e.value.status == 1


def _search_profiles():
    # log h on the search grid: a plain CDF (bulk at v = 0), a censored-like
    # interior peak (narrow and wide), a flat profile and one that sits at -inf
    # on part of the grid
    v = np.array([0.0] + [1e-4 * 2e6 ** ((j - 1) / 22) for j in range(1, 24)])
    yield np.log1p(-0.5 * (1 - np.exp(-40.0 * v))) * 300.0
    yield 60.0 * (1 - np.exp(-v)) - 4.0 * v
    yield 400.0 * (1 - np.exp(-3.0 * v)) - 30.0 * v
    yield np.full(24, -3.0)
    yield np.where(v < 1.0, -np.inf, -2.0 * v)


@pytest.mark.parametrize("beta,gamma", [(0.0, 2.0), (0.0, 0.3), (0.5, 1.0), (2.0, 0.5)])
@pytest.mark.parametrize("n", [1, 2, 8, 48, 64])
def test_mixture_rule_matches_the_oracle(beta, gamma, n):
    # the library's search scales, window and Gauss-Legendre rule against the
    # oracle's (numpy's leggauss and the inverse of eq. (8))
    from oracle import mixture as M
    mix = V.make_mixture(beta, gamma, n)
    osc = np.array([M.scale_at(v, beta, gamma) for v in M.search_v()])
    np.testing.assert_allclose(V.vecchia_mixture_search(mix), osc, rtol=1e-13, atol=0.0)
    for h in _search_profiles():
        win, v, sc, lw = V.vecchia_mixture_rule(mix, h)
        owin = M.window(h)
        assert win == owin
        ov, olw = M.legendre_rule(owin[0], owin[1], n)
        np.testing.assert_allclose(v, ov, rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(sc, [M.scale_at(float(x), beta, gamma) for x in ov], rtol=1e-12, atol=0.0)
        np.testing.assert_allclose(lw, olw, rtol=1e-13, atol=1e-12)


def test_mixture_arguments_rejected_on_the_host():
    assert ctypes.sizeof(V.vecchia_mixture) == 24
    for mix in (V.make_mixture(-0.1, 2.0, 8), V.make_mixture(0.0, 0.0, 8), V.make_mixture(0.0, 2.0, 0),
                V.make_mixture(0.0, 2.0, 65), V.make_mixture(float("nan"), 2.0, 8)):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_mixture_rule(mix, np.zeros(24))
        assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_mixture_rule(V.make_mixture(0.0, 2.0, 8), np.full(24, np.nan))   # NaN search value
    assert e.value.status == 1


def test_censored_matrix_plan_host_setup_runs_before_device_work():
    # the host part of a censored matrix plan (neighbour lists, k_i, SOV
    # dimensions) runs before any device allocation; without a device the call
    # then fails with an error instead of returning a plan
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present: the GPU tests build these plans")
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_plan_from_cov_censored(np.eye(4), 3, 2, nbr=[[], [0], [0, 1], [1, 2]], stream=0)
    assert e.value.status == 4   # E_HIP: the host set-up passed, the device work could not start


def test_mixture_batch_arguments_rejected_on_the_host():
    q = V.make_qmc(1024, 4, 1, V.VECCHIA_FP64)
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_mixbatch_create([], 16, q)
    assert e.value.status == 1
    for n_nodes in (0, 65):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_mixbatch_create([None], n_nodes, q)
        assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_mixbatch_create([None], 16, V.make_qmc(0, 4, 1, V.VECCHIA_FP64))
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_mixbatch_create([None], 16, q)                                 # null plan
    assert e.value.status == 1
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_mixbatch_destroy(None)
    assert e.value.status == 1



def test_anisotropic_map_gives_the_mahalanobis_distance():
    # Section 4.1: distances between mapped points equal the oracle's |Omega|,
    # computed from the rotation and scaling matrices as printed
    from oracle import covariance as C
    rng = np.random.default_rng(12)
    pts = rng.uniform(-5.0, 24.0, (40, 2))
    for phi, A in ((1.10, 2.29), (0.0, 1.0), (2.9, 1.5), (math.pi / 2, 3.0)):
        mp = V.vecchia_map_anisotropic(pts, phi, A)
        for i in range(0, 40, 3):
            for j in range(1, 40, 5):
                want = C.mahalanobis_distance(pts[i], pts[j], phi, A)
                got = float(np.hypot(*(mp[i] - mp[j])))
                assert abs(got - want) <= 1e-13 * max(1.0, want)
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_map_anisotropic(pts, 1.0, 0.0)
    assert e.value.status == 1


def test_oracle_anisotropic_coords_match_its_distance():
    from oracle import covariance as C
    pts = np.random.default_rng(3).uniform(-5.0, 24.0, (20, 2))
    mp = C.anisotropic_coords(pts, 1.10, 2.29)
    for i in range(20):
        for j in range(i):
            want = C.mahalanobis_distance(pts[i], pts[j], 1.10, 2.29)
            assert abs(float(np.hypot(*(mp[i] - mp[j]))) - want) <= 1e-13 * want


def test_mahalanobis_special_cases():
    # no rotation: the second coordinate is stretched by A; a quarter turn: the
    # first one is
    from oracle import covariance as C
    assert abs(C.mahalanobis_distance([1.0, 2.0], [0.0, 0.0], 0.0, 3.0) - math.hypot(1.0, 6.0)) < 1e-14
    assert abs(C.mahalanobis_distance([1.0, 2.0], [0.0, 0.0], math.pi / 2, 3.0) - math.hypot(2.0, 3.0)) < 1e-14
    assert abs(C.mahalanobis_distance([0.3, -0.4], [0.0, 0.0], 0.7, 1.0) - 0.5) < 1e-15


def test_block_plan_arguments_rejected_on_the_host():
    locs = np.random.default_rng(1).random((20, 2))
    cov = V.make_cov(V.VECCHIA_COV_MATERN, 1.5, 1.0, 0.1, 0.0)
    for m, p in ((10, 6), (4, 13), (1, 0), (0, 65)):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_plan_block(locs, W.ORDER_COORD, m, p, cov, stream=0)
        assert e.value.status == 1
    S = np.eye(4)
    for terms in ([([0, 1], 2)], [([0, 0], 1)], [([0, 5], 1)], [([], 0)], [(list(range(4)), -1)]):
        with pytest.raises(V.VecchiaError) as e:
            V.vecchia_plan_from_cov_block(S, terms, stream=0)
        assert e.value.status == 1


def test_binding_constants_match_the_header():
    import re
    from paper_2007_15195_amd import vecchia as V
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                            "vecchia.h")).read()
    defines = dict(re.findall(r"#define (VECCHIA_[A-Z0-9_]+) (\d+)", hdr))
    checked = 0
    for name, val in defines.items():
        if hasattr(V, name):
            assert getattr(V, name) == int(val), name
            checked += 1
    assert checked >= 2
    assert V.MIX_SEARCH_NODES == int(defines["VECCHIA_MIX_SEARCH_NODES"])
    assert V.make_qmc(64, 2, 1, V.VECCHIA_FP32_LOOP, independent=True).flags == V.VECCHIA_QMC_INDEPENDENT



def test_empty_inputs_are_rejected_before_gpu_work():
    cov = V.make_cov(V.VECCHIA_COV_MATERN, 1.5, 1.0, 0.1, 0.0)
    none = np.zeros((0, 2))
    calls = [lambda: V.vecchia_order(none, W.ORDER_COORD),
             lambda: V.vecchia_plan(none, W.ORDER_COORD, 2, cov, stream=0),
             lambda: V.vecchia_plan_from_cov(np.zeros((0, 0)), 0, stream=0),
             lambda: V.vecchia_plan_block(none, W.ORDER_COORD, 2, 2, cov, stream=0),
             lambda: V.vecchia_plan_censored(none, np.zeros(0, dtype=bool), W.ORDER_COORD, 2, cov, stream=0)]
    for f in calls:
        with pytest.raises(V.VecchiaError) as e:
            f()
        assert e.value.status == 1
