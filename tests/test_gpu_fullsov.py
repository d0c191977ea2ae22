"""GPU tests of the full-dimension SOV estimate (the paper's comparator,
Section 3.1) through the C ABI, against oracle.fullsov and closed forms."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import covariance
from oracle import fullsov as FS
from tests import closed_forms as cf
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _full(V, torch, plan, x_np, q, scale=1.0, cov=None):
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    V.vecchia_full_logcdf(plan, x, q, out, scale=scale, cov_override=cov)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("D,N,R", [(1, 64, 2), (7, 300, 4), (60, 1000, 4), (203, 700, 3)])
def test_fp64_full_matches_the_oracle(D, N, R):
    # several dimension blocks (64) and Cholesky blocks (32) with ragged ends,
    # point counts that are not multiples of the 16-point wave tile
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(D, 5, 500 + D, ordering=W.ORDER_MAXMIN, n_points=N, n_shifts=R)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    got = _full(V, torch, plan, inst.x, V.make_qmc(N, R, 9, V.VECCHIA_FP64), scale=1.3)
    perm, _ = V.vecchia_plan_neighbours(plan)
    V.vecchia_plan_destroy(plan)
    c = inst.cov
    S = covariance.cov_matrix(inst.locs[perm], c.family, c.nu, c.sigma2, c.range, c.nugget)
    lf, se, _ = FS.logcdf_full(S, inst.x[perm] / 1.3, N, R, 9)
    print("D", D, "gpu", got, "oracle", lf, se, flush=True)
    assert abs(got[0] - lf) <= 1e-10 * max(1.0, abs(lf))
    if R > 1:
        assert abs(got[1] - se) <= 1e-6 * se + 1e-12


def test_full_against_closed_forms_through_matrix_plans():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    D, rho = 40, 0.45
    rng = np.random.default_rng(3)
    b = 0.8 + rng.normal(0.0, 0.4, D)
    Sig = (1 - rho) * np.eye(D) + rho
    plan = V.vecchia_plan_from_cov(Sig, 1)
    got = _full(V, torch, plan, b, V.make_qmc(4096, 8, 2, V.VECCHIA_FP64))
    want = math.log(cf.equicorrelated_cdf(b, rho))
    assert abs(got[0] - want) <= 4 * got[1] + 1e-10, (got, want)
    # a diagonal covariance: the integrand is constant
    dplan = V.vecchia_plan_from_cov(np.diag(np.linspace(0.5, 2.0, 50)), 1)
    bb = np.linspace(-1.0, 2.0, 50)
    got = _full(V, torch, dplan, bb, V.make_qmc(256, 4, 2, V.VECCHIA_FP64))
    from scipy.special import log_ndtr
    want = float(np.sum(log_ndtr(bb / np.sqrt(np.linspace(0.5, 2.0, 50)))))
    assert abs(got[0] - want) <= 1e-12 * abs(want)
    V.vecchia_plan_destroy(plan)
    V.vecchia_plan_destroy(dplan)


def test_full_agrees_with_vecchia_on_a_grid():
    # the comparator and the Vecchia log-CDF on the 400-point grid: both within a
    # few SE of each other at m = 30 is not expected (the approximation has its
    # own error); the test checks the comparator is repeatable across seeds
    # within its SE and that the Vecchia value converges towards it as m grows
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.grid400_exponential()
    plan = V.vecchia_plan(inst.locs, inst.ordering, 30, inst.cov)
    a = _full(V, torch, plan, inst.x, V.make_qmc(4096, 10, 1, V.VECCHIA_FP64))
    b = _full(V, torch, plan, inst.x, V.make_qmc(4096, 10, 2, V.VECCHIA_FP64))
    assert abs(a[0] - b[0]) <= 5 * math.hypot(a[1], b[1]), (a, b)
    errs = []
    for m in (2, 10, 30):
        p = V.vecchia_plan(inst.locs, inst.ordering, m, inst.cov)
        x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        V.vecchia_logcdf(p, x, V.make_qmc(4096, 10, 1, V.VECCHIA_FP64), out)
        torch.cuda.synchronize()
        errs.append(abs(out.cpu().numpy()[0] - a[0]))
        V.vecchia_plan_destroy(p)
    V.vecchia_plan_destroy(plan)
    print("full", a, b, "|vecchia - full| at m = 2, 10, 30:", errs, flush=True)
    assert errs[2] < errs[0]


def test_full_rejects_fp32_and_censored_plans():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(30, 3, 1)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VecchiaError):
        V.vecchia_full_logcdf(plan, x, V.make_qmc(64, 2, 1, V.VECCHIA_FP32_LOOP), out)
    V.vecchia_plan_destroy(plan)
    cplan = V.vecchia_plan_censored(inst.locs, np.arange(30) < 3, inst.ordering, inst.m, inst.cov)
    with pytest.raises(V.VecchiaError):
        V.vecchia_full_logcdf(cplan, x, V.make_qmc(64, 2, 1, V.VECCHIA_FP64), out)
    V.vecchia_plan_destroy(cplan)


def test_full_with_infinite_thresholds():
    # +inf: the component is unconstrained (the estimator matches the oracle's to
    # 1e-10); -inf anywhere: log F = -inf
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(40, 5, 541, ordering=W.ORDER_MAXMIN, n_points=300, n_shifts=4)
    x = inst.x.copy()
    x[[3, 17, 30]] = np.inf
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    q = V.make_qmc(300, 4, 9, V.VECCHIA_FP64)
    got = _full(V, torch, plan, x, q)
    perm, _ = V.vecchia_plan_neighbours(plan)
    c = inst.cov
    S = covariance.cov_matrix(inst.locs[perm], c.family, c.nu, c.sigma2, c.range, c.nugget)
    lf, se, _ = FS.logcdf_full(S, x[perm], 300, 4, 9)
    assert abs(got[0] - lf) <= 1e-10 * max(1.0, abs(lf))
    x[11] = -np.inf
    got = _full(V, torch, plan, x, q)
    assert got[0] == -math.inf
    V.vecchia_plan_destroy(plan)


def test_full_profile_hook_records_the_kernel():
    # the measurement hook: one record per call, with D(D-1)/2 FMAs per point
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(70, 5, 3, ordering=W.ORDER_MAXMIN, n_points=200, n_shifts=3)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q = V.make_qmc(200, 3, 5, V.VECCHIA_FP64)
    V.vecchia_profile_reset()
    V.vecchia_profile_enable(1)
    try:
        V.vecchia_full_logcdf(plan, x, q, out)
        torch.cuda.synchronize()
    finally:
        V.vecchia_profile_enable(0)
    ms, launches, fmas = V.vecchia_profile_read(V.VECCHIA_PROFILE_FULL_SOV, V.VECCHIA_FP64)
    V.vecchia_profile_reset()
    V.vecchia_plan_destroy(plan)
    assert launches == 1 and ms > 0.0
    assert fmas == 70 * 69 // 2 * 200 * 3
