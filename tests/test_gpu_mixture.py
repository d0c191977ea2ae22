"""GPU tests of the scale-mixture outer integral (Section 4, eqs. (8)-(9))
through the C ABI, against the oracle's rule on the same seeded inputs."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mixture as M
from tests.gpu_helpers import oracle_run, torch_cuda

pytestmark = pytest.mark.gpu


def _gpu_mixture(V, torch, plan, x_np, mix, q, cov=None):
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    nodes = torch.empty((mix.n_nodes, 2), dtype=torch.float64, device="cuda")
    V.vecchia_mixture_logcdf(plan, x, mix, q, out, nodes=nodes, cov_override=cov)
    torch.cuda.synchronize()
    return out.cpu().numpy(), nodes.cpu().numpy()


@pytest.mark.parametrize("beta,gamma", [(0.0, 2.0), (1.0, 3.0)])
def test_fp64_mixture_matches_the_oracle(beta, gamma):
    # the two sides take the window from their own search values (equal to
    # 1e-10): the same search points fall below the cut on both
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    # thresholds well above 0, so log Phi_D(x / r) falls steeply from r = 1 and the
    # window is short
    inst = W.small_random_instance(300, 5, 95, n_points=1000, n_shifts=4, mean_x=2.0, sd_x=0.3)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    mix = V.make_mixture(beta, gamma, 16)
    got, nodes = _gpu_mixture(V, torch, plan, inst.x, mix, V.as_qmc(inst.qmc))
    V.vecchia_plan_destroy(plan)
    ev = lambda r: (lambda d: (d["logF"], d["se"]))(oracle_run(inst, scale=r))
    ns = M.search_n_points(inst.qmc.n_points)
    evs = lambda r: (lambda d: (d["logF"], d["se"]))(oracle_run(inst, scale=r, n_points=ns))
    ref = M.logcdf_mixture(ev, beta, gamma, 16, eval_search=evs)
    print("logG", got, ref["logG"], ref["se"], "window", ref["window"], flush=True)
    assert ref["window"][1] < 200.0
    assert abs(got[0] - ref["logG"]) <= 1e-9 * max(1.0, abs(ref["logG"]))
    assert abs(got[1] - ref["se"]) <= 1e-6 * ref["se"] + 1e-12
    np.testing.assert_allclose(nodes[:, 0], ref["node_logF"], rtol=1e-6, atol=1e-8)


def test_zero_thresholds_return_the_orthant_value():
    # Phi_D(0 / r) = Phi_D(0) at every node: log G equals the plain evaluation of
    # the same plan (bitwise per node, to the rule's 1e-13 on e^-v) and sits within
    # a few SE of the closed form
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    S = np.array([[1.0, 0.3, 0.5], [0.3, 1.0, 0.2], [0.5, 0.2, 1.0]])
    plan = V.vecchia_plan_from_cov(S, 2)
    q = V.make_qmc(4096, 8, 5, V.VECCHIA_FP64)
    x = torch.zeros(3, dtype=torch.float64, device="cuda")
    single = torch.empty(2, dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, single)
    torch.cuda.synchronize()
    one = single.cpu().numpy()
    for beta, gamma in ((0.0, 2.0), (0.5, 1.0), (2.0, 0.3)):
        got, nodes = _gpu_mixture(V, torch, plan, np.zeros(3), V.make_mixture(beta, gamma, 32), q)
        assert np.all(nodes[:, 0] == one[0])
        assert abs(got[0] - one[0]) <= 1e-12
    exact = math.log(1.0 / 8.0 + (math.asin(0.3) + math.asin(0.5) + math.asin(0.2)) / (4.0 * math.pi))
    assert abs(one[0] - exact) <= 4.0 * one[1]
    V.vecchia_plan_destroy(plan)


def test_fp32_mixture_on_the_2500_point_workload():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.uniform2500_matern15()
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    mix = V.make_mixture(0.0, 2.0, 32)
    q32 = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, V.VECCHIA_FP32_LOOP)
    q64 = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, V.VECCHIA_FP64)
    g32, n32 = _gpu_mixture(V, torch, plan, inst.x, mix, q32)
    g64, n64 = _gpu_mixture(V, torch, plan, inst.x, mix, q64)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    plain = torch.empty(2, dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q64, plain)
    torch.cuda.synchronize()
    p64 = plain.cpu().numpy()
    V.vecchia_plan_destroy(plan)
    print("logG fp32", g32, "fp64", g64, "unmixed", p64, flush=True)
    assert np.all(np.isfinite(n32)) and np.isfinite(g32[0]) and g32[1] > 0
    assert abs(g32[0] - g64[0]) <= 1e-2 * abs(g64[0])
    # R >= 1 shrinks these (mostly positive) thresholds: the mixture lies below
    # the unmixed CDF, and every node below it too
    assert g64[0] < p64[0] and np.all(n64[:, 0] < p64[0])
