"""vecchia_logcdf_noalloc, the evaluation on the library's static per-GPU
scratch array, against vecchia_logcdf on the same plans and inputs: two calls
in a row (the second on a smaller input), bit-for-bit equal outputs, for a
plain plan in both precisions (with terms handed to the FP64 kernels) and a
censored plan (many ranges, several descriptor stores); a workspace beyond the
array is rejected before any GPU work."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _both(V, torch, plan, x, q, nt, scale=1.0):
    res = []
    for f in (V.vecchia_logcdf, V.vecchia_logcdf_noalloc):
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        t = torch.full((nt, 2), float("nan"), dtype=torch.float64, device="cuda")
        f(plan, x, q, out, scale=scale, terms=t)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), t.cpu().numpy()))
    return res


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_noalloc_equals_logcdf_on_two_calls(prec):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    big = W.uniform2500_matern15(n_points=2000, n_shifts=10)
    small = W.small_random_instance(300, 6, 55, n_points=700, n_shifts=5, mean_x=-1.5, sd_x=1.0)
    for inst in (big, small):
        print(f"noalloc case {inst.name} precision {prec}", flush=True)
        plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
        x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
        q = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, prec)
        (oa, ta), (ob, tb) = _both(V, torch, plan, x, q, inst.D, inst.scale)
        V.vecchia_plan_destroy(plan)
        assert np.all(np.isfinite(ta[:, 0])) and np.isfinite(oa[0])
        assert np.array_equal(oa, ob) and np.array_equal(ta, tb)


def test_noalloc_censored_plan_equals_logcdf():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    for D, seed in ((1500, 61), (400, 62)):
        print(f"noalloc censored D {D}", flush=True)
        rep = W.censored_replicate(D, 12, seed, frac_obs=0.2, n_points=512, n_shifts=4)
        inst = rep.inst
        plan = V.vecchia_plan_censored(inst.locs, rep.observed, inst.ordering, inst.m, inst.cov)
        x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
        for prec in (W.PREC_FP64, W.PREC_FP32):
            q = V.make_qmc(512, 4, inst.qmc.seed, prec)
            (oa, ta), (ob, tb) = _both(V, torch, plan, x, q, inst.D)
            assert np.isfinite(oa[0])
            assert np.array_equal(oa, ob) and np.array_equal(ta, tb)
        V.vecchia_plan_destroy(plan)


def test_noalloc_rejects_a_workspace_beyond_the_scratch_array():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rng = np.random.default_rng(3)
    D = 40000
    locs = rng.random((D, 2))
    plan = V.vecchia_plan(locs, W.ORDER_COORD, 20, V.make_cov(V.VECCHIA_COV_MATERN, 1.5, 1.0, 0.05, 1e-8))
    x = torch.zeros(D, dtype=torch.float64, device="cuda")
    out = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VecchiaError) as ei:
        V.vecchia_logcdf_noalloc(plan, x, V.make_qmc(10_000, 10, 1, V.VECCHIA_FP32_LOOP), out)
    assert ei.value.status == 1 and "bytes" in str(ei.value)   # VECCHIA_E_INVALID
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 7.0)   # nothing was enqueued
    V.vecchia_plan_destroy(plan)
