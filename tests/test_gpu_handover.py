"""Terms of FP32 evaluations handed to the FP64 kernels: at set-up (a chain limit
below -4 standard deviations) and after the FP32 pass (a log-term SE above
0.02). Every qualifying term is handed over, however many there are, so a
term's value depends only on its instance: two runs are bit for bit equal, a
batch row equals its instance run alone, and a mixture batch row equals its
single mixture, with far more than one eighth of 2,000+ terms handed over. The
handed-over terms equal the FP64 mode's values, and every FP32 term is within
1e-3 of the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import oracle_run, torch_cuda

pytestmark = pytest.mark.gpu


def _deep(D, seed, n_points=512, n_shifts=5, mean_x=-2.4):
    return W.small_random_instance(D, 10, seed, n_points=n_points, n_shifts=n_shifts, mean_x=mean_x, sd_x=0.6,
                                   rho=0.1)


def _run(V, torch, plan, x, q, nt):
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    t = torch.empty((nt, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, out, terms=t)
    torch.cuda.synchronize()
    return out.cpu().numpy(), t.cpu().numpy()


def test_many_handed_over_terms_are_repeatable_and_match_fp64_and_the_oracle():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = _deep(2400, 17)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    q32 = V.make_qmc(512, 5, inst.qmc.seed, V.VECCHIA_FP32_LOOP)
    o1, t1 = _run(V, torch, plan, x, q32, inst.D)
    o2, t2 = _run(V, torch, plan, x, q32, inst.D)
    o64, t64 = _run(V, torch, plan, x, V.make_qmc(512, 5, inst.qmc.seed, V.VECCHIA_FP64), inst.D)
    V.vecchia_plan_destroy(plan)
    assert np.array_equal(o1, o2) and np.array_equal(t1, t2)
    handed = np.abs(t1[:, 0] - t64[:, 0]) <= 1e-10
    print("handed over (equal to FP64):", int(handed.sum()), "of", inst.D, flush=True)
    assert handed.sum() > inst.D // 8
    # every term whose FP64 SE exceeds the re-run bar is among them
    assert np.all(handed[t64[:, 1] > 0.025])
    o = oracle_run(inst)
    assert np.max(np.abs(t1[:, 0] - o["terms"][:, 0])) <= 1e-3
    assert abs(o1[0] - o["logF"]) <= 1e-2 * abs(o["logF"])


def test_batch_rows_with_handed_over_terms_equal_each_instance_alone():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = [_deep(2100, 31), W.small_random_instance(900, 10, 32, n_points=512, n_shifts=5), _deep(2600, 33)]
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    qs = [V.make_qmc(512, 5, i.qmc.seed, V.VECCHIA_FP32_LOOP) for i in insts]
    b = V.vecchia_batch_create(plans, qs)
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    out = torch.empty((len(insts), 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(b, x, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for j, (p, i) in enumerate(zip(plans, insts)):
        one, _ = _run(V, torch, p, torch.tensor(i.x, dtype=torch.float64, device="cuda"), qs[j], i.D)
        assert np.array_equal(got[j], one), j
    V.vecchia_batch_destroy(b)
    for p in plans:
        V.vecchia_plan_destroy(p)


def test_mixture_batch_with_handed_over_terms_equals_single_mixtures():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = [_deep(2000, 41, mean_x=-2.0), _deep(2200, 42, mean_x=-2.0)]
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    q = V.make_qmc(512, 4, 77, V.VECCHIA_FP32_LOOP)
    mb = V.vecchia_mixbatch_create(plans, 12, q)
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    mix = V.make_mixture(0.0, 2.0, 12)
    out = torch.empty((len(insts), 2), dtype=torch.float64, device="cuda")
    V.vecchia_mixbatch_logcdf(mb, x, mix, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for t, (p, i) in enumerate(zip(plans, insts)):
        one = torch.empty(2, dtype=torch.float64, device="cuda")
        V.vecchia_mixture_logcdf(p, torch.tensor(i.x, dtype=torch.float64, device="cuda"), mix,
                                 V.make_qmc(512, 4, 77 + t, V.VECCHIA_FP32_LOOP), one)
        torch.cuda.synchronize()
        assert np.array_equal(got[t], one.cpu().numpy()), t
    V.vecchia_mixbatch_destroy(mb)
    for p in plans:
        V.vecchia_plan_destroy(p)
