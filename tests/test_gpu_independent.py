"""GPU parity of the independent-points estimator (VECCHIA_QMC_INDEPENDENT:
each term's numerator from its lattice, its denominator from a second one)
against the oracle's, plus its bookkeeping in batches. Bars as in the other
parity tests: FP64 1e-10 per term, FP32 1e-3 per term."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import block as BZ
from oracle import censored as CZ
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _run(V, torch, plan, x_np, q, n_terms, scale=1.0):
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    t = torch.empty((n_terms, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, out, scale=scale, terms=t)
    torch.cuda.synchronize()
    return out.cpu().numpy(), t.cpu().numpy()


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
@pytest.mark.parametrize("D,m,N,R,seed", [(150, 10, 300, 4, 71), (90, 40, 200, 3, 72), (37, 3, 100, 3, 73)])
def test_plain_plan_matches_the_oracle(prec, D, m, N, R, seed):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(D, m, seed, n_points=N, n_shifts=R)
    c = inst.cov
    plan = V.vecchia_plan(inst.locs, inst.ordering, m, c)
    q = V.make_qmc(N, R, inst.qmc.seed, prec, independent=True)
    out, terms = _run(V, torch, plan, inst.x, q, D, scale=1.3)
    V.vecchia_plan_destroy(plan)
    o = oracle.logcdf(inst.locs, inst.x, m, c.family, c.nu, c.sigma2, c.range, c.nugget, inst.ordering, N, R,
                      inst.qmc.seed, scale=1.3, independent=True, processes=oracle.vecchia.default_processes())
    d = np.abs(terms[:, 0] - o["terms"][:, 0])
    if prec == W.PREC_FP64:
        assert d.max() <= 1e-10, d.max()
        np.testing.assert_allclose(terms[:, 1], o["terms"][:, 1], rtol=1e-6, atol=1e-12)
        assert abs(out[0] - o["logF"]) <= 1e-10
    else:
        assert d.max() <= 1e-3, d.max()
        assert abs(out[0] - o["logF"]) <= 1e-2 * abs(o["logF"])


def test_block_and_censored_plans_match_the_oracle():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(60, 3, 74, n_points=256, n_shifts=3)
    c = inst.cov
    plan = V.vecchia_plan_block(inst.locs, inst.ordering, 3, 3, c)
    q = V.make_qmc(256, 3, inst.qmc.seed, V.VECCHIA_FP64, independent=True)
    _, terms = _run(V, torch, plan, inst.x, q, V.plan_n_terms(plan))
    V.vecchia_plan_destroy(plan)
    o = BZ.logcdf_block(inst.locs, inst.x, 3, 3, c.family, c.nu, c.sigma2, c.range, c.nugget, inst.ordering,
                        256, 3, inst.qmc.seed, independent=True)
    assert np.max(np.abs(terms[:, 0] - o["terms"][:, 0])) <= 1e-10
    np.testing.assert_allclose(terms[:, 1], o["terms"][:, 1], rtol=1e-6, atol=1e-12)
    rep = W.censored_replicate(300, 10, 75, frac_obs=0.1, n_points=512, n_shifts=3)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    q = V.make_qmc(512, 3, i.qmc.seed, V.VECCHIA_FP64, independent=True)
    _, terms = _run(V, torch, plan, i.x, q, 300)
    V.vecchia_plan_destroy(plan)
    c = i.cov
    ref = CZ.loglik(i.locs, i.x, rep.observed, i.m, c.family, c.nu, c.sigma2, c.range, c.nugget, i.ordering,
                    512, 3, i.qmc.seed, perm=i.perm, independent=True,
                    processes=oracle.vecchia.default_processes())
    ok = np.abs(ref["terms"][:, 0]) <= 100
    assert np.max(np.abs(terms[ok, 0] - ref["terms"][ok, 0])) <= 1e-10
    assert np.max(np.abs(terms[~ok, 0] - ref["terms"][~ok, 0]) / np.abs(ref["terms"][~ok, 0]), initial=0) <= 1e-12


def test_shared_points_have_the_smaller_error_bar_and_agree():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.uniform2500_matern15()
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    shared = _run(V, torch, plan, inst.x, V.make_qmc(2000, 10, 3, V.VECCHIA_FP32_LOOP), inst.D)
    indep = _run(V, torch, plan, inst.x, V.make_qmc(2000, 10, 3, V.VECCHIA_FP32_LOOP, independent=True), inst.D)
    V.vecchia_plan_destroy(plan)
    assert abs(shared[0][0] - indep[0][0]) <= 4 * math.hypot(shared[0][1], indep[0][1])
    se_s, se_i = shared[1][:, 1], indep[1][:, 1]
    ok = se_s > 0
    assert np.median(se_i[ok] / se_s[ok]) > 1.5
    assert indep[0][1] > 1.5 * shared[0][1]


def test_batch_with_mixed_flags_equals_single_calls():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = [W.small_random_instance(200, 10, 76, n_points=500, n_shifts=3),
             W.small_random_instance(120, 5, 77, n_points=300, n_shifts=4)]
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    qs = [V.make_qmc(500, 3, 9, V.VECCHIA_FP32_LOOP, independent=True),
          V.make_qmc(300, 4, 9, V.VECCHIA_FP32_LOOP),
          V.make_qmc(500, 3, 9, V.VECCHIA_FP64, independent=True)]
    pl = [plans[0], plans[1], plans[0]]
    xs = [insts[0].x, insts[1].x, insts[0].x]
    alone = [_run(V, torch, p, x, q, len(x))[0] for p, x, q in zip(pl, xs, qs)]
    b = V.vecchia_batch_create(pl, qs)
    x = torch.tensor(np.concatenate(xs), dtype=torch.float64, device="cuda")
    out = torch.empty((3, 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(b, x, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for j in range(3):
        assert got[j, 0] == alone[j][0] and got[j, 1] == alone[j][1], j
    V.vecchia_batch_destroy(b)
    q = V.make_qmc(64, 2, 1, V.VECCHIA_FP64)
    q.flags = 2
    with pytest.raises(V.VecchiaError) as e:
        _run(V, torch, plans[1], insts[1].x, q, 120)
    assert e.value.status == 1
    for p in plans:
        V.vecchia_plan_destroy(p)
