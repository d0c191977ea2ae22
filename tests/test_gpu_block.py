"""GPU tests of the joint (block) conditional terms (Section 3.2) through the C
ABI, against oracle.block on the same seeded inputs."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import block as B
from tests import closed_forms as cf
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _run(V, torch, plan, x_np, q, n_terms, scale=1.0):
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    t = torch.empty((n_terms, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, out, scale=scale, terms=t)
    torch.cuda.synchronize()
    return out.cpu().numpy(), t.cpu().numpy()


def _oracle(inst, p, n_points=None):
    c = inst.cov
    return B.logcdf_block(inst.locs, inst.x, inst.m, p, c.family, c.nu, c.sigma2, c.range, c.nugget,
                          inst.ordering, n_points or inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed,
                          perm=inst.perm, processes=oracle.vecchia.default_processes())


@pytest.mark.parametrize("D,m,p,order", [(600, 4, 3, W.ORDER_MAXMIN), (257, 5, 5, W.ORDER_COORD),
                                         (100, 1, 16, W.ORDER_MAXMIN)])
def test_block_terms_match_the_oracle(D, m, p, order):
    torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(D, m, 40 + p, ordering=order)
    plan = V.vecchia_plan_block(inst.locs, order, m, p, inst.cov)
    perm, _ = V.vecchia_plan_neighbours(plan)
    off, var, split = V.vecchia_plan_block_terms(plan)
    V.vecchia_plan_destroy(plan)
    operm, groups, conds = B.block_plan(inst.locs, order, m, p)
    assert np.array_equal(perm, operm)
    assert len(off) - 1 == len(groups)
    for g, (G, C) in enumerate(zip(groups, conds)):
        v = var[off[g]:off[g + 1]]
        assert split[g] == len(C)
        assert np.array_equal(v, np.concatenate([C, G])), g


@pytest.mark.parametrize("m,p", [(4, 3), (5, 5), (2, 8), (15, 4)])
def test_fp64_block_logcdf_matches_the_oracle(m, p):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(300, m, 70 + p, n_points=1000, n_shifts=4)
    plan = V.vecchia_plan_block(inst.locs, inst.ordering, m, p, inst.cov)
    nt = V.plan_n_terms(plan)
    out, terms = _run(V, torch, plan, inst.x, V.as_qmc(inst.qmc), nt)
    assert V.vecchia_plan_status(plan) == -1
    V.vecchia_plan_destroy(plan)
    ref = _oracle(inst, p)
    print("logF", out, ref["logF"], ref["se"], flush=True)
    np.testing.assert_allclose(terms[:, 0], ref["terms"][:, 0], rtol=0.0, atol=1e-10)
    np.testing.assert_allclose(terms[:, 1], ref["terms"][:, 1], rtol=1e-6, atol=1e-12)
    assert abs(out[0] - ref["logF"]) <= 1e-10 * max(1.0, abs(ref["logF"]))


def test_fp32_block_logcdf_within_tolerance():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.uniform2500_matern15()
    for m, p in ((5, 5), (10, 2), (15, 4)):     # (15, 4): terms of 64 variables, general kernel
        plan = V.vecchia_plan_block(inst.locs, inst.ordering, m, p, inst.cov)
        nt = V.plan_n_terms(plan)
        q32 = V.make_qmc(4096, 8, 3, V.VECCHIA_FP32_LOOP)
        q64 = V.make_qmc(4096, 8, 3, V.VECCHIA_FP64)
        o32, t32 = _run(V, torch, plan, inst.x, q32, nt)
        o64, t64 = _run(V, torch, plan, inst.x, q64, nt)
        V.vecchia_plan_destroy(plan)
        d = np.abs(t32[:, 0] - t64[:, 0])
        print("m", m, "p", p, "fp32", o32, "fp64", o64, "max term diff", d.max(), flush=True)
        assert d.max() <= 1e-3
        assert abs(o32[0] - o64[0]) <= 1e-2 * abs(o64[0])


def test_group_size_one_is_the_plain_plan():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(500, 7, 3)
    q = V.as_qmc(inst.qmc)
    p1 = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    p2 = V.vecchia_plan_block(inst.locs, inst.ordering, inst.m, 1, inst.cov)
    a, ta = _run(V, torch, p1, inst.x, q, inst.D)
    b, tb = _run(V, torch, p2, inst.x, q, inst.D)
    V.vecchia_plan_destroy(p1)
    V.vecchia_plan_destroy(p2)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_explicit_terms_against_closed_forms(precision):
    # equicorrelated covariance: m = D - 1 groups telescope to Phi_D, and every
    # term (split 0 included) is a ratio of one-factor integrals
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    prec = V.VECCHIA_FP64 if precision == "fp64" else V.VECCHIA_FP32_LOOP
    D, rho = 9, 0.3
    Sig = (1 - rho) * np.eye(D) + rho
    x = np.array([0.8, 0.1, -0.4, 1.3, 0.6, -0.1, 0.9, 0.2, 0.4])
    groups = [np.arange(0, 3), np.arange(3, 6), np.arange(6, 9)]
    conds = [np.zeros(0, np.int64), np.array([2, 0]), np.array([5, 1, 3, 4])]
    terms = [(np.concatenate([C, G]), len(C)) for G, C in zip(groups, conds)]
    plan = V.vecchia_plan_from_cov_block(Sig, terms)
    out, t = _run(V, torch, plan, x, V.make_qmc(4096, 8, 12, prec), 3)
    V.vecchia_plan_destroy(plan)
    ref = B.logcdf_block_from_cov(Sig, x, groups, conds, 4096, 8, 12)
    for g, (G, C) in enumerate(zip(groups, conds)):
        v = np.concatenate([C, G])
        den = 1.0 if len(C) == 0 else cf.equicorrelated_cdf(x[C], rho)
        want = math.log(cf.equicorrelated_cdf(x[v], rho) / den)
        assert abs(t[g, 0] - want) <= 4 * t[g, 1] + (1e-10 if precision == "fp64" else 1e-6), (g, t[g], want)
        if precision == "fp64":
            assert abs(t[g, 0] - ref["terms"][g, 0]) <= 1e-10
        else:
            assert abs(t[g, 0] - ref["terms"][g, 0]) <= 1e-5
    # the whole CDF through all-earlier conditioning sets
    full = [(np.arange(0, g + 3 if g + 3 <= D else D), g) for g in range(0, D, 3)]
    plan = V.vecchia_plan_from_cov_block(Sig, full)
    out, _ = _run(V, torch, plan, x, V.make_qmc(8192, 8, 4, prec), len(full))
    V.vecchia_plan_destroy(plan)
    want = math.log(cf.equicorrelated_cdf(x, rho))
    assert abs(out[0] - want) <= 4 * out[1] + 1e-9, (out, want)


def test_block_and_plain_instances_in_one_batch():
    # block terms and plain terms of equal K run in separate launches of one
    # batch; every row equals its instance alone
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = [W.small_random_instance(400, 4, 90 + k) for k in range(3)]
    plans = [V.vecchia_plan_block(insts[0].locs, insts[0].ordering, 4, 3, insts[0].cov),
             V.vecchia_plan(insts[1].locs, insts[1].ordering, 4, insts[1].cov),
             V.vecchia_plan_block(insts[2].locs, insts[2].ordering, 4, 2, insts[2].cov)]
    qs = [V.as_qmc(i.qmc) for i in insts]
    alone = [_run(V, torch, p, i.x, q, V.plan_n_terms(p))[0] for p, i, q in zip(plans, insts, qs)]
    b = V.vecchia_batch_create(plans, qs)
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    out = torch.empty((3, 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(b, x, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    V.vecchia_batch_destroy(b)
    for p in plans:
        V.vecchia_plan_destroy(p)
    for k in range(3):
        assert np.array_equal(got[k], alone[k]), k
