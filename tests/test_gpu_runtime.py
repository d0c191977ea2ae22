"""GPU tests of the runtime around the kernels: batched launches, HIP-graph
replay, in-place re-planning, the serving loop (each result the same alone and
in a mix) and the kernel timing hook."""
import math
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _instances():
    return [W.small_random_instance(300, 10, 41, n_points=1000, n_shifts=4, precision=W.PREC_FP32),
            W.small_random_instance(120, 3, 42, nu=0.5, n_points=777, n_shifts=3, precision=W.PREC_FP64),
            W.small_random_instance(1, 5, 43, n_points=64, n_shifts=2, precision=W.PREC_FP32),
            W.small_random_instance(200, 31, 44, nu=2.5, n_points=300, n_shifts=2, precision=W.PREC_FP32,
                                    scale=1.7)]


def _single(V, torch, plan, inst, stream=None):
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, V.as_qmc(inst.qmc), out, scale=inst.scale, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_batch_matches_single_evaluations_bitwise():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = _instances()
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    singles = [_single(V, torch, p, i) for p, i in zip(plans, insts)]
    batch = V.vecchia_batch_create(plans, [i.qmc for i in insts])
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    out = torch.empty((len(insts), 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(batch, x, out, scales=[i.scale for i in insts])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, np.array(singles))
    assert list(V.vecchia_batch_status(batch, len(insts))) == [-1] * len(insts)
    V.vecchia_batch_destroy(batch)
    for p in plans:
        V.vecchia_plan_destroy(p)


def test_graph_replays_match_eager_result():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(500, 10, 51, n_points=2048, n_shifts=4, precision=W.PREC_FP32)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    stream = torch.cuda.Stream()
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    outs = []
    for rep in range(5):                       # call 1 eager, later calls replay a graph
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()               # the fill runs on torch's stream, not on `stream`
        V.vecchia_logcdf(plan, x, V.as_qmc(inst.qmc), out, stream=stream)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        junk = torch.randn(1 << 16, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        del junk
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # a different seed through the same graph changes the estimate
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    q = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed + 1, inst.qmc.precision)
    V.vecchia_logcdf(plan, x, q, out, stream=stream)
    torch.cuda.synchronize()
    o2 = out.cpu().numpy()
    assert o2[0] != outs[0][0] and abs(o2[0] - outs[0][0]) < 10 * (o2[1] + outs[0][1])
    V.vecchia_plan_destroy(plan)


def test_replan_equals_fresh_plan():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    a = W.small_random_instance(400, 8, 61, n_points=512, n_shifts=3)
    b = W.small_random_instance(400, 8, 62, n_points=512, n_shifts=3)
    plan = V.vecchia_plan(a.locs, a.ordering, a.m, a.cov)
    fresh = V.vecchia_plan(b.locs, b.ordering, b.m, b.cov)
    V.vecchia_replan(plan, b.locs, b.ordering)
    torch.cuda.synchronize()
    p1, n1 = V.vecchia_plan_neighbours(plan)
    p2, n2 = V.vecchia_plan_neighbours(fresh)
    assert np.array_equal(p1, p2) and np.array_equal(n1, n2)
    assert np.array_equal(_single(V, torch, plan, b), _single(V, torch, fresh, b))
    V.vecchia_plan_destroy(plan)
    V.vecchia_plan_destroy(fresh)


def test_server_results_same_alone_and_in_mix():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = _instances()
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    alone = [_single(V, torch, p, i) for p, i in zip(plans, insts)]
    xs = [torch.tensor(i.x, dtype=torch.float64, device="cuda") for i in insts]
    srv = V.vecchia_server_create(1 << 30, 4)
    tickets = []
    for rep in range(3):                       # 12 overlapping requests
        for j, i in enumerate(insts):
            tickets.append((j, V.vecchia_submit(srv, plans[j], xs[j], i.qmc, scale=i.scale)))
    results = {}
    t_end = time.time() + 60
    while len(results) < len(tickets) and time.time() < t_end:
        for k, (j, t) in enumerate(tickets):
            if k in results:
                continue
            r = V.vecchia_poll(srv, t)
            if r is not None:
                results[k] = (j, r)
        time.sleep(0.001)
    assert len(results) == len(tickets)
    for k, (j, (lf, se, lat)) in results.items():
        assert lf == alone[j][0] and (se == alone[j][1] or (math.isnan(se) and math.isnan(alone[j][1])))
        assert lat > 0
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_poll(srv, 999999)
    assert e.value.status == 1
    V.vecchia_server_destroy(srv)
    for p in plans:
        V.vecchia_plan_destroy(p)


def test_server_rejects_request_over_budget_and_busy_plan():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(400, 10, 71, n_points=4096, n_shifts=8)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    srv = V.vecchia_server_create(4096, 2)
    with pytest.raises(V.VecchiaError) as e:
        V.vecchia_submit(srv, plan, x, inst.qmc)
    assert e.value.status == 2
    V.vecchia_server_destroy(srv)
    srv = V.vecchia_server_create(1 << 28, 1)
    t = V.vecchia_submit(srv, plan, x, inst.qmc)
    busy = None
    try:
        V.vecchia_plan_destroy(plan)
    except V.VecchiaError as err:
        busy = err.status
    r = None
    t_end = time.time() + 30
    while r is None and time.time() < t_end:
        r = V.vecchia_poll(srv, t)
        time.sleep(0.001)
    assert r is not None
    V.vecchia_server_destroy(srv)
    if busy is not None:
        assert busy == 5
        V.vecchia_plan_destroy(plan)


def test_profile_hook_counts_the_main_launch():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(600, 10, 81, n_points=2048, n_shifts=4, precision=W.PREC_FP32)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    V.vecchia_profile_reset()
    V.vecchia_profile_enable(1)
    for _ in range(3):
        _single(V, torch, plan, inst)
    V.vecchia_profile_enable(0)
    ms, launches, steps = V.vecchia_profile_read(10, V.VECCHIA_FP32_LOOP)
    V.vecchia_profile_reset()
    assert launches == 3 and ms > 0
    assert steps == 3 * (600 - 10) * 4 * 2048 * 10
    V.vecchia_plan_destroy(plan)


def test_server_mix_of_plan_kinds_equals_standalone_calls():
    # plans of every kind in one stream of overlapping requests: a long chain
    # (general kernel), joint block terms, a censored replicate and an explicit
    # covariance; each result equals the same request run alone, bit for bit
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    long_i = W.small_random_instance(150, 45, 61, n_points=300, n_shifts=3, precision=W.PREC_FP32)
    blk_i = W.small_random_instance(240, 4, 62, n_points=500, n_shifts=3, precision=W.PREC_FP32)
    rep = W.censored_replicate(300, 10, 63, frac_obs=0.1, n_points=400, n_shifts=3)
    S = 0.6 * np.eye(12) + 0.4
    cov_x = np.random.default_rng(64).normal(0.5, 0.5, size=12)
    reqs = [
        (V.vecchia_plan(long_i.locs, long_i.ordering, long_i.m, long_i.cov), long_i.x,
         V.make_qmc(300, 3, 5, V.VECCHIA_FP32_LOOP), 1.0),
        (V.vecchia_plan_block(blk_i.locs, blk_i.ordering, 4, 3, blk_i.cov), blk_i.x,
         V.make_qmc(500, 3, 6, V.VECCHIA_FP64), 1.3),
        (V.vecchia_plan_censored(rep.inst.locs, rep.observed, rep.inst.ordering, rep.inst.m, rep.inst.cov),
         rep.inst.x, V.make_qmc(400, 3, 7, V.VECCHIA_FP32_LOOP), 1.1),
        (V.vecchia_plan_from_cov(S, 11), cov_x, V.make_qmc(256, 4, 8, V.VECCHIA_FP64), 1.0),
    ]
    xs = [torch.tensor(x, dtype=torch.float64, device="cuda") for _, x, _, _ in reqs]
    alone = []
    for (p, _, q, sc), x in zip(reqs, xs):
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        V.vecchia_logcdf(p, x, q, out, scale=sc)
        torch.cuda.synchronize()
        alone.append(out.cpu().numpy())
    assert all(np.isfinite(a[0]) for a in alone)
    srv = V.vecchia_server_create(1 << 30, 3)
    tickets = [(j, V.vecchia_submit(srv, p, xs[j], q, scale=sc))
               for _ in range(2) for j, (p, _, q, sc) in enumerate(reqs)]
    results = {}
    t_end = time.time() + 60
    while len(results) < len(tickets) and time.time() < t_end:
        for k, (j, t) in enumerate(tickets):
            if k not in results:
                r = V.vecchia_poll(srv, t)
                if r is not None:
                    results[k] = (j, r)
        time.sleep(0.001)
    assert len(results) == len(tickets)
    for k, (j, (lf, se, _)) in results.items():
        assert lf == alone[j][0] and se == alone[j][1], (k, j, lf, alone[j])
    V.vecchia_server_destroy(srv)
    for p, _, _, _ in reqs:
        V.vecchia_plan_destroy(p)


def test_saved_ordering_reproduces_the_plan():
    # a plan is saved as its permutation (vecchia_plan_neighbours) and rebuilt
    # with ORDER_GIVEN: same neighbours, same log-CDF bit for bit, no maxmin pass
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(3000, 12, 81, n_points=512, n_shifts=3, precision=W.PREC_FP32)
    a = V.vecchia_plan(inst.locs, W.ORDER_MAXMIN, inst.m, inst.cov)
    perm, nbr = V.vecchia_plan_neighbours(a)
    b = V.vecchia_plan(inst.locs, W.ORDER_GIVEN, inst.m, inst.cov, perm=perm)
    perm2, nbr2 = V.vecchia_plan_neighbours(b)
    assert np.array_equal(perm, perm2) and np.array_equal(nbr, nbr2)
    ra, rb = _single(V, torch, a, inst), _single(V, torch, b, inst)
    assert ra[0] == rb[0] and ra[1] == rb[1]
    V.vecchia_plan_destroy(a)
    V.vecchia_plan_destroy(b)
