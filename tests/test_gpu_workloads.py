"""GPU tests at the full sizes of the measured workloads: the launch-shape
autotuner, the batched uneven launch (512 instances of mixed D, m and nu) and
the 250,000-location tail instance, each checked against the oracle on sampled
outputs and through properties that hold at any size."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import neighbours as oracle_neighbours
from oracle import ordering as oracle_ordering
from tests.gpu_helpers import nbr_lists, oracle_run, sample_terms, torch_cuda

pytestmark = pytest.mark.gpu

FP64_TERM_TOL = 1e-10
FP32_TERM_TOL = 1e-3
FP32_REL_TOL = 1e-2


def _terms_run(V, torch, plan, inst, precision, stream=None):
    q = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, precision)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((inst.D, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, out, scale=inst.scale, terms=terms, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), terms.cpu().numpy()


def test_autotune_choice_and_parity_with_tuned_chunks():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    try:
        chunks, ms = V.vecchia_autotune(V.VECCHIA_FP32_LOOP, 4096, 8, [1, 2, 3, 4], stream=0)
        print("fp32 chunks", chunks, "ms", ms, flush=True)
        assert all(c in (256, 512, 1024, 2048, 4096) for c in chunks)
        assert all(t > 0 for t in ms)
        assert [V.vecchia_tuning_get(V.VECCHIA_FP32_LOOP, k) for k in range(1, 5)] == chunks
        chunks64, _ = V.vecchia_autotune(V.VECCHIA_FP64, 1000, 4, [4], stream=0)
        print("fp64 chunks", chunks64, flush=True)
        assert all(c in (256, 512, 1024) for c in chunks64)
        # a tuned chunk only regroups the FP64 partial sums
        V.vecchia_tuning_set(V.VECCHIA_FP64, 4, 256)
        inst = W.small_random_instance(300, 4, 81, n_points=1000, n_shifts=4)
        plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
        _, t256 = _terms_run(V, torch, plan, inst, V.VECCHIA_FP64)
        V.vecchia_plan_destroy(plan)
        V.vecchia_tuning_set(V.VECCHIA_FP64, 4, 1024)
        plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
        out, t1024 = _terms_run(V, torch, plan, inst, V.VECCHIA_FP64)
        V.vecchia_plan_destroy(plan)
        o = oracle_run(inst)
        for t in (t256, t1024):
            assert np.max(np.abs(t[:, 0] - o["terms"][:, 0])) <= FP64_TERM_TOL
        assert abs(out[0] - o["logF"]) <= FP64_TERM_TOL
    finally:
        for p in (V.VECCHIA_FP32_LOOP, V.VECCHIA_FP64):
            for k in range(1, 5):
                V.vecchia_tuning_set(p, k, 0)


def test_batched_uneven_512_instances():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    insts = W.batched_uneven()
    assert len(insts) == 512
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in insts]
    print("plans built; terms", sum(i.D for i in insts), flush=True)
    batch = V.vecchia_batch_create(plans, [i.qmc for i in insts])
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    out = torch.empty((len(insts), 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(batch, x, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert list(V.vecchia_batch_status(batch, len(insts))) == [-1] * len(insts)
    assert np.all(np.isfinite(got)) and np.all(got[:, 0] < 0) and np.all(got[:, 1] > 0)
    V.vecchia_batch_destroy(batch)
    # sampled instances: the smallest and largest D and one of every m; each
    # alone equals its batch row bitwise, and its sampled terms match the oracle
    Ds = np.array([i.D for i in insts])
    pick = {int(np.argmin(Ds)), int(np.argmax(Ds))}
    for m in (5, 10, 15, 20):
        pick.add(next(j for j, i in enumerate(insts) if i.m == m))
    for j in sorted(pick):
        inst = insts[j]
        alone, terms = _terms_run(V, torch, plans[j], inst, V.VECCHIA_FP32_LOOP)
        assert np.array_equal(alone, got[j]), j
        perm, nbr = V.vecchia_plan_neighbours(plans[j])
        sub = sample_terms(inst.D, inst.m, 12, 200 + j)
        o = oracle_run(inst, terms_subset=sub, plan_cache=(perm, nbr_lists(perm, nbr)))
        sel = ~np.isnan(o["terms"][:, 0])
        d = np.abs(terms[sel, 0] - o["terms"][sel, 0])
        print(f"instance {j}: D={inst.D} m={inst.m} nu={inst.cov.nu} max|d|={d.max():.2e}", flush=True)
        assert np.all(d <= FP32_TERM_TOL), (j, d.max())
    for p in plans:
        V.vecchia_plan_destroy(p)


def test_uniform250k_tail_instance():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.uniform250k_tail()
    D, m = inst.D, inst.m
    plan = V.vecchia_plan(inst.locs, inst.ordering, m, inst.cov)
    perm, nbr = V.vecchia_plan_neighbours(plan)
    print("plan built", flush=True)
    # ordering: a permutation whose first picks are the maxmin definition's
    assert np.array_equal(np.sort(perm), np.arange(D))
    assert np.array_equal(perm[:300], oracle_ordering.maxmin_order(inst.locs, n_first=300))
    # neighbours: brute force on sampled plan positions, bit-exact
    s = inst.locs[perm]
    rng = np.random.default_rng(250)
    q = np.concatenate([np.arange(0, 25), rng.choice(np.arange(25, D), 150, replace=False), [D - 1]])
    ref = oracle_neighbours.knn_preceding(s, m, queries=q)
    for i, r in zip(q, ref):
        row = nbr[i][nbr[i] >= 0]
        assert np.array_equal(row, r), i
    # terms: FP64 to 1e-10 and FP32 to 1e-3 against the oracle on sampled terms
    out32, t32 = _terms_run(V, torch, plan, inst, V.VECCHIA_FP32_LOOP)
    print("fp32 done", out32, flush=True)
    out64, t64 = _terms_run(V, torch, plan, inst, V.VECCHIA_FP64)
    print("fp64 done", out64, flush=True)
    assert V.vecchia_plan_status(plan) == -1
    sub = sample_terms(D, m, 16, 251)
    o = oracle_run(inst, terms_subset=sub, plan_cache=(perm, nbr_lists(perm, nbr)))
    sel = ~np.isnan(o["terms"][:, 0])
    d64 = np.abs(t64[sel, 0] - o["terms"][sel, 0])
    d32 = np.abs(t32[sel, 0] - o["terms"][sel, 0])
    # joint-tail regime: log-terms near -1e-3, so also the relative error of -log-term
    rel32 = d32 / np.abs(o["terms"][sel, 0])
    print(f"max|d64|={d64.max():.2e} max|d32|={d32.max():.2e} max rel32={rel32.max():.2e}", flush=True)
    assert np.all(d64 <= FP64_TERM_TOL)
    assert np.all(d32 <= FP32_TERM_TOL)
    assert np.all(rel32 <= FP32_REL_TOL)
    # totals: the FP64 path covers every term, so FP32 is held against it
    assert abs(out32[0] - out64[0]) <= FP32_REL_TOL * abs(out64[0])
    assert np.max(np.abs(t32[:, 0] - t64[:, 0])) <= FP32_TERM_TOL
    V.vecchia_plan_destroy(plan)


def test_serving_mix_equals_standalone_calls():
    # requests shaped like the serving stream (mixed D and m, per-request
    # covariance range and scale factor, 2048-8192 points) submitted together;
    # every result must equal the same request evaluated alone, bitwise
    import time
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    st = W.serving_stream(n_plans=5, n_requests=30, d_min=1000, d_max=20000)
    plans = [V.vecchia_plan(p.locs, p.ordering, p.m, p.cov) for p in st.plans]
    xs = [torch.tensor(r.x, dtype=torch.float64, device="cuda") for r in st.requests]
    torch.cuda.synchronize()
    alone = []
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    for r, x in zip(st.requests, xs):
        V.vecchia_logcdf(plans[r.plan_id], x, V.as_qmc(r.qmc), out, scale=r.scale, cov_override=r.cov)
        torch.cuda.synchronize()
        alone.append(out.cpu().numpy().copy())
    srv = V.vecchia_server_create(4 << 30, 8)
    tickets = [V.vecchia_submit(srv, plans[r.plan_id], x, r.qmc, scale=r.scale, cov_override=r.cov)
               for r, x in zip(st.requests, xs)]
    got = {}
    t_end = time.time() + 120
    while len(got) < len(tickets) and time.time() < t_end:
        for k, t in enumerate(tickets):
            if k not in got:
                res = V.vecchia_poll(srv, t)
                if res is not None:
                    got[k] = res
        time.sleep(0.001)
    V.vecchia_server_destroy(srv)
    assert len(got) == len(tickets)
    for k, (lf, se, lat) in got.items():
        assert lf == alone[k][0] and se == alone[k][1], k
        assert np.isfinite(lf) and lf < 0 and lat > 0
    print("requests", len(tickets), "m values", sorted({st.plans[r.plan_id].m for r in st.requests}), flush=True)
    for p in plans:
        V.vecchia_plan_destroy(p)


def test_served_requests_match_the_oracle():
    # three requests shaped like the serving stream's, served in a mix with
    # larger ones, against the oracle: one with a covariance override, one with
    # a scale factor (eq. (9)'s Phi_D(x / r)), one with m = 30; in FP64 (1e-10)
    # and FP32 (1e-2 relative in log F)
    import time
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rng = np.random.default_rng(515)
    specs = [  # (D, m, range of the plan, override or None, scale, N)
        (1500, 12, 0.1, W.Cov(W.COV_MATERN, 1.5, 1.3, 0.23, 1e-8), 1.0, 2048),
        (1200, 8, 0.1, None, 2.7183, 2048),
        (900, 30, 0.15, W.Cov(W.COV_MATERN, 1.5, 1.0, 0.05, 1e-8), 1.4142, 4096),
    ]
    checked = []
    for D, m, rho, ov, scale, N in specs:
        locs = rng.random((D, 2))
        x = rng.normal(1.5, 0.5, D)
        checked.append(W.Instance(f"served_D{D}_m{m}", locs, x, m, W.ORDER_MAXMIN,
                                  W.Cov(W.COV_MATERN, 1.5, 1.0, rho, 1e-8), W.QMC(N, 8, 600 + D, W.PREC_FP64),
                                  scale=scale))
    st = W.serving_stream(n_plans=3, n_requests=6, d_min=5000, d_max=20000)
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov) for i in checked]
    others = [V.vecchia_plan(p.locs, p.ordering, p.m, p.cov) for p in st.plans]
    xs = [torch.tensor(i.x, dtype=torch.float64, device="cuda") for i in checked]
    xo = [torch.tensor(r.x, dtype=torch.float64, device="cuda") for r in st.requests]
    torch.cuda.synchronize()
    srv = V.vecchia_server_create(4 << 30, 8)
    tickets = []
    for prec in (V.VECCHIA_FP64, V.VECCHIA_FP32_LOOP):
        for k, (inst, (_, _, _, ov, _, _)) in enumerate(zip(checked, specs)):
            q = V.make_qmc(inst.qmc.n_points, 8, inst.qmc.seed, prec)
            tickets.append(((prec, k), V.vecchia_submit(srv, plans[k], xs[k], q, scale=inst.scale,
                                                        cov_override=ov)))
            r = st.requests[len(tickets) % len(st.requests)]
            tickets.append((None, V.vecchia_submit(srv, others[r.plan_id], xo[len(tickets) % len(xo)], r.qmc,
                                                   scale=r.scale, cov_override=r.cov)))
    got = {}
    t_end = time.time() + 120
    while len(got) < len(tickets) and time.time() < t_end:
        for j, (key, t) in enumerate(tickets):
            if j not in got:
                res = V.vecchia_poll(srv, t)
                if res is not None:
                    got[j] = (key, res)
        time.sleep(0.001)
    V.vecchia_server_destroy(srv)
    assert len(got) == len(tickets)
    res = {key: r for key, r in got.values() if key is not None}
    for k, (inst, (_, _, _, ov, _, _)) in enumerate(zip(checked, specs)):
        c = ov or inst.cov
        o = oracle.logcdf(inst.locs, inst.x, inst.m, c.family, c.nu, c.sigma2, c.range, c.nugget, inst.ordering,
                          inst.qmc.n_points, 8, inst.qmc.seed, scale=inst.scale,
                          processes=oracle.vecchia.default_processes())
        lf64, se64, _ = res[(V.VECCHIA_FP64, k)]
        lf32, se32, _ = res[(V.VECCHIA_FP32_LOOP, k)]
        print(inst.name, "oracle", o["logF"], "fp64", lf64, "fp32", lf32, flush=True)
        assert abs(lf64 - o["logF"]) <= 1e-10
        assert abs(se64 - o["se"]) <= 1e-6 * o["se"]
        assert abs(lf32 - o["logF"]) <= FP32_REL_TOL * abs(o["logF"])
    for p in plans + others:
        V.vecchia_plan_destroy(p)


def test_launch_split_beyond_the_work_item_limit():
    # 64-point chunks on 70,000 terms x 8 shifts x 4096 points give 35.8M work
    # items (one wave each): more than one launch can hold (2^32 work-items), so
    # the QMC launch is split; the result must match the default chunking up to
    # the FP64 regrouping of the partial sums
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rng = np.random.default_rng(90)
    D, m = 70_000, 5
    locs = rng.random((D, 2))
    cov = V.make_cov(V.VECCHIA_COV_MATERN, 1.5, 1.0, 0.05, 1e-8)
    x = torch.tensor(rng.normal(1.5, 0.5, D), dtype=torch.float64, device="cuda")
    q = V.make_qmc(4096, 8, 91, V.VECCHIA_FP32_LOOP)
    res = []
    try:
        for chunk in (0, 64):
            V.vecchia_tuning_set(V.VECCHIA_FP32_LOOP, m, chunk)
            plan = V.vecchia_plan(locs, W.ORDER_COORD, m, cov)
            out = torch.empty(2, dtype=torch.float64, device="cuda")
            terms = torch.empty((D, 2), dtype=torch.float64, device="cuda")
            V.vecchia_logcdf(plan, x, q, out, terms=terms)
            torch.cuda.synchronize()
            assert V.vecchia_plan_status(plan) == -1
            res.append((out.cpu().numpy(), terms.cpu().numpy()))
            V.vecchia_plan_destroy(plan)
    finally:
        V.vecchia_tuning_set(V.VECCHIA_FP32_LOOP, m, 0)
    (o1, t1), (o2, t2) = res
    print("logF", o1[0], o2[0], flush=True)
    assert np.all(np.isfinite(t2[:, 0]))
    assert np.max(np.abs(t1[:, 0] - t2[:, 0])) <= 1e-12
    assert abs(o1[0] - o2[0]) <= 1e-11 * abs(o1[0])
