"""GPU tests of the censored likelihood (Section 4, eq. (11)) through the C ABI,
against the oracle (oracle.censored) on the same seeded inputs."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
import workloads as W
from oracle import censored as CZ
from oracle import mixture as M
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu

FP64_TERM_TOL = 1e-10
FP32_TERM_TOL = 1e-3


def _gpu_loglik(V, torch, plan, x_np, q, scale=1.0, terms=True):
    D = len(x_np)
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    t = torch.empty((D, 2), dtype=torch.float64, device="cuda") if terms else None
    V.vecchia_logcdf(plan, x, q, out, scale=scale, terms=t)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (t.cpu().numpy() if terms else None)


def _oracle(rep, n_points=None, scale=1.0):
    i, c = rep.inst, rep.inst.cov
    return CZ.loglik(i.locs, i.x, rep.observed, i.m, c.family, c.nu, c.sigma2, c.range, c.nugget, i.ordering,
                     n_points or i.qmc.n_points, i.qmc.n_shifts, i.qmc.seed, scale=scale, perm=i.perm,
                     processes=oracle.vecchia.default_processes())


@pytest.mark.parametrize("D,order,frac", [(2000, W.ORDER_MAXMIN, 0.05), (1500, W.ORDER_COORD, 0.3),
                                          (30_000, W.ORDER_MAXMIN, 0.05)])
def test_censored_plan_matches_the_oracle(D, order, frac):
    # observed sites first (stable), neighbours in that order; the 30,000-site
    # plan searches through the grid (sampled rows against the definition)
    torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rep = W.censored_replicate(D, 10, 31 + D, frac_obs=frac, ordering=order)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    perm, nbr = V.vecchia_plan_neighbours(plan)
    n_obs = V.vecchia_plan_censoring(plan)
    V.vecchia_plan_destroy(plan)
    assert n_obs == int(rep.observed.sum())
    if D <= 4000:
        operm, onbrs, on = CZ.censored_plan(i.locs, rep.observed, i.ordering, i.m)
        assert on == n_obs and np.array_equal(perm, operm)
        for k in range(D):
            row = nbr[k][nbr[k] >= 0]
            assert np.array_equal(row, onbrs[k]), k
    else:
        base = oracle.ordering.order(i.locs, i.ordering)
        want = np.concatenate([base[rep.observed[base]], base[~rep.observed[base]]])
        assert np.array_equal(perm, want)
        rng = np.random.default_rng(5)
        q = np.unique(np.concatenate([np.arange(0, 24), n_obs + np.arange(0, 24),
                                      rng.choice(D, 300, replace=False), [D - 1]]))
        ref = oracle.neighbours.knn_preceding(i.locs[perm], i.m, queries=q)
        for k, r in zip(q, ref):
            assert np.array_equal(nbr[k][nbr[k] >= 0], r), int(k)


@pytest.mark.parametrize("frac", [0.05, 0.3])
def test_fp64_censored_loglik_matches_the_oracle(frac):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rep = W.censored_replicate(400, 10, 77, frac_obs=frac, n_points=1000, n_shifts=4)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    out, terms = _gpu_loglik(V, torch, plan, i.x, V.as_qmc(i.qmc))
    assert V.vecchia_plan_status(plan) == -1
    V.vecchia_plan_destroy(plan)
    ref = _oracle(rep)
    print("logL", out, ref["logL"], ref["se"], flush=True)
    # a density term can be large (an observed value far from its conditional
    # mean): 1e-10 absolute, or 1e-12 relative for terms beyond 100
    np.testing.assert_allclose(terms[:, 0], ref["terms"][:, 0], rtol=1e-12, atol=FP64_TERM_TOL)
    np.testing.assert_allclose(terms[:, 1], ref["terms"][:, 1], rtol=1e-6, atol=1e-12)
    assert np.all(terms[rep.observed, 1] == 0.0)           # density terms are exact
    assert abs(out[0] - ref["logL"]) <= 1e-10 * max(1.0, abs(ref["logL"]))
    assert abs(out[1] - ref["se"]) <= 1e-6 * ref["se"] + 1e-12


def test_fp32_censored_loglik_within_tolerance():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rep = W.censored_replicate(2500, 10, 99, frac_obs=0.05, n_points=4096, n_shifts=8, rho=0.1)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    q32 = V.make_qmc(i.qmc.n_points, i.qmc.n_shifts, i.qmc.seed, V.VECCHIA_FP32_LOOP)
    q64 = V.make_qmc(i.qmc.n_points, i.qmc.n_shifts, i.qmc.seed, V.VECCHIA_FP64)
    o32, t32 = _gpu_loglik(V, torch, plan, i.x, q32)
    o64, t64 = _gpu_loglik(V, torch, plan, i.x, q64)
    V.vecchia_plan_destroy(plan)
    d = np.abs(t32[:, 0] - t64[:, 0])
    print("fp32", o32, "fp64", o64, "max term diff", d.max(), flush=True)
    assert d.max() <= FP32_TERM_TOL
    assert abs(o32[0] - o64[0]) <= 1e-2 * abs(o64[0])
    # the density terms are computed in FP64 in both modes
    assert np.array_equal(t32[rep.observed, 0], t64[rep.observed, 0])


def test_no_observed_site_equals_the_plain_plan():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(600, 8, 5)
    q = V.as_qmc(inst.qmc)
    p1 = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov)
    p2 = V.vecchia_plan_censored(inst.locs, np.zeros(inst.D, bool), inst.ordering, inst.m, inst.cov)
    a, ta = _gpu_loglik(V, torch, p1, inst.x, q)
    b, tb = _gpu_loglik(V, torch, p2, inst.x, q)
    V.vecchia_plan_destroy(p1)
    V.vecchia_plan_destroy(p2)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)


def test_matrix_plans_exact_cases():
    # all observed with m = D - 1: the library logpdf; equicorrelated with three
    # observed: the oracle on the same explicit covariance
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rng = np.random.default_rng(8)
    pts = rng.random((9, 2))
    S = oracle.covariance.cov_matrix(pts, 0, 0.5, 1.3, 0.5, 0.01)
    x = rng.normal(0.5, 1.0, 9)
    q = V.make_qmc(64, 2, 3, V.VECCHIA_FP64)
    for r in (1.0, 2.5):
        plan = V.vecchia_plan_from_cov_censored(S, 8, 9)
        out, _ = _gpu_loglik(V, torch, plan, x, q, scale=r)
        V.vecchia_plan_destroy(plan)
        want = multivariate_normal(np.zeros(9), S).logpdf(x / r) - 9 * math.log(r)
        assert abs(out[0] - want) <= 1e-11 * abs(want) and out[1] == 0.0
    D, n_I, rho = 8, 3, 0.4
    Sig = (1 - rho) * np.eye(D) + rho
    xe = np.array([1.9, 2.4, 1.7, 0.9, 1.2, 0.4, 1.0, 1.5])
    nb = [list(range(i)) for i in range(D)]
    plan = V.vecchia_plan_from_cov_censored(Sig, 7, n_I, nbr=nb)
    out, terms = _gpu_loglik(V, torch, plan, xe, V.make_qmc(4096, 8, 13, V.VECCHIA_FP64))
    V.vecchia_plan_destroy(plan)
    ref = CZ.loglik_from_cov(Sig, xe, n_I, nb, 4096, 8, 13)
    np.testing.assert_allclose(terms[:, 0], ref["terms"][:, 0], rtol=0.0, atol=FP64_TERM_TOL)
    assert abs(out[0] - ref["logL"]) <= 1e-10 * abs(ref["logL"])


def test_censored_batch_equals_each_replicate_alone():
    # replicates with different numbers of observed sites in one batched launch
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    reps = [W.censored_replicate(300 + 50 * k, 10, 200 + k, frac_obs=0.02 + 0.1 * k) for k in range(4)]
    plans = [V.vecchia_plan_censored(r.inst.locs, r.observed, r.inst.ordering, r.inst.m, r.inst.cov)
             for r in reps]
    qs = [V.as_qmc(r.inst.qmc) for r in reps]
    alone = [_gpu_loglik(V, torch, p, r.inst.x, q, terms=False)[0] for p, r, q in zip(plans, reps, qs)]
    b = V.vecchia_batch_create(plans, qs)
    x = torch.tensor(np.concatenate([r.inst.x for r in reps]), dtype=torch.float64, device="cuda")
    out = torch.empty((len(reps), 2), dtype=torch.float64, device="cuda")
    V.vecchia_batch_logcdf(b, x, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    V.vecchia_batch_destroy(b)
    for p in plans:
        V.vecchia_plan_destroy(p)
    for k in range(len(reps)):
        assert np.array_equal(got[k], alone[k]), k


@pytest.mark.parametrize("beta,gamma", [(0.82, 1.0), (0.0, 2.0)])
def test_censored_mixture_matches_the_oracle(beta, gamma):
    # log G_I(x), eq. (11): the windowed rule over the censored plan on both sides
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rep = W.censored_replicate(150, 6, 123, frac_obs=0.06, n_points=512, n_shifts=4)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    mix = V.make_mixture(beta, gamma, 16)
    x = torch.tensor(i.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    nodes = torch.empty((16, 2), dtype=torch.float64, device="cuda")
    V.vecchia_mixture_logcdf(plan, x, mix, V.as_qmc(i.qmc), out, nodes=nodes)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    V.vecchia_plan_destroy(plan)
    pc = CZ.censored_plan(i.locs, rep.observed, i.ordering, i.m)
    c = i.cov

    def ev(r, n):
        d = CZ.loglik(i.locs, i.x, rep.observed, i.m, c.family, c.nu, c.sigma2, c.range, c.nugget, i.ordering,
                      n, i.qmc.n_shifts, i.qmc.seed, scale=r, plan_cache=pc,
                      processes=oracle.vecchia.default_processes())
        return d["logL"], d["se"]
    ns = M.search_n_points(i.qmc.n_points)
    ref = M.logcdf_mixture(lambda r: ev(r, i.qmc.n_points), beta, gamma, 16, eval_search=lambda r: ev(r, ns))
    print("logG_I", got, ref["logG"], ref["se"], "window", ref["window"], flush=True)
    assert ref["window"][0] > 0.0 or ref["window"][1] < 200.0
    assert abs(got[0] - ref["logG"]) <= 1e-9 * max(1.0, abs(ref["logG"]))
    np.testing.assert_allclose(nodes.cpu().numpy()[:, 0], ref["node_logF"], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32-independent"])
def test_mixture_batch_rows_equal_single_mixtures(precision):
    # the censored log-likelihood over replicates in one batch: row t equals
    # vecchia_mixture_logcdf on replicate t's plan with seed + t, bit for bit, for
    # two successive mixing laws (the batch's launches are reused)
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    prec = V.VECCHIA_FP64 if precision == "fp64" else V.VECCHIA_FP32_LOOP
    indep = precision.endswith("independent")
    reps = [W.censored_replicate(200 + 60 * k, 8, 300 + k, frac_obs=0.04 + 0.05 * k) for k in range(5)]
    plans = [V.vecchia_plan_censored(r.inst.locs, r.observed, r.inst.ordering, r.inst.m, r.inst.cov)
             for r in reps]
    q = V.make_qmc(1024, 4, 41, prec, independent=indep)
    mb = V.vecchia_mixbatch_create(plans, 16, q)
    x = torch.tensor(np.concatenate([r.inst.x for r in reps]), dtype=torch.float64, device="cuda")
    for beta, gamma in ((0.82, 1.0), (0.3, 1.5)):
        mix = V.make_mixture(beta, gamma, 16)
        out = torch.empty((len(reps), 2), dtype=torch.float64, device="cuda")
        total = torch.empty(2, dtype=torch.float64, device="cuda")
        V.vecchia_mixbatch_logcdf(mb, x, mix, out, total=total)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        tot = total.cpu().numpy()
        assert np.all(V.vecchia_mixbatch_status(mb, len(reps)) == -1)
        for t, (p, r) in enumerate(zip(plans, reps)):
            xs = torch.tensor(r.inst.x, dtype=torch.float64, device="cuda")
            one = torch.empty(2, dtype=torch.float64, device="cuda")
            V.vecchia_mixture_logcdf(p, xs, mix, V.make_qmc(1024, 4, 41 + t, prec, independent=indep), one)
            torch.cuda.synchronize()
            assert np.array_equal(got[t], one.cpu().numpy()), (beta, t)
        assert abs(tot[0] - got[:, 0].sum()) <= 1e-12 * abs(tot[0])
        assert abs(tot[1] - math.sqrt(np.sum(got[:, 1] ** 2))) <= 1e-12 * tot[1]
        print("replicates", got[:, 0], "total", tot, flush=True)
    V.vecchia_mixbatch_destroy(mb)
    for p in plans:
        V.vecchia_plan_destroy(p)
