"""GPU parity for infinite thresholds, against the oracle: +inf leaves a
component unconstrained; a -inf threshold makes every term that holds it
exactly -inf (SE 0), so log F = -inf; an observed site of a censored plan with
an infinite value has density 0. Bars as in the other parity tests: FP64
1e-10 per term, FP32 1e-3 per term and 1e-2 relative in log F; the exact
values (0 for a term whose own limit is +inf, -inf) must match exactly."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import block as BZ
from oracle import censored as CZ
from tests.gpu_helpers import gpu_run, oracle_run, torch_cuda

pytestmark = pytest.mark.gpu


def _with_limits(D, m, seed, n_inf, sign, N, R, precision):
    inst = W.small_random_instance(D, m, seed, n_points=N, n_shifts=R, precision=precision)
    rng = np.random.default_rng(seed + 1000)
    idx = rng.choice(D, size=n_inf, replace=False)
    x = inst.x.copy()
    x[idx] = sign * np.inf
    inst.x = x
    return inst, idx


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
@pytest.mark.parametrize("D,m,N,R,seed", [(200, 10, 300, 3, 41), (64, 31, 130, 2, 43), (90, 40, 200, 2, 42)])
def test_plus_inf_thresholds_match_the_oracle(prec, D, m, N, R, seed):
    inst, idx = _with_limits(D, m, seed, D // 8, 1.0, N, R, prec)
    g = gpu_run(inst, precision=prec)
    o = oracle_run(inst)
    gt, ot = g["terms"], o["terms"]
    assert np.all(np.isfinite(gt))
    # a term whose own limit is +inf is exactly 0 on both sides
    assert np.all(gt[idx] == 0.0) and np.all(ot[idx] == 0.0)
    tol = 1e-10 if prec == W.PREC_FP64 else 1e-3
    d = np.abs(gt[:, 0] - ot[:, 0])
    assert d.max() <= tol, (d.max(), int(np.argmax(d)))
    if prec == W.PREC_FP64:
        np.testing.assert_allclose(gt[:, 1], ot[:, 1], rtol=1e-6, atol=1e-12)
        assert abs(g["out"][0] - o["logF"]) <= 1e-10
    else:
        assert abs(g["out"][0] - o["logF"]) <= 1e-2 * abs(o["logF"])


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_minus_inf_threshold_gives_minus_inf(prec):
    base = W.small_random_instance(150, 10, 45, n_points=256, n_shifts=3, precision=prec)
    g0 = gpu_run(base, precision=prec)
    inst, idx = _with_limits(150, 10, 45, 1, -1.0, 256, 3, prec)
    g = gpu_run(inst, precision=prec)
    # the total SE still adds up the other terms' errors in quadrature
    assert g["out"][0] == -math.inf
    assert g["out"][1] == pytest.approx(math.sqrt(np.sum(g["terms"][:, 1] ** 2)), rel=1e-12)
    assert g["bad"] == -1
    perm, nbr = g["perm"], g["nbr"]
    pj = int(np.flatnonzero(perm == idx[0])[0])
    for i in range(150):
        involved = i == pj or pj in set(int(v) for v in nbr[i] if v >= 0)
        u = perm[i]
        if involved:
            assert g["terms"][u, 0] == -math.inf and g["terms"][u, 1] == 0.0, i
        else:
            assert np.array_equal(g["terms"][u], g0["terms"][u]), i
    if prec == W.PREC_FP64:
        o = oracle_run(inst)
        assert o["logF"] == -math.inf
        fin = np.isfinite(o["terms"][:, 0])
        assert np.array_equal(fin, np.isfinite(g["terms"][:, 0]))
        assert np.max(np.abs(g["terms"][fin, 0] - o["terms"][fin, 0])) <= 1e-10


def test_block_plan_with_infinite_limits():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    inst = W.small_random_instance(60, 3, 47, n_points=256, n_shifts=3)
    x = inst.x.copy()
    x[[3, 11, 40]] = np.inf
    c = inst.cov
    plan = V.vecchia_plan_block(inst.locs, inst.ordering, 3, 3, c)
    q = V.make_qmc(256, 3, inst.qmc.seed, V.VECCHIA_FP64)
    nt = V.plan_n_terms(plan)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((nt, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, xt, q, out, terms=terms)
    torch.cuda.synchronize()
    o = BZ.logcdf_block(inst.locs, x, 3, 3, c.family, c.nu, c.sigma2, c.range, c.nugget, inst.ordering,
                        256, 3, inst.qmc.seed)
    assert np.max(np.abs(terms.cpu().numpy()[:, 0] - o["terms"][:, 0])) <= 1e-10
    x[20] = -np.inf
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, xt, q, out, terms=terms)
    torch.cuda.synchronize()
    assert out.cpu().numpy()[0] == -math.inf
    V.vecchia_plan_destroy(plan)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_censored_plan_with_infinite_values(prec):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    rep = W.censored_replicate(300, 10, 49, frac_obs=0.1, n_points=512, n_shifts=3)
    i = rep.inst
    plan = V.vecchia_plan_censored(i.locs, rep.observed, i.ordering, i.m, i.cov)
    q = V.make_qmc(512, 3, i.qmc.seed, prec)
    obs_idx = np.flatnonzero(rep.observed)
    cen_idx = np.flatnonzero(~rep.observed)

    def run(x_np):
        x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        t = torch.empty((300, 2), dtype=torch.float64, device="cuda")
        V.vecchia_logcdf(plan, x, q, out, terms=t)
        torch.cuda.synchronize()
        return out.cpu().numpy(), t.cpu().numpy()

    x1 = i.x.copy()
    x1[cen_idx[:5]] = np.inf           # censored at +inf: no constraint
    out, terms = run(x1)
    assert np.isfinite(out[0])
    assert np.all(terms[cen_idx[:5]] == 0.0)
    c = i.cov
    ref = CZ.loglik(i.locs, x1, rep.observed, i.m, c.family, c.nu, c.sigma2, c.range, c.nugget, i.ordering,
                    512, 3, i.qmc.seed, perm=i.perm, processes=oracle.vecchia.default_processes())
    tol = 1e-10 if prec == W.PREC_FP64 else 1e-3
    assert np.max(np.abs(terms[:, 0] - ref["terms"][:, 0])) <= tol
    x2 = i.x.copy()
    x2[obs_idx[0]] = np.inf            # an observed value at +inf: density 0
    out, terms = run(x2)
    assert out[0] == -math.inf
    assert terms[obs_idx[0], 0] == -math.inf and terms[obs_idx[0], 1] == 0.0
    V.vecchia_plan_destroy(plan)


def test_mixture_of_a_minus_inf_threshold_is_minus_inf():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    S = np.array([[1.0, 0.3, 0.5], [0.3, 1.0, 0.2], [0.5, 0.2, 1.0]])
    plan = V.vecchia_plan_from_cov(S, 2)
    q = V.make_qmc(1024, 4, 5, V.VECCHIA_FP32_LOOP)
    mix = V.make_mixture(0.0, 2.0, 16)
    x = torch.tensor([0.5, -np.inf, 1.0], dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    V.vecchia_mixture_logcdf(plan, x, mix, q, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[0] == -math.inf and got[1] == 0.0
    V.vecchia_plan_destroy(plan)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_largest_point_count_against_the_closed_form(prec):
    # N = VECCHIA_MAX_POINTS = 2^30 lattice points: 2^19..2^21 work items for one
    # bivariate term, whose value is Owen's closed form
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    from tests import closed_forms as cf
    rho = 0.6
    S = np.array([[1.0, rho], [rho, 1.0]])
    b = np.array([0.4, -0.3])
    plan = V.vecchia_plan_from_cov(S, 1)
    x = torch.tensor(b, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((2, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, V.make_qmc(V.VECCHIA_MAX_POINTS, 2, 3, prec), out, terms=terms)
    torch.cuda.synchronize()
    V.vecchia_plan_destroy(plan)
    t = terms.cpu().numpy()
    want = math.log(cf.bivariate_owen(b[0], b[1], rho))
    tol = 1e-9 if prec == W.PREC_FP64 else 1e-6
    assert abs(out.cpu().numpy()[0] - want) <= tol, (out.cpu().numpy(), want)
    assert t[1, 1] < 1e-6


def test_largest_shift_count_matches_the_oracle():
    # R = VECCHIA_MAX_SHIFTS = 65536 shifts of 64 points: the finalize's per-lane
    # loops over shifts and its SE at their longest
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    S = np.array([[1.0, 0.45], [0.45, 1.0]])
    b = np.array([0.2, 0.9])
    plan = V.vecchia_plan_from_cov(S, 1)
    x = torch.tensor(b, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((2, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, V.make_qmc(64, V.VECCHIA_MAX_SHIFTS, 5, V.VECCHIA_FP64), out, terms=terms)
    torch.cuda.synchronize()
    V.vecchia_plan_destroy(plan)
    o = oracle.logcdf_from_cov(S, b, [[], [0]], 64, V.VECCHIA_MAX_SHIFTS, 5)
    t = terms.cpu().numpy()
    assert np.max(np.abs(t[:, 0] - o["terms"][:, 0])) <= 1e-10
    np.testing.assert_allclose(t[:, 1], o["terms"][:, 1], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("kind", ["block", "censored", "independent"])
def test_promoted_terms_of_every_plan_kind_match_fp64(kind):
    # deep lower-tail thresholds: FP32 evaluations hand the terms with a limit below
    # -4 sd to the FP64 kernel; block terms (denominator split), censored terms
    # (conditional rows) and the second lattice of the independent-points estimator
    # must all come out as in the FP64 mode
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    if kind == "censored":
        rep = W.censored_replicate(260, 8, 91, frac_obs=0.1, n_points=600, n_shifts=3)
        inst, observed = rep.inst, rep.observed
        x = inst.x.copy()
        x[~observed] -= 3.5                         # censoring limits deep in the lower tail
        plan = V.vecchia_plan_censored(inst.locs, observed, inst.ordering, inst.m, inst.cov)
    else:
        inst = W.small_random_instance(220, 4 if kind == "block" else 8, 92, n_points=600, n_shifts=3,
                                       mean_x=-2.0, sd_x=0.7)
        x = inst.x / 0.7
        plan = (V.vecchia_plan_block(inst.locs, inst.ordering, 4, 3, inst.cov) if kind == "block"
                else V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov))
    nt = V.plan_n_terms(plan)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    res = {}
    for prec in (V.VECCHIA_FP64, V.VECCHIA_FP32_LOOP):
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        t = torch.empty((nt, 2), dtype=torch.float64, device="cuda")
        V.vecchia_logcdf(plan, xt, V.make_qmc(600, 3, 5, prec, independent=kind == "independent"), out, terms=t)
        torch.cuda.synchronize()
        res[prec] = (out.cpu().numpy(), t.cpu().numpy())
    V.vecchia_plan_destroy(plan)
    t64, t32 = res[V.VECCHIA_FP64][1], res[V.VECCHIA_FP32_LOOP][1]
    fin = np.isfinite(t64[:, 0])
    d = np.abs(t32[fin, 0] - t64[fin, 0])
    assert np.all(d <= 1e-3), (d.max(), int(np.argmax(d)))
    # some terms were promoted: their values agree with FP64 to rounding
    assert np.sum(d <= 1e-10) > 0
