"""Helpers for the GPU tests: run an Instance through the C ABI and through the
oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def gpu_run(inst: W.Instance, precision=None, n_points=None, n_shifts=None, seed=None, stream=None,
            keep_plan=False, scale=None, cov_override=None):
    """Plan + logcdf on cuda:0. Returns dict(out, terms, perm, nbr, bad[, plan])."""
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    q = V.make_qmc(n_points or inst.qmc.n_points, n_shifts or inst.qmc.n_shifts,
                   inst.qmc.seed if seed is None else seed,
                   inst.qmc.precision if precision is None else precision)
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov, perm=inst.perm, stream=stream)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((inst.D, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q, out, scale=inst.scale if scale is None else scale,
                     cov_override=cov_override, terms=terms, stream=stream)
    torch.cuda.synchronize()
    bad = V.vecchia_plan_status(plan)
    perm, nbr = V.vecchia_plan_neighbours(plan)
    res = dict(out=out.cpu().numpy(), terms=terms.cpu().numpy(), perm=perm, nbr=nbr, bad=bad)
    if keep_plan:
        res["plan"] = plan
    else:
        V.vecchia_plan_destroy(plan)
    return res


def oracle_run(inst: W.Instance, n_points=None, n_shifts=None, seed=None, terms_subset=None,
               plan_cache=None, processes=None, scale=None):
    c = inst.cov
    return oracle.logcdf(inst.locs, inst.x, inst.m, c.family, c.nu, c.sigma2, c.range, c.nugget,
                         inst.ordering, n_points or inst.qmc.n_points, n_shifts or inst.qmc.n_shifts,
                         inst.qmc.seed if seed is None else seed,
                         scale=inst.scale if scale is None else scale, perm=inst.perm,
                         terms_subset=terms_subset, plan_cache=plan_cache,
                         processes=processes or oracle.vecchia.default_processes())


def nbr_lists(perm, nbr):
    return [np.array([v for v in row if v >= 0], dtype=np.int64) for row in nbr]


def sample_terms(D: int, m: int, n: int, seed: int):
    """All plan positions with k < m, plus n seeded others (plan indices)."""
    rng = np.random.default_rng(seed)
    head = list(range(min(m + 1, D)))
    rest = rng.choice(np.arange(len(head), D), size=min(n, max(0, D - len(head))), replace=False) \
        if D > len(head) else []
    return sorted(set(head) | set(int(v) for v in rest) | {D - 1})
