"""Benchmark of the Vecchia log-CDF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections c1,c2,c3,c4,c5,mix,cens,full]

Headline workload (the JSON line's value): D = 2,500 locations uniform in
[0,1]^2, Matern nu = 3/2 (range 0.1, nugget 1e-8), maxmin ordering, m = 10,
thresholds at the 0.9 marginal quantile plus N(0, 0.1^2) noise, 10^4 lattice
points x 10 shifts, FP32 SOV loop with FP64 Cholesky / accumulation. Inputs are
seeded synthetic data (workloads/); thresholds are resident on the device
before timing.

One step = the whole path for one instance: vecchia_replan (host maxmin
ordering + the GPU nearest-preceding-neighbour kernel) followed by
vecchia_logcdf (covariance + Cholesky, the QMC kernels, the segmented log-sum).
K steps are timed between two device synchronisations; value = terms per second
(D terms per step). The line also carries samples/s, the log-CDF-only rate,
the plain FP64 rate on the same inputs, the independent-points estimator's
time and SE beside the shared lattice's, the FP32-vs-FP64 error, the roofline of
the dominant kernel (its HIP-event time over the timed region), the CPU oracle
baseline on a bounded sample, and one object per further workload:
  c1_grid     D = 400 on a 20 x 20 grid, exponential covariance, coordinate
              order, m = 5, 1000 x 10 points: the plain FP64 form (and FP32);
  c3_batched  512 instances (D log-uniform in [100, 20000], m in {5,10,15,20},
              nu in {0.5,1.5,2.5}) in one batched evaluation, 4096 x 8 points;
  c4_large    D = 250,000, m = 20, thresholds at the 0.95 quantile, FP32 and
              FP64 on the same plan, 10^4 x 10 points;
  c5_serving  mixed requests (D in [1000, 100000], m in 5..30, per-request
              range and scale factor, 2048-8192 x 8 points) through the serving
              loop: capacity with every request queued at once, then Poisson
              arrivals at 80 % of it with p50/p99 latency;
  scale_mixture  the scale-mixture CDF E Phi_D(x / R), R Pareto(2), on the headline
              geometry (24 search evaluations at 1/16 size + 48 nodes per call);
  censored_likelihood  the censored log-likelihood of Section 4 over 1006 weekly
              replicates on 528 stations (about 356 present, 18 censored-above
              per week), anisotropic exponential model at Table 1's values,
              m = 10, 1000 x 10 points, 48 nodes per replicate, in one
              mixture batch; FP64 on 128 replicates for the comparison;
  full_dimension_comparator  the full-dimension SOV estimate against the
              Vecchia log-CDF (m = 5, 10, 30, 50) on 15 x 15 to 100 x 100
              grids of unit spacing, exponential range 1 and 5, 3607 x 10
              points (Section 3.1).
The launch shape of each workload is set by vecchia_autotune beforehand.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Dominant kernel figures used by the roofline (qmc_f32<10>, gfx950 build):
# VALU instructions per SOV step counted on the main path of the kernel's
# unrolled chain in its assembly (482 per 10-step chain, rare branches not
# taken); updated whenever the kernel changes.
SLOTS_PER_STEP_F32_K10 = 48.2
# MI355X FP32 vector peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 FMA lanes x 2:
# 78.64e12 full-rate VALU lane-slots per second.
VALU_PEAK_TSLOTS = 256 * 2.4e9 * 128 / 1e12
# Transcendental instructions per SOV step on that path (the rest are full-rate):
# Phi^-1 takes a log2, a sqrt and a reciprocal, Phi a reciprocal and an exp2.
TRANS_PER_STEP = {"exp": 1, "log": 1, "rcp": 2, "sqrt": 1}
# HBM bytes per launch of qmc_f32<10> from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (factors from a 256 MiB copy); None once the kernel changes.
TRAFFIC_BYTES_F32_K10 = 12.28e6    # (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000) per launch, profiles/qmc_f32_k10_uniform2500_pmc.md


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="uniform2500_matern15_m10",
                    choices=["uniform2500_matern15_m10", "grid400_exp_m5"])
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-terms", type=int, default=500)
    ap.add_argument("--fp32-only", action="store_true",
                    help="time the full FP32 step only (short runs under a profiler)")
    ap.add_argument("--censored-T", type=int, default=1006)
    ap.add_argument("--comparator-grids", type=lambda v: [int(t) for t in v.split(",")], default=[15, 30, 50, 75, 100])
    ap.add_argument("--sections", default="c1,c2,c3,c4,c5,mix,cens,full",
                    help="comma list of workloads to run besides the headline (c2 is always run)")
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--no-autotune", action="store_true")
    return ap.parse_args()


def make_instance(name):
    import workloads as W
    if name == "grid400_exp_m5":
        return W.grid400_exponential(precision=W.PREC_FP32)
    return W.uniform2500_matern15(precision=W.PREC_FP32)


def cpu_baseline(inst, n_terms):
    """The oracle as it stands on a bounded sample: its own plan of all D
    locations plus n_terms seeded terms; extrapolated to the full workload."""
    import oracle
    c = inst.cov
    procs = oracle.vecchia.default_processes()
    t0 = time.perf_counter()
    perm, nbrs = oracle.plan(inst.locs, inst.ordering, inst.m)
    t_plan = time.perf_counter() - t0
    rng = np.random.default_rng(7)
    sub = sorted(rng.choice(inst.D, size=min(n_terms, inst.D), replace=False).tolist())
    t0 = time.perf_counter()
    oracle.logcdf(inst.locs, inst.x, inst.m, c.family, c.nu, c.sigma2, c.range, c.nugget,
                  inst.ordering, inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed,
                  terms_subset=sub, plan_cache=(perm, nbrs), processes=procs)
    t_terms = time.perf_counter() - t0
    t_full = t_plan + t_terms * inst.D / len(sub)
    # one core: a smaller seeded sample in this process
    sub1 = sub[:max(1, len(sub) // 10)]
    t0 = time.perf_counter()
    oracle.logcdf(inst.locs, inst.x, inst.m, c.family, c.nu, c.sigma2, c.range, c.nugget,
                  inst.ordering, inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed,
                  terms_subset=sub1, plan_cache=(perm, nbrs), processes=1)
    t_one = time.perf_counter() - t0
    return {"value": inst.D / t_full, "unit": "terms/s", "cores": procs, "kind": "oracle",
            "sample": f"plan of all {inst.D} locations ({t_plan:.2f} s) + {len(sub)} of {inst.D} "
                      f"terms ({t_terms:.2f} s on {procs} processes), extrapolated to all terms",
            "single_core": {"value": inst.D / (t_plan + t_one * inst.D / len(sub1)), "unit": "terms/s",
                            "sample": f"the same plan + {len(sub1)} terms ({t_one:.2f} s) in one process"}}


def autotune(V, n_points, n_shifts, ms, sp):
    """Launch shape for both precisions at this workload's N, R and m values."""
    t0 = time.perf_counter()
    c32, _ = V.vecchia_autotune(V.VECCHIA_FP32_LOOP, n_points, n_shifts, ms, stream=sp)
    c64, _ = V.vecchia_autotune(V.VECCHIA_FP64, n_points, n_shifts, ms, stream=sp)
    return {"n_points": n_points, "n_shifts": n_shifts, "m": list(ms), "chunk_points_fp32": c32,
            "chunk_points_fp64": c64, "seconds": time.perf_counter() - t0}


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_c1(V, torch, args):
    """400-point grid, exponential covariance, coordinate order, m = 5: the plain FP64 form."""
    import workloads as W
    inst = W.grid400_exponential()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov, stream=sp)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    N, R, m, D = inst.qmc.n_points, inst.qmc.n_shifts, inst.m, inst.D
    res = {"workload": inst.name, "D": D, "m": m, "n_points": N, "n_shifts": R}
    for name, prec in (("fp64", V.VECCHIA_FP64), ("fp32", V.VECCHIA_FP32_LOOP)):
        q = V.make_qmc(N, R, inst.qmc.seed, prec)
        sec = _timed(torch, lambda: V.vecchia_logcdf(plan, x, q, out, stream=sp), 20)
        o = out.cpu().numpy()
        res[name] = {"ms": 1e3 * sec, "terms_per_s": D / sec, "samples_per_s": D * N * R / sec,
                     "logF": float(o[0]), "se": float(o[1])}
    V.vecchia_plan_destroy(plan)
    return res


def bench_mixture(V, torch, args):
    """Scale-mixture CDF G(x) = E Phi_D(x / R), R Pareto(gamma = 2) (eqs. (8)-(9)),
    on the headline geometry: 24 search evaluations at 1/16 of the lattice size,
    then 48 Gauss-Legendre nodes."""
    import workloads as W
    inst = W.uniform2500_matern15()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov, stream=sp)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    n_nodes = 48
    mix = V.make_mixture(0.0, 2.0, n_nodes)
    n_search = max(64, ((inst.qmc.n_points // 16 + 63) // 64) * 64)
    full_equiv = n_nodes + V.MIX_SEARCH_NODES * n_search / inst.qmc.n_points
    res = {"workload": inst.name + "_pareto2_mixture", "beta": 0.0, "gamma": 2.0, "n_nodes": n_nodes,
           "search_evaluations": V.MIX_SEARCH_NODES, "search_n_points": n_search,
           "full_size_evaluations_per_call": full_equiv}
    got = {}
    for name, prec, reps in (("fp32", V.VECCHIA_FP32_LOOP, 5), ("fp64", V.VECCHIA_FP64, 1)):
        q = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, prec)
        sec = _timed(torch, lambda: V.vecchia_mixture_logcdf(plan, x, mix, q, out, stream=sp), reps)
        o = out.cpu().numpy()
        got[name] = o
        res[name] = {"ms_per_call": 1e3 * sec, "calls_per_s": 1.0 / sec,
                     "terms_per_s": full_equiv * inst.D / sec, "logG": float(o[0]), "se": float(o[1])}
    res["fp32_speedup"] = res["fp64"]["ms_per_call"] / res["fp32"]["ms_per_call"]
    res["fp32_vs_fp64_rel"] = abs(got["fp32"][0] - got["fp64"][0]) / abs(got["fp64"][0])
    V.vecchia_plan_destroy(plan)
    return res


def bench_comparator(V, torch, args):
    """Full-dimension SOV (the paper's comparator, Section 3.1) against the
    Vecchia log-CDF on the simulation study's setting: regular grids of 15 x 15
    to 100 x 100 sites with unit spacing, exponential covariance with
    range 1 and 5, thresholds one smooth-field draw of that scale, 3607 lattice
    points x 10 shifts (the larger QM size of the study); Vecchia at m = 5, 10,
    30 and 50 in FP32 and FP64. Times are per call with inputs resident."""
    import workloads as W
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    N, R = 3607, 10
    rows = []
    for rho in (1.0, 5.0):
        for n in args.comparator_grids:
            locs = W.grid_locations(n, n) * (n - 1)
            rng = np.random.Generator(np.random.PCG64(W.seed_for(7, n) + int(rho)))
            xv = W.smooth_field(locs, rng, 0.5, rho)
            cov = V.make_cov(V.VECCHIA_COV_EXPONENTIAL, 0.5, 1.0, rho, 0.0)
            x = torch.tensor(xv, dtype=torch.float64, device="cuda")
            out = torch.empty(2, dtype=torch.float64, device="cuda")
            D = n * n
            row = {"grid": f"{n}x{n}", "D": D, "range": rho}
            plan = V.vecchia_plan(locs, V.VECCHIA_ORDER_MAXMIN, 30, cov, stream=sp)
            q64 = V.make_qmc(N, R, 11, V.VECCHIA_FP64)
            sec = _timed(torch, lambda: V.vecchia_full_logcdf(plan, x, q64, out, stream=sp), 1)
            o = out.cpu().numpy()
            row["full_sov_fp64"] = {"seconds": sec, "logF": float(o[0]), "se": float(o[1]),
                                    "points_per_s": N * R / sec}
            V.vecchia_plan_destroy(plan)
            for m in (5, 10, 30, 50):
                p = V.vecchia_plan(locs, V.VECCHIA_ORDER_MAXMIN, m, cov, stream=sp)
                for name, prec in (("fp32", V.VECCHIA_FP32_LOOP), ("fp64", V.VECCHIA_FP64)):
                    q = V.make_qmc(N, R, 11, prec)
                    sec = _timed(torch, lambda: V.vecchia_logcdf(p, x, q, out, stream=sp), 3)
                    o = out.cpu().numpy()
                    row[f"vecchia_m{m}_{name}"] = {"seconds": sec, "logF": float(o[0]), "se": float(o[1])}
                V.vecchia_plan_destroy(p)
            rows.append(row)
    return {"workload": "exp_grids_unit_spacing_comparator", "n_points": N, "n_shifts": R, "rows": rows}


# Section 4.1 / Table 1: range, rotation angle, aspect ratio and mixing law
# of the application's fitted model (gamma fixed at 1).
APP_RHO, APP_PHI, APP_ASPECT, APP_BETA, APP_GAMMA = 1.31, 1.10, 2.29, 0.82, 1.0


def bench_censored(V, torch, args):
    """Censored log-likelihood sum_t log G_{I_t}(x_t) (Section 4, eqs. (9), (11))
    over T = 1006 weekly replicates on 528 stations (about 356 present and 18
    above the censoring level per week), anisotropic exponential covariance
    through the coordinate map, m = 10, 1000 x 10 lattice points, 48 nodes per
    replicate, all replicates in one mixture batch; FP64 on the first 128
    replicates for the precision comparison."""
    import workloads as W
    _, reps = W.network_replicates(T=args.censored_T, n_points=1000, n_shifts=10)
    T = len(reps)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    cov = V.make_cov(V.VECCHIA_COV_EXPONENTIAL, 0.5, 1.0, APP_RHO, 0.0)
    t0 = time.perf_counter()
    plans = []
    for r in reps:
        mapped = V.vecchia_map_anisotropic(r.inst.locs, APP_PHI, APP_ASPECT)
        plans.append(V.vecchia_plan_censored(mapped, r.observed, V.VECCHIA_ORDER_MAXMIN, 10, cov, stream=sp))
    t_plans = time.perf_counter() - t0
    D = np.array([r.inst.D for r in reps])
    n_obs = np.array([int(r.observed.sum()) for r in reps])
    n_nodes = 48
    mix = V.make_mixture(APP_BETA, APP_GAMMA, n_nodes)
    n_search = max(64, ((1000 // 16 + 63) // 64) * 64)
    res = {"workload": f"network528_T{T}_censored_m10", "replicates": T, "mean_D": float(D.mean()),
           "mean_observed": float(n_obs.mean()), "n_points": 1000, "n_shifts": 10, "n_nodes": n_nodes,
           "search_n_points": n_search, "beta": APP_BETA, "gamma": APP_GAMMA, "plan_seconds": t_plans}
    got = {}
    for name, prec, nrep, reps_t in (("fp32", V.VECCHIA_FP32_LOOP, T, 2), ("fp64", V.VECCHIA_FP64, min(T, 128), 1),
                                     ("fp32_subset", V.VECCHIA_FP32_LOOP, min(T, 128), 2)):
        q = V.make_qmc(1000, 10, 2024, prec)
        mb = V.vecchia_mixbatch_create(plans[:nrep], n_nodes, q)
        x = torch.tensor(np.concatenate([r.inst.x for r in reps[:nrep]]), dtype=torch.float64, device="cuda")
        out = torch.empty((nrep, 2), dtype=torch.float64, device="cuda")
        total = torch.empty(2, dtype=torch.float64, device="cuda")
        sec = _timed(torch, lambda: V.vecchia_mixbatch_logcdf(mb, x, mix, out, total=total, stream=sp), reps_t)
        o = out.cpu().numpy()
        tot = total.cpu().numpy()
        got[name] = o
        terms = float(D[:nrep].sum()) * (n_nodes + V.MIX_SEARCH_NODES * n_search / 1000)
        res[name] = {"replicates": nrep, "seconds_per_likelihood": sec, "replicates_per_s": nrep / sec,
                     "full_size_terms_per_s": terms / sec, "loglik": float(tot[0]), "se": float(tot[1])}
        V.vecchia_mixbatch_destroy(mb)
    res["fp32_speedup_on_subset"] = res["fp64"]["seconds_per_likelihood"] / res["fp32_subset"]["seconds_per_likelihood"]
    d = np.abs(got["fp32_subset"][:, 0] - got["fp64"][:, 0])
    res["fp32_vs_fp64"] = {"max_abs_replicate": float(d.max()),
                           "rel_total": abs(got["fp32_subset"][:, 0].sum() - got["fp64"][:, 0].sum())
                           / abs(got["fp64"][:, 0].sum())}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_censored(reps, n_nodes, 2024)
    for p in plans:
        V.vecchia_plan_destroy(p)
    return res


def cpu_baseline_censored(reps, n_nodes, seed):
    """The oracle on one replicate (the first with the median number of present
    sites): its full mixture rule over the censored Vecchia terms."""
    import oracle
    from oracle import censored as CZ
    from oracle import mixture as M
    import workloads as W
    D = np.array([r.inst.D for r in reps])
    t = int(np.flatnonzero(D == int(np.median(D)))[0]) if np.any(D == int(np.median(D))) else 0
    r = reps[t]
    procs = oracle.vecchia.default_processes()
    mapped = oracle.covariance.anisotropic_coords(r.inst.locs, APP_PHI, APP_ASPECT)
    t0 = time.perf_counter()
    pc = CZ.censored_plan(mapped, r.observed, W.ORDER_MAXMIN, 10)

    def ev(scale, n):
        d = CZ.loglik(mapped, r.inst.x, r.observed, 10, W.COV_EXPONENTIAL, 0.5, 1.0, APP_RHO, 0.0, W.ORDER_MAXMIN,
                      n, 10, seed + t, scale=scale, plan_cache=pc, processes=procs)
        return d["logL"], d["se"]
    ns = M.search_n_points(1000)
    M.logcdf_mixture(lambda sc: ev(sc, 1000), APP_BETA, APP_GAMMA, n_nodes, eval_search=lambda sc: ev(sc, ns))
    sec = time.perf_counter() - t0
    return {"value": 1.0 / sec, "unit": "replicates/s", "cores": procs, "kind": "oracle",
            "sample": f"replicate {t} (D = {r.inst.D}, {int(r.observed.sum())} observed): plan, 24 search and "
                      f"{n_nodes} node evaluations ({sec:.1f} s on {procs} processes)"}


def bench_c3(V, torch, args):
    """512 instances of mixed D, m and nu in one batched evaluation (FP32 loop)."""
    import workloads as W
    insts = W.batched_uneven()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    tuned = None if args.no_autotune else autotune(V, 4096, 8, [5, 10, 15, 20], sp)
    t0 = time.perf_counter()
    plans = [V.vecchia_plan(i.locs, i.ordering, i.m, i.cov, stream=sp) for i in insts]
    t_plans = time.perf_counter() - t0
    terms = sum(i.D for i in insts)
    chains = sum(i.D * i.qmc.n_points * i.qmc.n_shifts for i in insts)
    steps = sum(i.qmc.n_points * i.qmc.n_shifts * (i.m * (i.D - i.m) + i.m * (i.m - 1) // 2) for i in insts)
    x = torch.tensor(np.concatenate([i.x for i in insts]), dtype=torch.float64, device="cuda")
    out = torch.empty((len(insts), 2), dtype=torch.float64, device="cuda")
    res = {"workload": "batched_uneven_512", "instances": len(insts), "terms": terms,
           "plan_seconds_all": t_plans}
    for name, prec, reps in (("fp32", V.VECCHIA_FP32_LOOP, 3), ("fp64", V.VECCHIA_FP64, 1)):
        batch = V.vecchia_batch_create(plans, [V.make_qmc(i.qmc.n_points, i.qmc.n_shifts, i.qmc.seed, prec)
                                               for i in insts])
        torch.cuda.synchronize()
        sec = _timed(torch, lambda: V.vecchia_batch_logcdf(batch, x, out, stream=sp), reps)
        res[name] = {"ms": 1e3 * sec, "terms_per_s": terms / sec, "samples_per_s": chains / sec,
                     "sov_steps_per_s": steps / sec}
        bad = V.vecchia_batch_status(batch, len(insts))
        res[name]["not_pd_instances"] = int(np.sum(bad >= 0))
        if name == "fp32":
            o32 = out.cpu().numpy().copy()
        else:
            o64 = out.cpu().numpy().copy()
        V.vecchia_batch_destroy(batch)
    rel = np.abs(o32[:, 0] - o64[:, 0]) / np.abs(o64[:, 0])
    res["fp32_vs_fp64_rel_total"] = {"max": float(rel.max()), "median": float(np.median(rel))}
    res["fp32_speedup"] = res["fp64"]["ms"] / res["fp32"]["ms"]
    if tuned is not None:
        res["autotune"] = tuned
    for p in plans:
        V.vecchia_plan_destroy(p)
    return res


def bench_c4(V, torch, args):
    """D = 250,000, m = 20, thresholds at the 0.95 quantile: FP32 and FP64."""
    import workloads as W
    inst = W.uniform250k_tail()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    tuned = None if args.no_autotune else autotune(V, inst.qmc.n_points, inst.qmc.n_shifts, [inst.m], sp)
    t0 = time.perf_counter()
    plan = V.vecchia_plan(inst.locs, inst.ordering, inst.m, inst.cov, stream=sp)
    t_plan = time.perf_counter() - t0
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = torch.empty((inst.D, 2), dtype=torch.float64, device="cuda")
    N, R, m, D = inst.qmc.n_points, inst.qmc.n_shifts, inst.m, inst.D
    steps = N * R * (m * (D - m) + m * (m - 1) // 2)
    res = {"workload": inst.name, "D": D, "m": m, "n_points": N, "n_shifts": R, "plan_seconds": t_plan}
    got = {}
    for name, prec, reps in (("fp32", V.VECCHIA_FP32_LOOP, 3), ("fp64", V.VECCHIA_FP64, 1)):
        q = V.make_qmc(N, R, inst.qmc.seed, prec)
        sec = _timed(torch, lambda: V.vecchia_logcdf(plan, x, q, out, stream=sp), reps)
        V.vecchia_logcdf(plan, x, q, out, terms=terms, stream=sp)
        torch.cuda.synchronize()
        got[name] = (out.cpu().numpy().copy(), terms.cpu().numpy()[:, 0].copy())
        res[name] = {"ms": 1e3 * sec, "terms_per_s": D / sec, "samples_per_s": D * N * R / sec,
                     "sov_steps_per_s": steps / sec, "logF": float(got[name][0][0]), "se": float(got[name][0][1])}
    res["fp32_speedup"] = res["fp64"]["ms"] / res["fp32"]["ms"]
    d = np.abs(got["fp32"][1] - got["fp64"][1])
    nz = got["fp64"][1] != 0.0          # log-terms that round to 0 in FP64 have no relative error
    res["fp32_vs_fp64"] = {"rel_total": abs(got["fp32"][0][0] - got["fp64"][0][0]) / abs(got["fp64"][0][0]),
                           "max_abs_term": float(d.max()),
                           "max_rel_term": float(np.max(d[nz] / np.abs(got["fp64"][1][nz]))),
                           "terms_rounding_to_zero": int(np.sum(~nz))}
    if tuned is not None:
        res["autotune"] = tuned
    V.vecchia_plan_destroy(plan)
    return res


def _serve(V, srv, plans, reqs, xs, arrivals):
    """Submit each request at its arrival time (seconds from start), poll until
    all are done; returns (wall seconds, latencies)."""
    pending = {}
    lat = []
    t0 = time.perf_counter()
    k = 0
    while k < len(reqs) or pending:
        now = time.perf_counter() - t0
        while k < len(reqs) and arrivals[k] <= now:
            r = reqs[k]
            pending[k] = V.vecchia_submit(srv, plans[r.plan_id], xs[k], r.qmc, scale=r.scale, cov_override=r.cov)
            k += 1
        for j in list(pending):
            got = V.vecchia_poll(srv, pending[j])
            if got is not None:
                lat.append(got[2])
                del pending[j]
        time.sleep(0.0002)
    return time.perf_counter() - t0, np.array(lat)


def bench_c5(V, torch, args):
    """Serving loop: capacity, then Poisson arrivals at 80 % of it."""
    import workloads as W
    st = W.serving_stream(n_requests=args.serving_requests)
    t0 = time.perf_counter()
    plans = [V.vecchia_plan(p.locs, p.ordering, p.m, p.cov) for p in st.plans]
    t_plans = time.perf_counter() - t0
    xs = [torch.tensor(r.x, dtype=torch.float64, device="cuda") for r in st.requests]
    torch.cuda.synchronize()
    reqs = st.requests
    terms = sum(st.plans[r.plan_id].D for r in reqs)
    srv = V.vecchia_server_create(8 << 30, 16)
    # warm-up: a few requests (first launches, graph-free server path)
    _serve(V, srv, plans, reqs[:8], xs[:8], np.zeros(8))
    wall, lat_cap = _serve(V, srv, plans, reqs, xs, np.zeros(len(reqs)))
    rate = len(reqs) / wall
    arr = np.array([r.arrival_s for r in reqs])
    arr = arr / arr[-1] * (len(reqs) / (0.8 * rate))          # same Poisson pattern at 80 % load
    wall80, lat = _serve(V, srv, plans, reqs, xs, arr)
    V.vecchia_server_destroy(srv)
    for p in plans:
        V.vecchia_plan_destroy(p)
    return {"workload": "serving_stream", "plans": len(plans), "requests": len(reqs),
            "plan_seconds_all": t_plans, "hbm_budget_bytes": 8 << 30, "slots": 16,
            "capacity": {"requests_per_s": rate, "terms_per_s": terms / wall},
            "poisson_80pct": {"offered_requests_per_s": 0.8 * rate, "requests_per_s": len(reqs) / wall80,
                              "terms_per_s": terms / wall80,
                              "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
                              "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
                              "latency_ms_max": 1e3 * float(lat.max())}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the terms of an instance are independent, so a multi-GPU run would split them by range)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2007_15195_amd import vecchia as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    inst = make_instance(args.workload)
    D, m = inst.D, inst.m
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    tuned = None
    if not args.no_autotune and not args.fp32_only:
        tuned = autotune(V, inst.qmc.n_points, inst.qmc.n_shifts, [m], sp)
    plan = V.vecchia_plan(inst.locs, inst.ordering, m, inst.cov, stream=sp)
    x = torch.tensor(inst.x, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q32 = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, V.VECCHIA_FP32_LOOP)
    q64 = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, V.VECCHIA_FP64)
    torch.cuda.synchronize()                     # inputs resident before the bench stream uses them
    n_qmc_terms = D - 1 if m > 0 else 0          # terms with k >= 1 run the QMC loop
    samples_per_step = n_qmc_terms * inst.qmc.n_points * inst.qmc.n_shifts

    def step(q):
        V.vecchia_replan(plan, inst.locs, inst.ordering, stream=sp)
        V.vecchia_logcdf(plan, x, q, out, stream=sp)

    # ---- full path, FP32 loop: warmup, then the timed region with kernel events
    for _ in range(args.warmup):
        step(q32)
    torch.cuda.synchronize()
    V.vecchia_profile_reset()
    V.vecchia_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(q32)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    V.vecchia_profile_enable(0)
    k_ms, k_launches, k_steps = V.vecchia_profile_read(m, V.VECCHIA_FP32_LOOP)
    V.vecchia_profile_reset()
    ms_per_step = 1e3 * t_full / args.steps
    lf32 = out.cpu().numpy().copy()
    if args.fp32_only:
        V.vecchia_plan_destroy(plan)
        print(json.dumps({"workload": inst.name, "ms_per_step": ms_per_step,
                          "qmc_kernel_avg_ms": k_ms / max(k_launches, 1), "logF": float(lf32[0])}),
              flush=True)
        return

    # ---- log-CDF only (resident plan, HIP graph replay)
    for _ in range(2):
        V.vecchia_logcdf(plan, x, q32, out, stream=sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        V.vecchia_logcdf(plan, x, q32, out, stream=sp)
    torch.cuda.synchronize()
    ms_logcdf = 1e3 * (time.perf_counter() - t0) / args.steps

    # ---- plain FP64 on the same inputs
    terms32 = torch.empty((D, 2), dtype=torch.float64, device="cuda")
    terms64 = torch.empty((D, 2), dtype=torch.float64, device="cuda")
    V.vecchia_logcdf(plan, x, q32, out, terms=terms32, stream=sp)
    V.vecchia_logcdf(plan, x, q64, out, terms=terms64, stream=sp)
    torch.cuda.synchronize()
    lf64 = out.cpu().numpy().copy()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        V.vecchia_logcdf(plan, x, q64, out, stream=sp)
    torch.cuda.synchronize()
    ms_fp64 = 1e3 * (time.perf_counter() - t0) / args.fp64_steps
    t32, t64 = terms32.cpu().numpy(), terms64.cpu().numpy()

    # ---- the paper-literal estimator (separate points for each term's numerator
    # and denominator) against the shared lattice, same N x R: time and SE
    qind = V.make_qmc(inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, V.VECCHIA_FP32_LOOP, independent=True)
    V.vecchia_logcdf(plan, x, qind, out, stream=sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_ind = max(1, args.steps // 2)
    for _ in range(n_ind):
        V.vecchia_logcdf(plan, x, qind, out, stream=sp)
    torch.cuda.synchronize()
    ms_ind = 1e3 * (time.perf_counter() - t0) / n_ind
    lind = out.cpu().numpy().copy()
    V.vecchia_plan_destroy(plan)

    # measured issue rates (wave64 instructions per CU per ns) and the ceiling
    # they give this kernel's instruction mix
    rates = V.vecchia_calibrate_valu(stream=sp)
    n_trans = sum(TRANS_PER_STEP.values())
    ns_per_wave_step = ((SLOTS_PER_STEP_F32_K10 - n_trans) / rates["fma"] +
                        sum(c / rates[k] for k, c in TRANS_PER_STEP.items()))
    ceiling = SLOTS_PER_STEP_F32_K10 * 64 * 256 / ns_per_wave_step / 1e3   # T lane-slots/s
    kernel_avg_ms = k_ms / max(k_launches, 1)
    steps_per_launch = k_steps / max(k_launches, 1)
    achieved = steps_per_launch * SLOTS_PER_STEP_F32_K10 / (kernel_avg_ms * 1e-3) / 1e12
    res = {
        "metric": "Vecchia terms/s (m=10; plan + log-CDF per step)",
        "value": D / (ms_per_step * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": inst.name, "D": D, "m": m, "n_points": inst.qmc.n_points,
                   "n_shifts": inst.qmc.n_shifts, "ordering": "maxmin",
                   "covariance": "matern nu=1.5 range=0.1 nugget=1e-8",
                   "loop_precision": "fp32 (fp64 cholesky/accumulate)"},
        "samples_per_s": samples_per_step / (ms_per_step * 1e-3),
        "logcdf_only": {"ms": ms_logcdf, "terms_per_s": D / (ms_logcdf * 1e-3),
                        "samples_per_s": samples_per_step / (ms_logcdf * 1e-3)},
        "fp64_plain": {"ms": ms_fp64, "terms_per_s": D / (ms_fp64 * 1e-3),
                       "fp32_speedup": ms_fp64 / ms_logcdf},
        "independent_points": {"ms": ms_ind, "logF": float(lind[0]), "se": float(lind[1]),
                               "shared_logF": float(lf32[0]), "shared_se": float(lf32[1]),
                               "se_ratio": float(lind[1] / lf32[1]), "time_ratio": ms_ind / ms_logcdf},
        "accuracy_fp32_vs_fp64": {"logF_fp32": float(lf32[0]), "logF_fp64": float(lf64[0]),
                                  "se_fp64": float(lf64[1]),
                                  "rel_total": abs(lf32[0] - lf64[0]) / abs(lf64[0]),
                                  "max_abs_term": float(np.max(np.abs(t32[:, 0] - t64[:, 0])))},
        "roofline": {"bound": "alu", "kernel": f"qmc_f32<{m}>",
                     "achieved": achieved, "peak": VALU_PEAK_TSLOTS, "unit": "T VALU-slots/s",
                     "frac": achieved / VALU_PEAK_TSLOTS, "traffic": TRAFFIC_BYTES_F32_K10,
                     "avg_launch_ms": kernel_avg_ms, "sov_steps_per_launch": steps_per_launch,
                     "slots_per_step": SLOTS_PER_STEP_F32_K10,
                     "measured_rates_wave_instr_per_cu_ns": {k: round(v, 4) for k, v in rates.items()},
                     "measured_ceiling": ceiling, "frac_of_measured_ceiling": achieved / ceiling},
    }
    if tuned is not None:
        res["autotune"] = tuned
    sections = set(args.sections.split(","))
    if "c1" in sections:
        res["c1_grid"] = bench_c1(V, torch, args)
    if "c3" in sections:
        res["c3_batched"] = bench_c3(V, torch, args)
    if "c4" in sections:
        res["c4_large"] = bench_c4(V, torch, args)
    if "c5" in sections:
        res["c5_serving"] = bench_c5(V, torch, args)
    if "mix" in sections:
        res["scale_mixture"] = bench_mixture(V, torch, args)
    if "cens" in sections:
        res["censored_likelihood"] = bench_censored(V, torch, args)
    if "full" in sections:
        res["full_dimension_comparator"] = bench_comparator(V, torch, args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inst, args.cpu_terms)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
