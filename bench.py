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
              loop after 50 warm-up requests: capacity with 1000 requests
              queued at once, then the same requests as Poisson arrivals at
              50, 80 and 95 % of it with p50/p99 latency (16 GB budget);
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
# unrolled chain in its assembly (rare branches not taken); cross-checked on
# every run against SQ_INSTS_VALU x 64 / steps of the committed counter profile
# (within 2 %, the difference being each work item's set-up).
SLOTS_PER_STEP_F32_K10 = 48.2
# MI355X FP32 vector peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 FMA lanes x 2:
# 78.64e12 full-rate VALU lane-slots per second. FP64 vector peak 78.6 TFLOP/s.
VALU_PEAK_TSLOTS = 256 * 2.4e9 * 128 / 1e12
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# Transcendental instructions per SOV step on that path (the rest are full-rate):
# Phi^-1 takes a log2, a sqrt and a reciprocal, Phi a reciprocal and an exp2.
TRANS_PER_STEP = {"exp": 1, "log": 1, "rcp": 2, "sqrt": 1}
# rocprofv3 counter summaries of the QMC kernels at the headline workload; each
# holds a `counters_json:` line with per-dispatch counters and the hash of the
# kernel sources it was taken on (a changed kernel makes its figures stale).
PMC_F32 = os.path.join(ROOT, "profiles", "qmc_f32_k10_uniform2500_pmc.md")
PMC_F64 = os.path.join(ROOT, "profiles", "qmc_f64_k10_uniform2500_pmc.md")
KERNEL_SOURCES = ["kernels_qmc.hip", "device_math_f32.h", "lattice.h", "fp32_math_coeffs.h", "vecchia_internal.h",
                  "device_math_f64.h", "fp64_math_coeffs.h"]


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2007_15195_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(path):
    """The `counters_json:` line of a committed counter summary, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("counters_json:"):
                return json.loads(line[len("counters_json:"):])
    return None


def counter_figures(c, sha, avg_launch_s, steps_per_launch, peak_tflops, prec):
    """Per-step instruction and FLOP figures of a counter profile, and the FLOP
    rate they give at the live launch time: FMA = 2 flops, ADD / MUL and a
    transcendental 1 flop each, per lane (x 64)."""
    if c is None:
        return {"status": "missing"}
    k = c["counters"]
    st = float(c["sov_steps_per_dispatch"])
    sfx = "F32" if prec == 32 else "F64"
    flops = 64.0 * (2.0 * k[f"SQ_INSTS_VALU_FMA_{sfx}"] + k[f"SQ_INSTS_VALU_ADD_{sfx}"] +
                    k[f"SQ_INSTS_VALU_MUL_{sfx}"] + k[f"SQ_INSTS_VALU_TRANS_{sfx}"])
    fps = flops / st
    achieved = fps * steps_per_launch / avg_launch_s / 1e12
    out = {"status": "current" if c.get("source_sha") == sha else "stale (kernel changed since)",
           "source_sha": c.get("source_sha"), "valu_slots_per_step": 64.0 * k["SQ_INSTS_VALU"] / st,
           "flops_per_step": fps, "achieved_tflops": achieved, "peak_tflops": peak_tflops,
           "frac": achieved / peak_tflops}
    if "FETCH_SIZE" in k and "WRITE_SIZE" in k:
        out["traffic_bytes"] = 1024.0 * (k["FETCH_SIZE"] * c["fetch_factor"] + k["WRITE_SIZE"] * c["write_factor"])
    return out


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
    ap.add_argument("--fp64-only", action="store_true",
                    help="time the plain FP64 log-CDF only (short runs under a profiler)")
    ap.add_argument("--censored-T", type=int, default=1006)
    ap.add_argument("--comparator-grids", type=lambda v: [int(t) for t in v.split(",")], default=[15, 30, 50, 75, 100])
    ap.add_argument("--sections", default="c1,c2,c3,c4,c5,mix,cens,full",
                    help="comma list of workloads to run besides the headline (c2 is always run)")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--sections-only", action="store_true",
                    help="run only the listed sections and print their objects (for profiling runs)")
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
            "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "sample": f"plan of all {inst.D} locations ({t_plan:.2f} s) + {len(sub)} of {inst.D} "
                      f"terms ({t_terms:.2f} s on {procs} processes), extrapolated to all terms",
            "single_core": {"value": inst.D / (t_plan + t_one * inst.D / len(sub1)), "unit": "terms/s",
                            "sample": f"the same plan + {len(sub1)} terms ({t_one:.2f} s) in one process"}}


def cpu_baseline_subset(V, insts, plans, total_terms, n_inst, n_terms, seed):
    """The oracle on a seeded subset of a large workload: n_inst instances (every
    instance when there are fewer), each with its k < m terms and n_terms seeded
    others, on the plan's own ordering and neighbour lists (read back from the GPU
    plan, whose sets the tests hold equal to the oracle's: the oracle's exact
    O(D^2) maxmin alone would take minutes at these sizes). Terms/s on the sample,
    extrapolated to all terms of the workload by its mean cost per term."""
    import oracle
    rng = np.random.default_rng(abs(hash(seed)) % (2 ** 32))
    pick = sorted(rng.choice(len(insts), size=min(n_inst, len(insts)), replace=False).tolist())
    procs = oracle.vecchia.default_processes()
    t_terms, n_done, steps_done = 0.0, 0, 0.0
    for j in pick:
        inst, plan = insts[j], plans[j]
        perm, nbr = V.vecchia_plan_neighbours(plan)
        nbrs = [np.array([v for v in row if v >= 0], dtype=np.int64) for row in nbr]
        head = list(range(min(inst.m + 1, inst.D)))
        rest = rng.choice(np.arange(len(head), inst.D), size=min(n_terms, inst.D - len(head)), replace=False)
        sub = sorted(set(head) | set(int(v) for v in rest))
        c = inst.cov
        t0 = time.perf_counter()
        oracle.logcdf(inst.locs, inst.x, inst.m, c.family, c.nu, c.sigma2, c.range, c.nugget, inst.ordering,
                      inst.qmc.n_points, inst.qmc.n_shifts, inst.qmc.seed, terms_subset=sub,
                      plan_cache=(perm.astype(np.int64), nbrs), processes=procs)
        t_terms += time.perf_counter() - t0
        n_done += len(sub)
        steps_done += inst.qmc.n_points * inst.qmc.n_shifts * sum(min(i, inst.m) for i in sub)
    all_steps = sum(i.qmc.n_points * i.qmc.n_shifts * (i.m * (i.D - i.m) + i.m * (i.m - 1) // 2) for i in insts)
    steps_per_s = steps_done / t_terms
    return {"value": total_terms / (all_steps / steps_per_s), "unit": "terms/s (extrapolated)", "cores": procs,
            "kind": "oracle", "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "sov_steps_per_s": steps_per_s,
            "sample": f"{n_done} terms of {len(pick)} instance(s) ({t_terms:.1f} s on {procs} processes; "
                      f"plans read back from the GPU), extrapolated by SOV steps to all {total_terms} terms"}


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
            # the product-and-recursion kernel alone (HIP events on its stream)
            V.vecchia_profile_reset()
            V.vecchia_profile_enable(1)
            V.vecchia_full_logcdf(plan, x, q64, out, stream=sp)
            torch.cuda.synchronize()
            V.vecchia_profile_enable(0)
            k_ms, _, k_fma = V.vecchia_profile_read(V.VECCHIA_PROFILE_FULL_SOV, V.VECCHIA_FP64)
            V.vecchia_profile_reset()
            row["full_sov_fp64"] = {"seconds": sec, "logF": float(o[0]), "se": float(o[1]),
                                    "points_per_s": N * R / sec, "kernel_ms": k_ms,
                                    "kernel_tflops": 2.0 * k_fma / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None}
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
    # compact rows: seconds and log F of the full-dimension estimate and of the
    # Vecchia log-CDF at each m (FP32 / FP64)
    table = []
    for row in rows:
        t = {"grid": row["grid"], "range": row["range"],
             "full": [round(row["full_sov_fp64"]["seconds"], 4), round(row["full_sov_fp64"]["logF"], 3),
                      round(row["full_sov_fp64"]["se"], 3)]}
        for mm in (5, 10, 30, 50):
            a, b = row[f"vecchia_m{mm}_fp32"], row[f"vecchia_m{mm}_fp64"]
            t[f"m{mm}"] = [round(a["seconds"], 4), round(b["seconds"], 4), round(a["logF"], 3)]
        table.append(t)
    big = [r for r in rows if r["D"] == 10_000]
    summary = {}
    if big:
        tf = [r["full_sov_fp64"]["kernel_tflops"] for r in big if r["full_sov_fp64"]["kernel_tflops"]]
        summary = {"full_sov_seconds_100x100": [r["full_sov_fp64"]["seconds"] for r in big],
                   "vecchia_m30_fp32_seconds_100x100": [r["vecchia_m30_fp32"]["seconds"] for r in big],
                   "full_sov_kernel_ms_100x100": [round(r["full_sov_fp64"]["kernel_ms"], 2) for r in big],
                   "full_sov_kernel_fp64_frac_100x100": [round(t / FP64_PEAK_TFLOPS, 4) for t in tf]}
    return {"workload": "exp_grids_unit_spacing_comparator", "n_points": N, "n_shifts": R,
            "columns": "full: [s, logF, se]; mK: [fp32 s, fp64 s, fp32 logF]", "rows": table, **summary}


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
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_subset(V, insts, plans, terms, 12, 150, "c3")
    if tuned is not None:
        res["autotune_chunk_points"] = {"fp32": tuned["chunk_points_fp32"], "fp64": tuned["chunk_points_fp64"]}
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
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_subset(V, [inst], [plan], D, 1, 1200, "c4")
    d = np.abs(got["fp32"][1] - got["fp64"][1])
    nz = got["fp64"][1] != 0.0          # log-terms that round to 0 in FP64 have no relative error
    res["fp32_vs_fp64"] = {"rel_total": abs(got["fp32"][0][0] - got["fp64"][0][0]) / abs(got["fp64"][0][0]),
                           "max_abs_term": float(d.max()),
                           "max_rel_term": float(np.max(d[nz] / np.abs(got["fp64"][1][nz]))),
                           "terms_rounding_to_zero": int(np.sum(~nz))}
    if tuned is not None:
        res["autotune_chunk_points"] = {"fp32": tuned["chunk_points_fp32"], "fp64": tuned["chunk_points_fp64"]}
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
    """Serving loop: 50 warm-up requests, then capacity with 1000 requests queued
    at once, then the same 1000 requests as Poisson arrivals at 50, 80 and 95 %
    of that capacity (p50 / p99 latency per load); 16 GB HBM budget, 16 slots."""
    import workloads as W
    n_warm, n_req = 50, args.serving_requests
    st = W.serving_stream(n_requests=n_warm + n_req)
    t0 = time.perf_counter()
    plans = [V.vecchia_plan(p.locs, p.ordering, p.m, p.cov) for p in st.plans]
    t_plans = time.perf_counter() - t0
    xs = [torch.tensor(r.x, dtype=torch.float64, device="cuda") for r in st.requests]
    torch.cuda.synchronize()
    warm, reqs, xr = st.requests[:n_warm], st.requests[n_warm:], xs[n_warm:]
    terms = sum(st.plans[r.plan_id].D for r in reqs)
    samples = sum(st.plans[r.plan_id].D * r.qmc.n_points * r.qmc.n_shifts for r in reqs)
    sov = sum(r.qmc.n_points * r.qmc.n_shifts * (st.plans[r.plan_id].m * (st.plans[r.plan_id].D - st.plans[r.plan_id].m)
                                                  + st.plans[r.plan_id].m * (st.plans[r.plan_id].m - 1) // 2)
              for r in reqs)
    budget, slots = 16 << 30, 16
    srv = V.vecchia_server_create(budget, slots)
    _serve(V, srv, plans, warm, xs[:n_warm], np.zeros(n_warm))
    wall, _ = _serve(V, srv, plans, reqs, xr, np.zeros(len(reqs)))
    rate = len(reqs) / wall
    res = {"workload": "serving_stream", "plans": len(plans), "warmup_requests": n_warm, "requests": len(reqs),
           "plan_seconds_all": t_plans, "hbm_budget_bytes": budget, "slots": slots,
           "mean_m": float(np.mean([st.plans[r.plan_id].m for r in reqs])),
           "capacity": {"requests_per_s": rate, "terms_per_s": terms / wall, "samples_per_s": samples / wall,
                        "sov_steps_per_s": sov / wall}}
    arr = np.array([r.arrival_s for r in reqs])
    arr = arr - arr[0]
    for load in (0.5, 0.8, 0.95):
        a = arr / arr[-1] * (len(reqs) / (load * rate))      # the same Poisson pattern at this load
        w, lat = _serve(V, srv, plans, reqs, xr, a)
        res[f"poisson_{int(round(100 * load))}pct"] = {
            "offered_requests_per_s": load * rate, "requests_per_s": len(reqs) / w, "terms_per_s": terms / w,
            "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)), "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
            "latency_ms_max": 1e3 * float(lat.max())}
    V.vecchia_server_destroy(srv)
    for p in plans:
        V.vecchia_plan_destroy(p)
    return res


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
    if args.sections_only:
        fns = {"c1": ("c1_grid", bench_c1), "c3": ("c3_batched", bench_c3), "c4": ("c4_large", bench_c4),
               "c5": ("c5_serving", bench_c5), "mix": ("scale_mixture", bench_mixture),
               "cens": ("censored_likelihood", bench_censored), "full": ("full_dimension_comparator", bench_comparator)}
        res = {}
        for sec in args.sections.split(","):
            if sec in fns:
                key, fn = fns[sec]
                res[key] = fn(V, torch, args)
                print(json.dumps({key: res[key]}), flush=True)
        return
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

    if args.fp64_only:
        for _ in range(max(1, args.warmup)):
            V.vecchia_logcdf(plan, x, q64, out, stream=sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            V.vecchia_logcdf(plan, x, q64, out, stream=sp)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        V.vecchia_plan_destroy(plan)
        print(json.dumps({"workload": inst.name, "fp64_ms_per_logcdf": ms, "logF": float(out.cpu().numpy()[0])}),
              flush=True)
        return

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
    # the plain FP64 kernel's own launch time (HIP events on its stream)
    V.vecchia_profile_reset()
    V.vecchia_profile_enable(1)
    for _ in range(args.fp64_steps):
        V.vecchia_logcdf(plan, x, q64, out, stream=sp)
    torch.cuda.synchronize()
    V.vecchia_profile_enable(0)
    k64_ms, k64_launches, k64_steps = V.vecchia_profile_read(m, V.VECCHIA_FP64)
    V.vecchia_profile_reset()
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
    sha = kernel_source_sha()
    c32 = counter_figures(load_counters(PMC_F32), sha, kernel_avg_ms * 1e-3, steps_per_launch, FP32_PEAK_TFLOPS, 32)
    k64_avg_ms = k64_ms / max(k64_launches, 1)
    c64 = counter_figures(load_counters(PMC_F64), sha, k64_avg_ms * 1e-3, k64_steps / max(k64_launches, 1),
                          FP64_PEAK_TFLOPS, 64)
    if c32.get("status") == "current":
        # the assembly count of the chain's main path against the executed instructions
        c32["slots_check"] = ("ok" if abs(c32["valu_slots_per_step"] / SLOTS_PER_STEP_F32_K10 - 1.0) <= 0.02
                              else "differs by more than 2 %")
    traffic = c32.get("traffic_bytes") if c32.get("status") == "current" else None
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
                     "frac": achieved / VALU_PEAK_TSLOTS, "traffic": traffic,
                     "avg_launch_ms": kernel_avg_ms, "sov_steps_per_launch": steps_per_launch,
                     "slots_per_step": SLOTS_PER_STEP_F32_K10,
                     "measured_rates_wave_instr_per_cu_ns": {k: round(v, 4) for k, v in rates.items()},
                     "measured_ceiling": ceiling, "frac_of_measured_ceiling": achieved / ceiling,
                     "fp32_flops": c32,
                     "fp64_plain_kernel": {"kernel": f"qmc_f64<{m}>", "avg_launch_ms": k64_avg_ms,
                                           "sov_steps_per_launch": k64_steps / max(k64_launches, 1),
                                           "fp64_flops": c64}},
    }
    if tuned is not None:
        res["autotune_chunk_points"] = [tuned["chunk_points_fp32"], tuned["chunk_points_fp64"]]
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
    res["summary"] = summary(res)
    print(json.dumps(res), flush=True)


def _r(v, k=4):
    return float(f"{v:.{k}g}") if isinstance(v, (int, float)) and v is not None and math.isfinite(v) else v


def summary(res):
    """The secondary figures in a few hundred bytes, last on the line."""
    out = {"fp64_plain_speedup": _r(res["fp64_plain"]["fp32_speedup"]),
           "fp32_vs_fp64_rel_total": _r(res["accuracy_fp32_vs_fp64"]["rel_total"], 2),
           "fp32_vs_fp64_max_term": _r(res["accuracy_fp32_vs_fp64"]["max_abs_term"], 2),
           "logcdf_only_terms_per_s": _r(res["logcdf_only"]["terms_per_s"])}
    if "c1_grid" in res:
        c = res["c1_grid"]
        out["c1"] = {"fp64_terms_per_s": _r(c["fp64"]["terms_per_s"]), "fp32_terms_per_s": _r(c["fp32"]["terms_per_s"])}
    if "c3_batched" in res:
        c = res["c3_batched"]
        out["c3"] = {"terms_per_s": _r(c["fp32"]["terms_per_s"]), "samples_per_s": _r(c["fp32"]["samples_per_s"]),
                     "sov_steps_per_s": _r(c["fp32"]["sov_steps_per_s"]), "fp32_speedup": _r(c["fp32_speedup"]),
                     "max_rel_vs_fp64": _r(c["fp32_vs_fp64_rel_total"]["max"], 2)}
        if "cpu_baseline" in c:
            out["c3"]["cpu_terms_per_s_extrapolated"] = _r(c["cpu_baseline"]["value"])
    if "c4_large" in res:
        c = res["c4_large"]
        out["c4"] = {"terms_per_s": _r(c["fp32"]["terms_per_s"]), "samples_per_s": _r(c["fp32"]["samples_per_s"]),
                     "fp32_speedup": _r(c["fp32_speedup"]), "rel_total_vs_fp64": _r(c["fp32_vs_fp64"]["rel_total"], 2)}
        if "cpu_baseline" in c:
            out["c4"]["cpu_terms_per_s_extrapolated"] = _r(c["cpu_baseline"]["value"])
    if "c5_serving" in res:
        c = res["c5_serving"]
        loads = [k for k in c if k.startswith("poisson_")]
        out["c5"] = {"capacity_terms_per_s": _r(c["capacity"]["terms_per_s"]),
                     "capacity_samples_per_s": _r(c["capacity"]["samples_per_s"]),
                     "capacity_sov_steps_per_s": _r(c["capacity"]["sov_steps_per_s"]),
                     "loads": [k[len("poisson_"):] for k in loads],
                     "p50_ms": [_r(c[k]["latency_ms_p50"], 3) for k in loads],
                     "p99_ms": [_r(c[k]["latency_ms_p99"], 3) for k in loads]}
    if "scale_mixture" in res:
        c = res["scale_mixture"]
        out["mixture"] = {"fp32_ms_per_call": _r(c["fp32"]["ms_per_call"]), "fp32_speedup": _r(c["fp32_speedup"])}
    if "censored_likelihood" in res:
        c = res["censored_likelihood"]
        out["censored"] = {"fp32_s_per_likelihood": _r(c["fp32"]["seconds_per_likelihood"]),
                           "fp32_speedup_subset": _r(c["fp32_speedup_on_subset"])}
    if "full_dimension_comparator" in res:
        c = res["full_dimension_comparator"]
        out["comparator_100x100"] = {k: [_r(v) for v in c[k]] for k in c if k.endswith("100x100")}
    return out


if __name__ == "__main__":
    main()
