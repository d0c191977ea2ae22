"""Benchmark of the Vecchia log-CDF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workload (default): D = 2,500 locations uniform in [0,1]^2, Matern nu = 3/2
(range 0.1, nugget 1e-8), maxmin ordering, m = 10, thresholds at the 0.9
marginal quantile plus N(0, 0.1^2) noise, 10^4 lattice points x 10 shifts, FP32
SOV loop with FP64 Cholesky / accumulation. Inputs are seeded synthetic data
(workloads/); thresholds are resident on the device before timing.

One step = the whole path for one instance: vecchia_replan (host maxmin
ordering + the GPU nearest-preceding-neighbour kernel) followed by
vecchia_logcdf (covariance + Cholesky, the QMC kernels, the segmented log-sum).
K steps are timed between two device synchronisations; value = terms per second
(D terms per step). The line also carries samples/s, the log-CDF-only rate,
the plain FP64 rate on the same inputs, the FP32-vs-FP64 error, the roofline of
the dominant kernel (its HIP-event time over the timed region) and the CPU
oracle baseline on a bounded sample.
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
# HBM bytes per launch of qmc_f32<10> from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (factors from a 256 MiB copy); None once the kernel changes.
TRAFFIC_BYTES_F32_K10 = 12.20e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform2500_matern15_m10",
                    choices=["uniform2500_matern15_m10", "grid400_exp_m5"])
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-terms", type=int, default=500)
    ap.add_argument("--fp32-only", action="store_true",
                    help="time the full FP32 step only (short runs under a profiler)")
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
    return {"value": inst.D / t_full, "unit": "terms/s", "cores": procs, "kind": "oracle",
            "sample": f"plan of all {inst.D} locations ({t_plan:.2f} s) + {len(sub)} of {inst.D} "
                      f"terms ({t_terms:.2f} s on {procs} processes), extrapolated to all terms"}


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
    V.vecchia_plan_destroy(plan)

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
        "accuracy_fp32_vs_fp64": {"logF_fp32": float(lf32[0]), "logF_fp64": float(lf64[0]),
                                  "se_fp64": float(lf64[1]),
                                  "rel_total": abs(lf32[0] - lf64[0]) / abs(lf64[0]),
                                  "max_abs_term": float(np.max(np.abs(t32[:, 0] - t64[:, 0])))},
        "roofline": {"bound": "alu", "kernel": f"qmc_f32<{m}>",
                     "achieved": achieved, "peak": VALU_PEAK_TSLOTS, "unit": "T VALU-slots/s",
                     "frac": achieved / VALU_PEAK_TSLOTS, "traffic": TRAFFIC_BYTES_F32_K10,
                     "avg_launch_ms": kernel_avg_ms, "sov_steps_per_launch": steps_per_launch,
                     "slots_per_step": SLOTS_PER_STEP_F32_K10},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inst, args.cpu_terms)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
