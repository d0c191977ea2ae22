"""Seeded synthetic inputs for the Vecchia log-CDF path.

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It only draws inputs (locations, thresholds, covariance parameters,
QMC sizes and seeds); it holds none of the method's arithmetic.

The shapes follow the paper's spatial workloads: Gaussian processes observed at
2-D locations (regular grids in the simulation study, Section 3; irregular
station networks in the application, Section 4.1), unit marginal variance, and
thresholds at high marginal quantiles (the censoring threshold of Section 4.1 is
the 0.95 quantile). The paper's precipitation data are not used; every input is
drawn from numpy's PCG64 generator with the seeds below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Standard-normal quantiles used to place thresholds (published constants).
Z_090 = 1.2815515655446004   # 0.90 quantile of N(0, 1)
Z_095 = 1.6448536269514722   # 0.95 quantile of N(0, 1)

ORDER_GIVEN, ORDER_COORD, ORDER_MAXMIN = 0, 1, 2
COV_EXPONENTIAL, COV_MATERN = 0, 1
PREC_FP64, PREC_FP32 = 0, 1


def seed_for(config: int, stream: int) -> int:
    """Seed of stream 0 (geometry), 1 (thresholds) or 2 (QMC) of a config."""
    return 20200730 + 10 * config + stream


@dataclass
class Cov:
    family: int = COV_MATERN
    nu: float = 0.5
    sigma2: float = 1.0
    range: float = 0.1
    nugget: float = 0.0


@dataclass
class QMC:
    n_points: int = 1000
    n_shifts: int = 10
    seed: int = 1
    precision: int = PREC_FP64


@dataclass
class Instance:
    """One Gaussian log-CDF evaluation: log P(X < x / scale)."""
    name: str
    locs: np.ndarray              # D x 2 float64
    x: np.ndarray                 # D float64, user index order
    m: int
    ordering: int
    cov: Cov
    qmc: QMC
    scale: float = 1.0
    perm: Optional[np.ndarray] = None   # only for ORDER_GIVEN

    @property
    def D(self) -> int:
        return int(self.locs.shape[0])


def grid_locations(nx: int, ny: int) -> np.ndarray:
    """Regular nx x ny grid in [0,1]^2 with the end points included.

    Point index a*ny + b sits at (a/(nx-1), b/(ny-1)).
    """
    a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    xs = a.reshape(-1) / max(nx - 1, 1)
    ys = b.reshape(-1) / max(ny - 1, 1)
    return np.stack([xs, ys], axis=1).astype(np.float64)


def uniform_locations(D: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((D, 2), dtype=np.float64)


# ---------------------------------------------------------------------------
# Workloads named by what they are.
# ---------------------------------------------------------------------------

def grid400_exponential(n_points: int = 1000, n_shifts: int = 10,
                        precision: int = PREC_FP64) -> Instance:
    """D=400 on a 20x20 grid, exponential(range 0.2), coordinate order, m=5,
    thresholds N(1, 0.25^2), 1000 lattice points x 10 shifts."""
    locs = grid_locations(20, 20)
    rng = np.random.Generator(np.random.PCG64(seed_for(1, 1)))
    x = rng.normal(1.0, 0.25, size=400)
    return Instance("grid400_exp_m5", locs, x, 5, ORDER_COORD,
                    Cov(COV_EXPONENTIAL, 0.5, 1.0, 0.2, 0.0),
                    QMC(n_points, n_shifts, seed_for(1, 2), precision))


def uniform2500_matern15(n_points: int = 10_000, n_shifts: int = 10,
                         precision: int = PREC_FP32, nugget: float = 1e-8) -> Instance:
    """D=2,500 uniform in [0,1]^2, Matern nu=1.5 (range 0.1), maxmin order,
    m=10, thresholds at the 0.9 marginal quantile plus N(0, 0.1^2)."""
    rng = np.random.Generator(np.random.PCG64(seed_for(2, 0)))
    locs = uniform_locations(2500, rng)
    rng_x = np.random.Generator(np.random.PCG64(seed_for(2, 1)))
    x = Z_090 + rng_x.normal(0.0, 0.1, size=2500)
    return Instance("uniform2500_matern15_m10", locs, x, 10, ORDER_MAXMIN,
                    Cov(COV_MATERN, 1.5, 1.0, 0.1, nugget),
                    QMC(n_points, n_shifts, seed_for(2, 2), precision))


def batched_uneven(n_instances: int = 512, d_min: int = 100, d_max: int = 20_000,
                   n_points: int = 4096, n_shifts: int = 8,
                   precision: int = PREC_FP32, nugget: float = 1e-8) -> List[Instance]:
    """Instances with D log-uniform in [d_min, d_max], m in {5,10,15,20},
    Matern nu in {0.5,1.5,2.5}, range U(0.05,0.3), uniform points, maxmin
    order, thresholds N(1.5, 0.5^2)."""
    rng = np.random.Generator(np.random.PCG64(seed_for(3, 0)))
    out = []
    for j in range(n_instances):
        D = int(round(np.exp(rng.uniform(np.log(d_min), np.log(d_max)))))
        m = int(rng.choice([5, 10, 15, 20]))
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        rho = float(rng.uniform(0.05, 0.3))
        locs = uniform_locations(D, rng)
        x = rng.normal(1.5, 0.5, size=D)
        out.append(Instance(f"batch{j}", locs, x, m, ORDER_MAXMIN,
                            Cov(COV_MATERN, nu, 1.0, rho, nugget),
                            QMC(n_points, n_shifts, seed_for(3, 2) + j, precision)))
    return out


def uniform250k_tail(D: int = 250_000, n_points: int = 10_000, n_shifts: int = 10,
                     precision: int = PREC_FP32, nugget: float = 1e-8) -> Instance:
    """D=250,000 uniform, Matern nu=1.5 (range 0.05), maxmin, m=20, every
    threshold at the 0.95 marginal quantile (joint-tail regime)."""
    rng = np.random.Generator(np.random.PCG64(seed_for(4, 0)))
    locs = uniform_locations(D, rng)
    x = np.full(D, Z_095)
    return Instance("uniform250k_matern15_m20_tail", locs, x, 20, ORDER_MAXMIN,
                    Cov(COV_MATERN, 1.5, 1.0, 0.05, nugget),
                    QMC(n_points, n_shifts, seed_for(4, 2), precision))


@dataclass
class Request:
    plan_id: int
    arrival_s: float
    x: np.ndarray
    scale: float
    cov: Cov
    qmc: QMC


@dataclass
class ServingStream:
    plans: List[Instance] = field(default_factory=list)
    requests: List[Request] = field(default_factory=list)


def serving_stream(n_plans: int = 16, n_requests: int = 1000, rate_per_s: float = 50.0,
                   d_min: int = 1000, d_max: int = 100_000, precision: int = PREC_FP32,
                   nugget: float = 1e-8) -> ServingStream:
    """Resident geometries with D log-uniform in [d_min, d_max], m uniform in
    5..30; Poisson arrivals; per-request Matern range U(0.02, 0.3) and a
    scale-mixture factor R ~ Pareto(alpha=2, scale 1) dividing the thresholds;
    2048, 4096 or 8192 lattice points x 8 shifts."""
    rng = np.random.Generator(np.random.PCG64(seed_for(5, 0)))
    st = ServingStream()
    for j in range(n_plans):
        D = int(round(np.exp(rng.uniform(np.log(d_min), np.log(d_max)))))
        m = int(rng.integers(5, 31))
        locs = uniform_locations(D, rng)
        st.plans.append(Instance(f"plan{j}", locs, np.zeros(D), m, ORDER_MAXMIN,
                                 Cov(COV_MATERN, 1.5, 1.0, 0.1, nugget),
                                 QMC(4096, 8, 0, precision)))
    rq = np.random.Generator(np.random.PCG64(seed_for(5, 1)))
    t = 0.0
    for r in range(n_requests):
        t += rq.exponential(1.0 / rate_per_s)
        pid = int(rq.integers(0, n_plans))
        D = st.plans[pid].D
        x = rq.normal(1.5, 0.5, size=D)
        scale = float(rq.random() ** -0.5)          # Pareto(alpha=2) by inversion
        rho = float(rq.uniform(0.02, 0.3))
        n_pts = int(rq.choice([2048, 4096, 8192]))
        st.requests.append(Request(pid, t, x, scale,
                                   Cov(COV_MATERN, 1.5, 1.0, rho, nugget),
                                   QMC(n_pts, 8, seed_for(5, 2) + r, precision)))
    return st


def small_random_instance(D: int, m: int, seed: int, ordering: int = ORDER_MAXMIN,
                          nu: float = 1.5, rho: float = 0.15, n_points: int = 512,
                          n_shifts: int = 4, mean_x: float = 1.0, sd_x: float = 0.5,
                          precision: int = PREC_FP64, nugget: float = 1e-8,
                          family: int = COV_MATERN, scale: float = 1.0) -> Instance:
    """A small seeded instance for parity tests (uniform points)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    locs = uniform_locations(D, rng)
    x = rng.normal(mean_x, sd_x, size=D)
    return Instance(f"small_D{D}_m{m}_s{seed}", locs, x, m, ordering,
                    Cov(family, nu, 1.0, rho, nugget),
                    QMC(n_points, n_shifts, seed + 7, precision), scale=scale)


# ---------------------------------------------------------------------------
# Censored replicates (Section 4: the censored likelihood of eq. (11)).
# ---------------------------------------------------------------------------

@dataclass
class CensoredReplicate:
    """One replicate: sites, thresholds and which values are observed.

    x[u] is the censoring threshold at a censored site and the observed value
    (above the threshold) at an observed site."""
    inst: Instance
    observed: np.ndarray          # D bools, user order


def smooth_field(locs: np.ndarray, rng: np.random.Generator, nu: float, rho: float,
                 n_features: int = 4000) -> np.ndarray:
    """A stationary, approximately Gaussian random field with unit variance
    and a Matern-like correlation scale rho, by random Fourier features:
    X(s) = sqrt(2 / J) sum_j cos(w_j . s + b_j), w_j = t_j / rho with t_j
    bivariate Student-t (2 nu degrees of freedom), b_j uniform on [0, 2 pi).
    Used only to draw plausible replicates (spatially coherent exceedances)."""
    g = rng.standard_normal((n_features, 2))
    chi = rng.chisquare(2.0 * nu, n_features)
    w = g / np.sqrt(chi / (2.0 * nu))[:, None] / rho
    b = rng.uniform(0.0, 2.0 * np.pi, n_features)
    return np.sqrt(2.0 / n_features) * np.cos(locs @ w.T + b).sum(axis=1)


def censored_replicate(D: int, m: int, seed: int, frac_obs: float = 0.05, ordering: int = ORDER_MAXMIN,
                       nu: float = 1.5, rho: float = 0.15, n_points: int = 512, n_shifts: int = 4,
                       precision: int = PREC_FP64, nugget: float = 1e-8, family: int = COV_MATERN,
                       min_obs: int = 1) -> CensoredReplicate:
    """Uniform sites and one draw of a smooth field (smooth_field, same nu and
    rho as the model) censored at its (1 - frac_obs) normal quantile u: sites
    above u are observed with their value, the others sit at u (at least
    min_obs sites observed: the largest values)."""
    from statistics import NormalDist
    rng = np.random.Generator(np.random.PCG64(seed))
    locs = uniform_locations(D, rng)
    X = smooth_field(locs, rng, nu if family == COV_MATERN else 0.5, rho)
    u = NormalDist().inv_cdf(1.0 - frac_obs)
    obs = X > u
    if obs.sum() < min_obs:
        obs[np.argsort(-X)[:min_obs]] = True
    x = np.where(obs, np.maximum(X, u), u)
    inst = Instance(f"censored_D{D}_m{m}_s{seed}", locs, x, m, ordering, Cov(family, nu, 1.0, rho, nugget),
                    QMC(n_points, n_shifts, seed + 7, precision))
    return CensoredReplicate(inst, obs)


def station_network(n: int = 528, seed: int = seed_for(6, 0)) -> np.ndarray:
    """n irregular station locations in a 29 x 12 box (degrees of longitude and
    latitude of a western/central European network; the paper's 528 stations
    are not used)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.uniform(-5.0, 24.0, n), rng.uniform(43.0, 55.0, n)], axis=1)


def network_replicates(T: int = 1006, n: int = 528, missing: float = 0.326, exceed: float = 0.05,
                       rho: float = 1.31, m: int = 10, n_points: int = 1000, n_shifts: int = 10,
                       precision: int = PREC_FP32, seed: int = seed_for(6, 1)):
    """T weekly replicates on station_network(n), shaped like the application of
    Section 4.1: each station missing with probability `missing` in a week
    (dropped from that replicate), one smooth-field draw per week (exponential
    correlation scale rho), censored at each station's empirical (1 - exceed)
    quantile over the T weeks. Returns (locs, [CensoredReplicate]); replicate t's
    Instance holds its present stations only (locations in the same units)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    locs = station_network(n)
    fields = np.stack([smooth_field(locs, rng, 0.5, rho, n_features=256) for _ in range(T)])
    u = np.quantile(fields, 1.0 - exceed, axis=0)
    present = rng.random((T, n)) >= missing
    reps = []
    for t in range(T):
        idx = np.flatnonzero(present[t])
        X = fields[t, idx]
        obs = X > u[idx]
        x = np.where(obs, X, u[idx])
        inst = Instance(f"network_week{t}", locs[idx], x, m, ORDER_MAXMIN, Cov(COV_EXPONENTIAL, 0.5, 1.0, rho, 0.0),
                        QMC(n_points, n_shifts, seed_for(6, 2), precision))
        reps.append(CensoredReplicate(inst, obs))
    return locs, reps
