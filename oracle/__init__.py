"""Plain, slow CPU FP64 oracle for the Vecchia approximation of a Gaussian log-CDF.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package. The GPU library
never calls it and shares no code, header, table or constant generator with it.

What it computes (Nascimento & Shaby, "A Vecchia Approximation for
High-Dimensional Gaussian Cumulative Distribution Functions Arising from Spatial
Data"):

* Section 2.2, eq. (6): log F(x) ~= log Phi(x_1) + sum_i [log Phi_{k+1}(x_{i,N_i})
  - log Phi_k(x_{N_i})], with N_i the k_i = min(m, i-1) nearest preceding
  locations (Section 2.1, the text after eq. (4)).
* Each ratio is estimated by Genz's separation-of-variables (SOV) transform to
  the unit cube (Introduction, Genz 1992) and a randomized rank-1 lattice QMC
  rule (Genz & Bretz 2009), numerator and denominator on the same points.
* Terms are computed on the log scale and summed at the end (Section 3.1).

Modules:
  lattice     Richtmyer rank-1 lattice, baker transform, SplitMix64 shifts.
  ordering    coordinate and maxmin orderings.
  neighbours  nearest preceding neighbours under the (d^2, index) order.
  covariance  exponential / Matern covariance with a nugget.
  sov         one Vecchia term: Cholesky + SOV chain + QMC mean and SE.
  vecchia     the whole log-CDF: order, neighbours, terms, log-space sum.
  mixture     the scale-mixture outer integral over R (eqs. (8)-(9), (11)).
  censored    the censored likelihood of one replicate in Vecchia form (eq. (11)).
  block       joint (block) conditional terms (Section 3.2).
  fullsov     the full-dimension SOV estimate, the paper's comparator (Section 3.1).

Where the paper leaves a point open (orderings, ties, lattice, shifts, SE,
shared numerator/denominator points), the module that takes the reading says
which one it takes in its own header. Parity of the Vecchia approximation itself against the true CDF for
m < D-1 and a general covariance is unpinned (no closed form exists); the tests
pin every component and the exact special cases instead.
"""
from . import lattice, ordering, neighbours, covariance, sov, vecchia, mixture, censored, block, fullsov  # noqa: F401
from .vecchia import logcdf, logcdf_from_cov, plan  # noqa: F401
