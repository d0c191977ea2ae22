"""Pins of the oracle's components against definitions that do not come from it:
published generator outputs, integer invariants, textbook covariance forms and
brute force on tiny inputs."""
import math
import os

import numpy as np
import pytest
from scipy.special import gamma, kv

from oracle import covariance, lattice, neighbours, ordering

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- lattice ---

def test_splitmix64_published_outputs():
    for idx, hexval in _read_golden("splitmix64_state0.txt"):
        assert lattice.splitmix64_output(0, int(idx)) == int(hexval, 16)


def test_first_primes_table():
    want = [int(v) for v in _read_golden("primes31.txt")[0]]
    assert lattice.first_primes(31) == want


def test_richtmyer_generator_is_frac_sqrt_prime():
    Z = lattice.richtmyer_generator()
    assert len(Z) == 63 and lattice.first_primes(63)[-1] == 307   # the 63rd prime
    for p, z in zip(lattice.first_primes(63), Z):
        ip = math.isqrt(p)
        full = (ip << 64) + z                      # floor(sqrt(p) * 2^64)
        assert full * full <= p << 128 < (full + 1) * (full + 1)
        assert abs(z / 2.0 ** 64 - (math.sqrt(p) - ip)) <= 2 * math.ulp(math.sqrt(p))
    assert len(set(Z)) == 63


def test_baker_transform_edges_and_symmetry():
    U = np.array([0, 1 << 63, (1 << 63) + 5, (1 << 63) - 5, 1, (1 << 64) - 1], dtype=np.uint64)
    W = lattice.baker_w(U)
    assert int(W[0]) == (1 << 64) - 1          # 2^64 saturates
    assert int(W[1]) == 0
    assert int(W[2]) == int(W[3]) == 10
    assert int(W[4]) == int(W[5]) == (1 << 64) - 2
    w = lattice.coord_f64(W)
    assert w[1] == 2.0 ** -53 and w[0] == 1.0 - 2.0 ** -53
    w32 = lattice.coord_f32_from_u(U)
    assert w32[1] == 2.0 ** -24 and w32[0] == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(5)
    U = rng.integers(1, 2 ** 63, size=1000, dtype=np.uint64)
    with np.errstate(over="ignore"):
        Uc = np.uint64(0) - U                       # 2^64 - U
    assert np.array_equal(lattice.baker_w(U), lattice.baker_w(Uc))
    # the FP32 coordinate is the midpoint of the FP64 coordinate's 2^-23 cell
    # (one cell lower only when U's low 40 bits are zero): within 2^-24
    edge = np.array([k << 40 for k in range(0, 1 << 24, 4099)] + [(1 << 63) + (3 << 40)], dtype=np.uint64)
    U = np.concatenate([rng.integers(0, 2 ** 64 - 1, size=100000, dtype=np.uint64), edge])
    W = lattice.baker_w(U)
    d = np.abs(lattice.coord_f32_from_u(U) - lattice.coord_f64(W))
    assert np.all(d <= 2.0 ** -24 + 2.0 ** -53)
    cell64 = (W >> np.uint64(41)).astype(np.int64)
    cell32 = np.floor(lattice.coord_f32_from_u(U) * 2 ** 23).astype(np.int64)
    low0 = (U & np.uint64((1 << 40) - 1)) == 0
    assert np.array_equal(cell32[~low0], cell64[~low0])


def test_lattice_rule_integrates_smooth_product():
    # int_[0,1]^5 prod_j 2 w_j dw = 1; a degenerate generator (equal Z_j,
    # points on a line) would give E[(2w)^5] = 16/3.
    N = 4093
    f = np.ones(N)
    for j in range(5):
        f *= 2.0 * lattice.points(N, j, lattice.shift(11, 0, 0, j))
    assert abs(f.mean() - 1.0) < 2e-3
    # int_[0,1]^3 prod_j 3 w_j^2 dw = 1: the error at N = 16381 is far below
    # plain Monte Carlo's (sd of the integrand / sqrt(N) ~ 1.4e-2)
    N = 16381
    g = np.ones(N)
    for j in range(3):
        g *= 3.0 * lattice.points(N, j, lattice.shift(3, 0, 0, j)) ** 2
    assert abs(g.mean() - 1.0) < 1e-3


def test_shift_keys_are_distinct():
    seen = set()
    for term in range(4):
        for r in range(3):
            for d in range(63):
                seen.add(lattice.shift(99, term, r, d))
    assert len(seen) == 4 * 3 * 63
    # the two key forms as stated
    assert lattice.shift(7, 5, 2, 31) == lattice.splitmix64_output(7, (5 << 21) | (2 << 5) | 31)
    assert lattice.shift(7, 5, 2, 32) == lattice.splitmix64_output(7, (1 << 62) | (5 << 22) | (2 << 6) | 32)


# ------------------------------------------------------------- covariance ---

def _matern_bessel(h, nu, sigma2, rho):
    a = np.sqrt(2.0 * nu) * h / rho
    return sigma2 * 2.0 ** (1.0 - nu) / gamma(nu) * a ** nu * kv(nu, a)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_closed_forms_match_bessel_form(nu):
    h = np.linspace(1e-4, 1.0, 200)
    got = covariance.kernel(h, covariance.COV_MATERN, nu, 1.7, 0.13)
    want = _matern_bessel(h, nu, 1.7, 0.13)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-300)
    assert covariance.kernel(np.array([0.0]), covariance.COV_MATERN, nu, 1.7, 0.13)[0] == 1.7


def test_exponential_is_matern_half():
    h = np.linspace(0, 2, 50)
    np.testing.assert_array_equal(covariance.kernel(h, covariance.COV_EXPONENTIAL, 0.0, 2.0, 0.3),
                                  2.0 * np.exp(-h / 0.3))


def test_cov_matrix_nugget_and_symmetry():
    pts = np.random.default_rng(1).random((6, 2))
    C = covariance.cov_matrix(pts, covariance.COV_MATERN, 1.5, 1.0, 0.2, 0.01)
    assert np.allclose(C, C.T)
    assert np.all(np.diag(C) == 1.01)
    assert np.all(np.linalg.eigvalsh(C) > 0)


# ---------------------------------------------------------------- ordering ---

def _brute_maxmin(locs):
    D = len(locs)
    d2 = lambda a, b: (a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1])
    cx = (min(p[0] for p in locs) + max(p[0] for p in locs)) / 2.0
    cy = (min(p[1] for p in locs) + max(p[1] for p in locs)) / 2.0
    first = min(range(D), key=lambda j: (d2(locs[j], (cx, cy)), j))
    sel = [first]
    while len(sel) < D:
        best, bestkey = None, None
        for j in range(D):
            if j in sel:
                continue
            md = min(d2(locs[j], locs[s]) for s in sel)
            key = (-md, j)
            if bestkey is None or key < bestkey:
                best, bestkey = j, key
        sel.append(best)
    return sel


@pytest.mark.parametrize("case", ["uniform", "grid", "dupes"])
def test_maxmin_matches_brute_force(case):
    rng = np.random.default_rng(3)
    if case == "uniform":
        locs = rng.random((40, 2))
    elif case == "grid":
        a, b = np.meshgrid(np.arange(6), np.arange(5), indexing="ij")
        locs = np.stack([a.ravel() / 5.0, b.ravel() / 4.0], axis=1)
    else:
        locs = np.round(rng.random((30, 2)) * 4) / 4.0      # many exact ties / duplicates
    got = ordering.maxmin_order(locs)
    assert list(got) == _brute_maxmin([tuple(p) for p in locs])


def test_coord_order_matches_sorted():
    rng = np.random.default_rng(4)
    locs = np.round(rng.random((50, 2)) * 3) / 3.0
    want = sorted(range(50), key=lambda j: (locs[j, 0], locs[j, 1], j))
    assert list(ordering.coord_order(locs)) == want


def test_given_order_validation():
    assert list(ordering.order(np.zeros((3, 2)), ordering.ORDER_GIVEN, np.array([2, 0, 1]))) == [2, 0, 1]
    with pytest.raises(ValueError):
        ordering.order(np.zeros((3, 2)), ordering.ORDER_GIVEN, np.array([0, 0, 1]))


# -------------------------------------------------------------- neighbours ---

@pytest.mark.parametrize("m", [0, 1, 3, 7])
def test_knn_preceding_matches_brute_force(m):
    rng = np.random.default_rng(7)
    s = np.concatenate([np.round(rng.random((25, 2)) * 3) / 3.0, rng.random((15, 2))])
    got = neighbours.knn_preceding(s, m)
    for i in range(len(s)):
        keys = sorted(((s[i, 0] - s[j, 0]) ** 2 + (s[i, 1] - s[j, 1]) ** 2, j) for j in range(i))
        assert list(got[i]) == [j for _, j in keys[:min(m, i)]]
