"""Randomized Richtmyer rank-1 lattice points for the SOV integrand.

The paper approximates each low-dimensional CDF with the QMC method of Genz &
Bretz (2009) (Section 2.2, after eq. (6)) and does not fix the point set.
Reading used here (all integer arithmetic, so any implementation of the same
definition produces the same bits):

* Generator: z_j = frac(sqrt(p_j)) with p_j the j-th prime (j = 0..62 for the
  63 dimensions a term can need), held as the 64-bit fixed-point integer
  Z_j = floor(frac(sqrt(p_j)) * 2^64) = isqrt(p_j * 2^128) mod 2^64.
* Shift: S = SplitMix64 output number n = (term << 21) | (shift << 5) | dim of
  the stream whose state starts at `seed` (Steele, Lea & Flood 2014), i.e.
  mix64(seed + (n + 1) * 0x9E3779B97F4A7C15 mod 2^64), for dim < 32; dimensions
  32..62 (terms of more than 32 variables) use n = 2^62 + (term << 22) +
  (shift << 6) + dim, a range the first form never reaches.
* Point p = 1..N of shift r in dimension j: U = (p * Z_j + S) mod 2^64.
* Baker (tent) transform: W = |2U - 2^64| (W = 2^64 saturates to 2^64 - 1).
* FP64 coordinate: the midpoint of the 2^-52 cell holding W / 2^64,
  w = (2 * floor(W / 2^12) + 1) * 2^-53, so 2^-53 <= w <= 1 - 2^-53 exactly.
* FP32 coordinate, from the upper 32 bits of U only: s = floor(U / 2^32) - 2^31
  as a signed integer, c = |s| >> 8 for s >= 0 and (|s| - 1) >> 8 for s < 0,
  w = (c + 1/2) 2^-23; within 2^-24 of the FP64 coordinate.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MAX_DIMS = 63
MAX_SHIFTS = 1 << 16


def first_primes(n: int) -> list:
    """The first n primes by trial division."""
    out = []
    c = 2
    while len(out) < n:
        if all(c % p for p in out if p * p <= c):
            out.append(c)
        c += 1
    return out


def richtmyer_generator(n_dims: int = MAX_DIMS) -> list:
    """Z_j = floor(frac(sqrt(p_j)) * 2^64) for the first n_dims primes."""
    return [math.isqrt(p << 128) & MASK64 for p in first_primes(n_dims)]


def splitmix64_mix(z: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood 2014; Vigna's constants)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_output(seed: int, n: int) -> int:
    """Output number n (0-based) of the SplitMix64 stream whose state starts at seed."""
    return splitmix64_mix((seed + (n + 1) * GOLDEN_GAMMA) & MASK64)


def shift(seed: int, term: int, r: int, dim: int, second: bool = False) -> int:
    """Random shift of dimension `dim` in replicate `r` of plan-order term `term`.
    second: the term's second, independent lattice (the denominator's points of
    the independent-points estimator), output number key + 2^61; no first-lattice
    key (below 2^53, or 2^62 + less than 2^54) and no full-dimension key
    (from 2^63) has bit 61 set."""
    assert 0 <= r < MAX_SHIFTS and 0 <= dim < 64 and term >= 0
    salt = (1 << 61) if second else 0
    if dim < 32:
        return splitmix64_output(seed, salt | (term << 21) | (r << 5) | dim)
    return splitmix64_output(seed, salt | (1 << 62) | (term << 22) | (r << 6) | dim)


def full_shift(seed: int, r: int, dim: int) -> int:
    """Random shift of dimension `dim` in replicate `r` of the full-dimension
    estimator (oracle.fullsov): SplitMix64 output n = 2^63 + r 2^32 + dim, a
    range no Vecchia term's key reaches."""
    assert 0 <= r < MAX_SHIFTS and 0 <= dim < (1 << 32)
    return splitmix64_output(seed, (1 << 63) | (r << 32) | dim)


def lattice_u(p: np.ndarray, Z: int, S: int) -> np.ndarray:
    """U = (p * Z + S) mod 2^64 for an array of point indices p (uint64)."""
    p = np.asarray(p, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return p * np.uint64(Z) + np.uint64(S)


def baker_w(U: np.ndarray) -> np.ndarray:
    """W = |2U - 2^64| with 2^64 saturated to 2^64 - 1 (uint64)."""
    U = np.asarray(U, dtype=np.uint64)
    half = np.uint64(1 << 63)
    with np.errstate(over="ignore"):
        hi = (U - half) * np.uint64(2)           # U >= 2^63: 2U - 2^64
        lo = (half - U) * np.uint64(2)           # U <  2^63: 2^64 - 2U (0 when U = 0)
    W = np.where(U >= half, hi, lo)
    W = np.where(U == 0, np.uint64(MASK64), W)
    return W


def coord_f64(W: np.ndarray) -> np.ndarray:
    n = (np.asarray(W, dtype=np.uint64) >> np.uint64(12)).astype(np.float64)
    return (2.0 * n + 1.0) * 2.0 ** -53


def coord_f32_from_u(U: np.ndarray) -> np.ndarray:
    s = (np.asarray(U, dtype=np.uint64) >> np.uint64(32)).astype(np.int64) - (1 << 31)
    c = np.where(s >= 0, s >> 8, (-s - 1) >> 8).astype(np.float64)
    return (c + 0.5) * 2.0 ** -23


def points(n_points: int, dim: int, S: int, Z: list | None = None,
           fp32: bool = False) -> np.ndarray:
    """Coordinates w_p (p = 1..N) of dimension `dim` for shift S."""
    Z = richtmyer_generator() if Z is None else Z
    p = np.arange(1, n_points + 1, dtype=np.uint64)
    U = lattice_u(p, Z[dim], S)
    return coord_f32_from_u(U) if fp32 else coord_f64(baker_w(U))
