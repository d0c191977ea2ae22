"""Stationary isotropic covariance of the Gaussian process.

The paper's simulations use the exponential model with unit variance (Section
3) and the application an exponential model exp(-h / rho) (Section 4.1). The
Matern family generalises it; its parameterisation is not in the paper, so the
common one is used:
  K(h) = sigma2 * 2^(1-nu) / Gamma(nu) * (sqrt(2 nu) h / rho)^nu * K_nu(sqrt(2 nu) h / rho),
whose half-integer cases have the closed forms below (nu = 1/2 is exp(-h/rho)).
A nugget tau >= 0 is added on the diagonal.
"""
from __future__ import annotations

import math

import numpy as np

COV_EXPONENTIAL, COV_MATERN = 0, 1


def kernel(h: np.ndarray, family: int, nu: float, sigma2: float, rho: float) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    if family == COV_EXPONENTIAL or (family == COV_MATERN and nu == 0.5):
        return sigma2 * np.exp(-h / rho)
    if family == COV_MATERN and nu == 1.5:
        a = math.sqrt(3.0) * h / rho
        return sigma2 * (1.0 + a) * np.exp(-a)
    if family == COV_MATERN and nu == 2.5:
        a = math.sqrt(5.0) * h / rho
        return sigma2 * (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError("supported: exponential, Matern nu in {0.5, 1.5, 2.5}")


def cov_matrix(pts: np.ndarray, family: int, nu: float, sigma2: float, rho: float,
               nugget: float) -> np.ndarray:
    dx = pts[:, None, 0] - pts[None, :, 0]
    dy = pts[:, None, 1] - pts[None, :, 1]
    h = np.sqrt(dx * dx + dy * dy)
    C = kernel(h, family, nu, sigma2, rho)
    C[np.diag_indices_from(C)] += nugget
    return C


def mahalanobis_distance(si, sj, phi: float, A: float) -> float:
    """Section 4.1's anisotropic distance: h = |Omega| with the row vector
    Omega = (s_i - s_j)^T R(phi)^-1 diag(1, A), R(phi) the rotation by phi
    (angle in [0, pi), aspect ratio A > 1). The exponential covariance
    exp(-h / rho) of that section uses it."""
    R = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    d = np.asarray(si, dtype=np.float64) - np.asarray(sj, dtype=np.float64)
    omega = d @ np.linalg.inv(R) @ np.diag([1.0, A])
    return float(math.sqrt(omega @ omega))


def anisotropic_coords(locs, phi: float, A: float) -> np.ndarray:
    """Points whose Euclidean distances are mahalanobis_distance: each row
    s^T R(phi)^-1 diag(1, A) (the map is linear, so differences map to Omega)."""
    R = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    return np.asarray(locs, dtype=np.float64) @ np.linalg.inv(R) @ np.diag([1.0, A])
