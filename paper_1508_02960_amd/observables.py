"""Host-side observables of a pressure-driven sphere-pack run (lattice units,
rho0 = 1, so the dynamic viscosity equals nu).

  permeability       eq. (Darcy): K_D = mu U / |grad P|, grad P = dp / L,
                     dp = delta_rho / 3, L = nx
  reynolds_p         Re_p = rho D U / mu with D the sphere diameter
  drag_coefficient   eq. (AnalyticForce): C_D = F / (6 pi mu U r)
  forchheimer_fit    eq. (Forchheimer): |grad P| = mu U / K_D + beta rho U^2,
                     fitted by least squares as |grad P|/U = mu/K_D + beta U;
                     C_F = beta sqrt(K_D)
  friction_factor    eq. (frictionFactor): F_K = (dp/L) sqrt(K_D) / (rho U^2),
                     Re_K = rho U sqrt(K_D) / mu
"""
from __future__ import annotations

import numpy as np


def viscosity(tau: float) -> float:
    """nu = (tau - 1/2) / 3 (omega+ = (3 nu + 1/2)^-1, Sec. 2.1)."""
    return (tau - 0.5) / 3.0


def pressure_gradient(delta_rho: float, nx: int) -> float:
    return delta_rho / 3.0 / nx


def permeability(U: float, delta_rho: float, nx: int, tau: float) -> float:
    return viscosity(tau) * U / pressure_gradient(delta_rho, nx)


def reynolds_p(U: float, diameter: float, tau: float) -> float:
    return U * diameter / viscosity(tau)


def drag_coefficient(F: float, U: float, radius: float, tau: float) -> float:
    return F / (6.0 * np.pi * viscosity(tau) * U * radius)


def delta_rho_for_reynolds(re_p: float, diameter: float, tau: float, nx: int, K: float) -> float:
    """Pressure jump that gives Re_p in the Darcy regime for permeability K:
    U = Re nu / D and dp/L = nu U / K, so delta_rho = 3 nx nu^2 Re / (D K)."""
    nu = viscosity(tau)
    return 3.0 * nx * nu * nu * re_p / (diameter * K)


def forchheimer_fit(grad_p, U, tau: float):
    """Least-squares fit of |grad P| / U = nu / K_D + beta U.

    Returns (K_D, beta, C_F)."""
    g = np.asarray(grad_p, dtype=np.float64)
    u = np.asarray(U, dtype=np.float64)
    A = np.stack([np.ones_like(u), u], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, g / u, rcond=None)
    K = viscosity(tau) / a
    return K, b, b * np.sqrt(K)


def friction_factor(grad_p: float, U: float, K: float, tau: float):
    """(F_K, Re_K)."""
    return grad_p * np.sqrt(K) / (U * U), U * np.sqrt(K) / viscosity(tau)
