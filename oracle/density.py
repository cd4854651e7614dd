"""The density-dependent dielectric of the paper's Secs. II.C-II.D and its
potential term, for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 7 (the smoothed step of Fattebert and Gygi), with x = rho / rho_0:
    eps(rho) = 1 + (eps_inf - 1)/2 * (1 + (1 - x^(2 beta)) / (1 + x^(2 beta)))
which equals 1 + (eps_inf - 1) / (1 + x^(2 beta)); the density entering it is
an electron density, so negative values are read as zero.
Eq. 8:  d eps / d rho = (1 - eps_inf)/rho_0 * 2 beta x^(2 beta - 1) / (1 + x^(2 beta))^2.
Eq. 6:  V_eps = -(1 / 8 pi) |grad phi|^2 d eps / d rho; on the grid |grad
phi|^2 at a node is the mean of the squared forward and backward differences
along each axis, the same weights with which a node permittivity enters the
discrete energy, so that V_eps_n h^3 = (dE/d eps_n)(d eps_n / d rho_n) is
exactly the derivative of the discrete energy through the permittivity (and
Eq. 5, dE/d rho = phi + V_eps, holds on the grid).
"""
from __future__ import annotations

import numpy as np

from .poisson import eps_gradient


def eps_of_density(rho, eps_inf, rho0, beta):
    """Eq. 7 at every node (float64 arrays)."""
    x = np.maximum(np.asarray(rho, dtype=np.float64), 0.0) / rho0
    p = x ** (2.0 * beta)
    return 1.0 + 0.5 * (eps_inf - 1.0) * (1.0 + (1.0 - p) / (1.0 + p))


def deps_drho(rho, eps_inf, rho0, beta):
    """Eq. 8 at every node."""
    x = np.maximum(np.asarray(rho, dtype=np.float64), 0.0) / rho0
    p = x ** (2.0 * beta)
    return (1.0 - eps_inf) / rho0 * 2.0 * beta * x ** (2.0 * beta - 1.0) / (1.0 + p) ** 2


def v_eps(phi, rho, h, eps_inf, rho0, beta):
    """Eq. 6 on the grid: (dE/d eps_n / h^3) * (d eps / d rho)_n."""
    h3 = h[0] * h[1] * h[2]
    return eps_gradient(phi, h) / h3 * deps_drho(rho, eps_inf, rho0, beta)
