"""Operator, vacuum solve, full solve and energies of the oracle (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid convention: arrays are indexed [k][j][i] = [z][y][x]; node n sits at
(i hx, j hy, k hz); every direction is periodic.  h = (hx, hy, hz).
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi
_AXIS = (2, 1, 0)  # array axis of direction x, y, z


def apply_A(phi, eps, h):
    """(A phi)_n = sum_d [eps_{n+e/2} (phi_{n+e} - phi_n) - eps_{n-e/2} (phi_n - phi_{n-e})] / h_d^2.

    The conservative 7-point form of div(eps grad phi) (paper Eq. 3), with the
    face permittivity taken as the mean of its two nodes.
    """
    out = np.zeros_like(phi)
    for d in range(3):
        ax = _AXIS[d]
        eps_face = 0.5 * (eps + np.roll(eps, -1, axis=ax))     # face n + e_d/2
        flux = eps_face * (np.roll(phi, -1, axis=ax) - phi) / (h[d] * h[d])
        out += flux - np.roll(flux, 1, axis=ax)
    return out


def vacuum_symbol(shape, h):
    """lambda(m) = sum_d (2 - 2 cos(2 pi m_d / n_d)) / h_d^2 on the rfft grid.

    -lambda is the eigenvalue of the 7-point vacuum Laplacian on the Fourier
    mode m; this is the discrete counterpart of G^2 in Eq. 15.
    """
    nz, ny, nx = shape
    lx = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(nx // 2 + 1) / nx)) / h[0] ** 2
    ly = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(ny) / ny)) / h[1] ** 2
    lz = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(nz) / nz)) / h[2] ** 2
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def vacuum_solve(r, h):
    """Zero-mean psi with L psi = r - mean(r), L the 7-point vacuum Laplacian.

    Fourier inversion as in Eq. 15 (psi~ = -r~ / lambda, psi~(0) = 0).
    """
    lam = vacuum_symbol(r.shape, h)
    rh = np.fft.rfftn(r)
    lam[0, 0, 0] = 1.0
    ph = -rh / lam
    ph[0, 0, 0] = 0.0
    return np.fft.irfftn(ph, s=r.shape, axes=(0, 1, 2))


def residual_norm(phi, eps, rho, h):
    b = -FOUR_PI * (rho - rho.mean())
    return np.linalg.norm(b - apply_A(phi, eps, h)) / np.linalg.norm(b)


def solve(rho, eps, h, tol=1e-12, max_iter=2000, return_info=False):
    """The unique zero-mean phi with A phi = b, b = -4 pi (rho - mean rho).

    Conjugate gradients on A (negative semi-definite, null space = constants)
    preconditioned by the vacuum solve, started from zero and stopped when
    ||b - A phi||_2 <= tol ||b||_2 (true residual, FP64).
    """
    b = -FOUR_PI * (rho - rho.mean())
    bnorm = np.linalg.norm(b)
    phi = np.zeros_like(b)
    if bnorm == 0.0:
        return (phi, dict(iters=0, rel_res=0.0)) if return_info else phi
    r = b.copy()
    z = vacuum_solve(r, h)
    p = z.copy()
    rz = np.vdot(r, z)
    it = 0
    rel = 1.0
    history = []
    while it < max_iter:
        Ap = apply_A(p, eps, h)
        alpha = rz / np.vdot(p, Ap)
        phi += alpha * p
        r -= alpha * Ap
        it += 1
        if it % 25 == 0:  # refresh the recursive residual with the true one
            r = b - apply_A(phi, eps, h)
        rel = np.linalg.norm(r) / bnorm
        history.append(float(rel))
        if rel <= tol:
            rel = np.linalg.norm(b - apply_A(phi, eps, h)) / bnorm
            if rel <= tol:
                break
            r = b - apply_A(phi, eps, h)
        z = vacuum_solve(r, h)
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    phi -= phi.mean()
    if return_info:
        return phi, dict(iters=it, rel_res=float(rel), history=history)
    return phi


def energy(rho, phi, h):
    """E = 1/2 int phi rho = 1/2 h^3 sum_n rho_n phi_n (Hartree energy, Sec. II.C),
    summed with exact (compensated) accumulation."""
    h3 = h[0] * h[1] * h[2]
    return 0.5 * h3 * math.fsum((rho * phi).ravel())


def energy_eps_form(phi, eps, h):
    """E = (1/8 pi) int eps |grad phi|^2 (Eq. 4) in its exact discrete form:
    (h^3 / 8 pi) sum over faces eps_f (D_f phi)^2."""
    h3 = h[0] * h[1] * h[2]
    terms = []
    for d in range(3):
        ax = _AXIS[d]
        eps_face = 0.5 * (eps + np.roll(eps, -1, axis=ax))
        dphi = (np.roll(phi, -1, axis=ax) - phi) / h[d]
        terms.append((eps_face * dphi * dphi).ravel())
    return h3 / (2.0 * FOUR_PI) * math.fsum(np.concatenate(terms))


def eps_gradient(phi, h):
    """dE/d eps_n = -(h^3 / 8 pi) sum_d 1/2 [(D+_d phi)_n^2 + (D-_d phi)_n^2].

    The discrete form of the first term of Eq. 11: each node permittivity
    enters the two faces it shares with its neighbours along every direction
    with weight 1/2.
    """
    h3 = h[0] * h[1] * h[2]
    g = np.zeros_like(phi)
    for d in range(3):
        ax = _AXIS[d]
        dp = (np.roll(phi, -1, axis=ax) - phi) / h[d]   # forward difference
        dm = (phi - np.roll(phi, 1, axis=ax)) / h[d]    # backward difference
        g += 0.5 * (dp * dp + dm * dm)
    return -h3 / (2.0 * FOUR_PI) * g
