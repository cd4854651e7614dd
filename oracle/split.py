"""The paper's one-pass dry/wet split (Sec. II.F), as a diagnostic.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Step 1: the vacuum potential phi_vac = L^{-1} b on the whole periodic box
(epsilon = 1, FFT).  Step 2: inside the wet slab W = planes [k0, k1) (mod nz)
the dielectric problem is solved again with phi_vac as Dirichlet data on every
node outside W.  Step 3: phi = the wet solution inside W, phi_vac outside.
This is exact only when the dielectric does not perturb the potential outside
W; the full solver does not use it, it reports how far it is from the exact
solution.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.fft import dst
from scipy.sparse.linalg import LinearOperator, cg

from .poisson import apply_A, vacuum_solve


def dirichlet_laplace_solve(v, h):
    """u with -L u = v on a slab of planes (axis 0), L the constant-coefficient
    7-point Laplacian, zero Dirichlet data on the planes just outside the slab,
    x and y periodic.

    Eigen-decomposition: Fourier modes in x and y, sine modes sin(pi k j / (m + 1))
    (j = 1..m, k = 1..m) in z, whose eigenvalue of -L is the sum over the axes of
    (2 - 2 cos theta_d) / h_d^2 with theta = 2 pi m_x / nx, 2 pi m_y / ny,
    pi k / (m + 1).  Only a preconditioner here: it sets how fast the wet solve
    converges, not what it converges to.
    """
    m, ny, nx = v.shape
    lx = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(nx // 2 + 1) / nx)) / h[0] ** 2
    ly = (2.0 - 2.0 * np.cos(2.0 * math.pi * np.arange(ny) / ny)) / h[1] ** 2
    lz = (2.0 - 2.0 * np.cos(math.pi * np.arange(1, m + 1) / (m + 1))) / h[2] ** 2
    lam = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
    vh = dst(np.fft.rfft2(v, axes=(1, 2)), type=1, axis=0)
    # DST-I applied twice is 2 (m + 1) times the identity
    uh = dst(vh / lam, type=1, axis=0) / (2.0 * (m + 1))
    return np.fft.irfft2(uh, s=(ny, nx), axes=(1, 2))


def one_pass_split(rho, eps, h, k0, k1, tol=1e-13, maxiter=20000):
    nz = rho.shape[0]
    b = -4.0 * math.pi * (rho - rho.mean())
    phi_vac = vacuum_solve(b, h)
    wet = np.zeros(nz, dtype=bool)
    wet[np.arange(k0, k1) % nz] = True
    mask = np.broadcast_to(wet[:, None, None], rho.shape)
    nW = int(mask.sum())

    def extend(xw):
        full = np.zeros_like(rho)
        full[mask] = xw
        return full

    def op(xw):
        return -apply_A(extend(xw), eps, h)[mask]

    dry_part = np.where(mask, 0.0, phi_vac)
    rhs = -(b - apply_A(dry_part, eps, h))[mask]
    # Preconditioner eps^-1/2 (-L_D)^-1 eps^-1/2 with the constant-coefficient
    # Dirichlet Laplacian of the slab (planes taken in slab order, k0 first)
    planes = np.arange(k0, k1) % nz
    sw = 1.0 / np.sqrt(eps)

    def prec(xw):
        full = extend(xw) * sw
        full[planes] = dirichlet_laplace_solve(full[planes], h)
        return (full * sw)[mask]

    A = LinearOperator((nW, nW), matvec=op, dtype=np.float64)
    M = LinearOperator((nW, nW), matvec=prec, dtype=np.float64)
    xw, info = cg(A, rhs, rtol=tol, atol=0.0, maxiter=maxiter, M=M)
    if info != 0:
        raise RuntimeError(f"wet-slab Dirichlet solve did not converge (info={info})")
    phi = np.where(mask, extend(xw), phi_vac)
    return phi - phi.mean()
