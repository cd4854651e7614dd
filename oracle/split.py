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
from scipy.sparse.linalg import LinearOperator, cg

from .poisson import apply_A, vacuum_solve


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
    # Jacobi preconditioner: the diagonal of -A is sum over faces eps_f / h^2
    diag = np.zeros_like(rho)
    for d, ax in zip(range(3), (2, 1, 0)):
        diag += 0.5 * (2 * eps + np.roll(eps, -1, ax) + np.roll(eps, 1, ax)) / h[d] ** 2
    dinv = 1.0 / diag[mask]
    A = LinearOperator((nW, nW), matvec=op, dtype=np.float64)
    M = LinearOperator((nW, nW), matvec=lambda v: dinv * v, dtype=np.float64)
    xw, info = cg(A, rhs, rtol=tol, atol=0.0, maxiter=maxiter, M=M)
    if info != 0:
        raise RuntimeError(f"wet-slab Dirichlet solve did not converge (info={info})")
    phi = np.where(mask, extend(xw), phi_vac)
    return phi - phi.mean()
