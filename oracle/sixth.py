"""The paper's sixth-order operator (Sec. II.F, Eqs. 16-18) in the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 16 expands div(eps grad phi) as grad eps . grad phi + eps lap phi (the
printed last term reads eps times the Laplacian of eps, a typo: it is the
Laplacian of phi).  Each derivative is the central seven-point formula of
Eq. 17 (first derivative) or Eq. 18 (second derivative) along one axis:
    D1 f_i = (1/h)   sum_{n=1..3} alpha_n (f_{i+n} - f_{i-n}),
    D2 f_i = (1/h^2) [beta_0 f_i + sum_{n=1..3} beta_n (f_{i+n} + f_{i-n})],
with alpha = (3/4, -3/20, 1/60) and beta = (-49/18, 3/2, -3/20, 1/90); both
are O(h^6) (the printed O(h^7) is one order too high).  Every axis is
periodic, so
    A6 phi = sum_d [(D1_d eps)(D1_d phi) + eps (D2_d phi)].

A6 is not symmetric, and its range is not the zero-mean vectors: the sum of
A6 phi is O(h^6) small but not zero.  The discrete problem is therefore read
as: the zero-mean phi and the constant c with A6 phi = b - c, b = -4 pi (rho -
mean rho); c is the extra uniform background that makes the system solvable.
Equivalently, with Q the removal of the mean, Q A6 phi = b on zero-mean phi.

Energy E = 1/2 h^3 sum rho phi as with the second-order operator.  Its
gradient needs the adjoint: the zero-mean lambda with Q A6^T lambda =
1/2 h^3 Q rho gives
    dE/d eps_n = sum_d D1_d(lambda D1_d phi)_n - lambda_n (sum_d D2_d phi)_n,
    dE/d rho_n = 1/2 h^3 phi_n - 4 pi lambda_n,
(for a symmetric operator lambda = -h^3 phi / 8 pi and these reduce to the
familiar -|grad phi|^2 h^3 / 8 pi and h^3 phi).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from .poisson import FOUR_PI, _AXIS, solve

ALPHA = (0.75, -0.15, 1.0 / 60.0)                       # Eq. 17: alpha_1..3
BETA = (-49.0 / 18.0, 1.5, -0.15, 1.0 / 90.0)           # Eq. 18: beta_0..3


def d1(f, h, d):
    """Sixth-order first derivative along direction d (Eq. 17), periodic."""
    ax = _AXIS[d]
    out = np.zeros_like(f)
    for n, a in enumerate(ALPHA, start=1):
        out += a * (np.roll(f, -n, axis=ax) - np.roll(f, n, axis=ax))
    return out / h[d]


def d2(f, h, d):
    """Sixth-order second derivative along direction d (Eq. 18), periodic."""
    ax = _AXIS[d]
    out = BETA[0] * f
    for n in range(1, 4):
        out = out + BETA[n] * (np.roll(f, -n, axis=ax) + np.roll(f, n, axis=ax))
    return out / (h[d] * h[d])


def apply_A6(phi, eps, h):
    """Eq. 16 (corrected) with the stencils of Eqs. 17-18."""
    out = np.zeros_like(phi)
    for d in range(3):
        out += d1(eps, h, d) * d1(phi, h, d) + eps * d2(phi, h, d)
    return out


def apply_A6T(psi, eps, h):
    """The transpose of apply_A6: D1 is antisymmetric and D2 symmetric, so
    A6^T psi = sum_d [-D1_d((D1_d eps) psi) + D2_d(eps psi)]."""
    out = np.zeros_like(psi)
    for d in range(3):
        out += -d1(d1(eps, h, d) * psi, h, d) + d2(eps * psi, h, d)
    return out


def symbol6(shape, h):
    """mu(m) = -sum_d (1/h_d^2)[beta_0 + 2 sum_n beta_n cos(2 pi n m_d / n_d)]
    on the rfft grid: -mu is the eigenvalue of sum_d D2_d on the mode m."""
    nz, ny, nx = shape

    def axis(n, hd, half):
        m = np.arange(n // 2 + 1 if half else n)
        th = 2.0 * math.pi * m / n
        s = BETA[0] + 2.0 * sum(BETA[k] * np.cos(k * th) for k in range(1, 4))
        return -s / (hd * hd)

    return axis(nz, h[2], False)[:, None, None] + axis(ny, h[1], False)[None, :, None] \
        + axis(nx, h[0], True)[None, None, :]


def vacuum_solve6(r, h):
    """Zero-mean psi with (sum_d D2_d) psi = r - mean(r), by Fourier inversion."""
    mu = symbol6(r.shape, h)
    rh = np.fft.rfftn(r)
    mu[0, 0, 0] = 1.0
    ph = -rh / mu
    ph[0, 0, 0] = 0.0
    return np.fft.irfftn(ph, s=r.shape, axes=(0, 1, 2))


def _precondition(r, eps, h):
    """The second-order operator's exact inverse on zero-mean r (the oracle's
    own PCG solve of A phi = r), a close spectral match to A6 and A6^T: their
    symbols differ by at most a factor 1.5 on every mode."""
    if eps is None:
        return vacuum_solve6(r, h)
    return solve(-r / FOUR_PI, eps, h, tol=1e-13, max_iter=4000)


def _gmres(apply_op, rhs, h, tol, max_iter, eps):
    """Zero-mean x with Q op(x) = rhs (rhs zero-mean): GMRES on Q op M with M
    the second-order inverse as right preconditioner, x = M y."""
    shape = rhs.shape
    size = rhs.size

    def qop(y):
        x = _precondition(y.reshape(shape), eps, h)
        v = apply_op(x)
        return (v - v.mean()).ravel()

    K = spla.LinearOperator((size, size), matvec=qop, dtype=np.float64)
    bn = np.linalg.norm(rhs)
    if bn == 0.0:
        return np.zeros(shape), 0, 0.0
    its = [0]

    def count(_):
        its[0] += 1

    y, info = spla.gmres(K, rhs.ravel(), rtol=tol, atol=0.0, restart=60, maxiter=max_iter,
                         callback=count, callback_type="pr_norm")
    x = _precondition(y.reshape(shape), eps, h)
    v = apply_op(x)
    rel = float(np.linalg.norm((v - v.mean()) - rhs) / bn)
    return x - x.mean(), its[0], rel


def solve6(rho, eps, h, tol=1e-12, max_iter=10, return_info=False):
    """The zero-mean phi with Q A6 phi = b, b = -4 pi (rho - mean rho).
    Also returns c = mean(b - A6 phi) in the info dict."""
    b = -FOUR_PI * (rho - rho.mean())
    phi, its, rel = _gmres(lambda x: apply_A6(x, eps, h), b, h, tol, max_iter, eps)
    if return_info:
        c = float(np.mean(b - apply_A6(phi, eps, h)))
        return phi, dict(iters=its, rel_res=rel, background=c)
    return phi


def residual_norm6(phi, eps, rho, h):
    b = -FOUR_PI * (rho - rho.mean())
    v = apply_A6(phi, eps, h)
    return float(np.linalg.norm((v - v.mean()) - b) / np.linalg.norm(b))


def adjoint6(rho, eps, h, tol=1e-12, max_iter=10):
    """The zero-mean lambda with Q A6^T lambda = 1/2 h^3 (rho - mean rho)."""
    h3 = h[0] * h[1] * h[2]
    f = 0.5 * h3 * (rho - rho.mean())
    lam, _, _ = _gmres(lambda x: apply_A6T(x, eps, h), f, h, tol, max_iter, eps)
    return lam


def eps_gradient6(phi, lam, h):
    """dE/d eps_n = sum_d D1_d(lambda D1_d phi)_n - lambda_n (sum_d D2_d phi)_n."""
    g = np.zeros_like(phi)
    for d in range(3):
        g += d1(lam * d1(phi, h, d), h, d) - lam * d2(phi, h, d)
    return g


def charge_potential6(phi, lam, h):
    """psi with h^3 psi_n = dE/d rho_n = 1/2 h^3 phi_n - 4 pi lambda_n."""
    h3 = h[0] * h[1] * h[2]
    return 0.5 * phi - FOUR_PI * lam / h3
