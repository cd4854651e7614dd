"""Pins of the oracle's sixth-order operator (Sec. II.F, Eqs. 16-18).

* Eqs. 17-18 on smooth periodic functions: the error falls as h^6 (the
  measured order on 16 -> 32 -> 64 points is 6, not the printed 7);
* the symbol used by the vacuum solve is the eigenvalue of the stencil on
  each Fourier mode, so with eps = 1 the solve is the Fourier inversion;
* A6 against the exact div(eps grad phi) of a manufactured periodic pair:
  sixth-order convergence; the discrete solution of A6 phi = b - c against the
  exact phi: sixth order, below 1e-4 relative already on 24^3 points, and the
  background c that makes the system solvable vanishes as h^6;
* A6^T is the transpose of A6;
* the adjoint gradient dE/d eps and dE/d rho against central differences of
  the energy;
* with the sixth-order operator and atoms, dE/dR against central differences.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import sixth as S
from paper_0904_4887_amd import workloads as W


def _grid(n, L):
    h = tuple(L[d] / n[d] for d in range(3))
    z, y, x = np.meshgrid(*(np.arange(n[d]) * h[d] for d in (2, 1, 0)), indexing="ij")
    return h, x, y, z


def test_stencils_are_sixth_order():
    L = (2.0, 3.0, 2.5)
    errs1, errs2 = [], []
    for m in (16, 32, 64):
        n = (m, m, m)
        h, x, y, z = _grid(n, L)
        k = 2 * math.pi / L[1] * 2
        f = np.sin(k * y + 0.3)
        errs1.append(np.abs(S.d1(f, h, 1) - k * np.cos(k * y + 0.3)).max())
        errs2.append(np.abs(S.d2(f, h, 1) + k * k * f).max())
    for e in (errs1, errs2):
        orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(5.8 < o < 6.3 for o in orders), (e, orders)


def test_symbol_is_the_stencil_eigenvalue_and_eps_one_is_the_fourier_inverse():
    n, L = (12, 18, 10), (3.0, 4.5, 2.0)
    h, x, y, z = _grid(n, L)
    m = (2, 5, 3)
    mode = np.cos(2 * math.pi * (m[0] * x / L[0] + m[1] * y / L[1] + m[2] * z / L[2]))
    lap = sum(S.d2(mode, h, d) for d in range(3))
    mu = S.symbol6(mode.shape, h)[m[2], m[1], m[0]]
    assert np.abs(lap + mu * mode).max() <= 1e-11 * mu
    rng = np.random.default_rng(3)
    rho = rng.normal(size=(n[2], n[1], n[0]))
    phi = S.solve6(rho, np.ones_like(rho), h, tol=1e-13)
    ref = S.vacuum_solve6(-4 * math.pi * (rho - rho.mean()), h)
    assert np.abs(phi - ref).max() <= 1e-11 * np.abs(ref).max()


def _manufactured(n, L=(2.0, 2.0, 3.0)):
    h, x, y, z = _grid(n, L)
    kx, ky, kz = 2 * math.pi / L[0], 2 * math.pi / L[1], 4 * math.pi / L[2]
    qx, qz = 2 * math.pi / L[0], 2 * math.pi / L[2]
    th = kx * x + ky * y + kz * z
    phi = np.sin(th)
    eps = 2.0 + np.cos(qx * x) * np.cos(qz * z)
    ex = -qx * np.sin(qx * x) * np.cos(qz * z)
    ez = -qz * np.cos(qx * x) * np.sin(qz * z)
    div = eps * (-(kx * kx + ky * ky + kz * kz) * np.sin(th)) + (ex * kx + ez * kz) * np.cos(th)
    return h, phi, eps, div


def test_operator_and_solution_converge_at_sixth_order():
    op_err, sol_err, bg = [], [], []
    for m in (12, 24, 48):
        h, phi, eps, div = _manufactured((m, m, m))
        op_err.append(np.abs(S.apply_A6(phi, eps, h) - div).max() / np.abs(div).max())
        rho = -div / (4 * math.pi)          # so that b = div (zero mean already)
        sol, info = S.solve6(rho, eps, h, tol=1e-13, return_info=True)
        sol_err.append(np.abs(sol - phi).max())
        # this pair has no common frequencies, so the discrete sum of A6 phi is 0
        assert abs(info["background"]) <= 1e-12
        # phi = cos(k x), eps = 2 + cos(k x): the sum of A6 phi is N (khat^2 - ktilde^2)/2
        # with the first- and second-derivative symbols khat, ktilde: O(h^6), not 0
        h1, x1 = h[0], np.arange(m) * h[0]
        k = 2 * math.pi / 2.0
        p1 = np.broadcast_to(np.cos(k * x1)[None, None, :], (m, m, m)).copy()
        e1 = 2.0 + p1
        khat = 2 * sum(a * math.sin(n * k * h1) for n, a in enumerate(S.ALPHA, start=1)) / h1
        ktil = -(S.BETA[0] + 2 * sum(b * math.cos(n * k * h1) for n, b in enumerate(S.BETA[1:], start=1))) / h1 ** 2
        got = float(np.mean(S.apply_A6(p1, e1, h)))
        assert abs(got - 0.5 * (khat ** 2 - ktil)) <= 1e-12 * k * k
        bg.append(abs(0.5 * (khat ** 2 - ktil)))
    for e in (op_err, sol_err, bg):
        orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(o > 5.5 for o in orders), (e, orders)
    assert sol_err[1] < 1e-4


def test_transpose():
    n, L = (10, 12, 14), (3.0, 3.6, 4.2)
    h = tuple(L[d] / n[d] for d in range(3))
    eps, _ = W.random_fields(n, 21, eps_lo=1.0, eps_hi=10.0)
    rng = np.random.default_rng(4)
    x = rng.normal(size=eps.shape)
    y = rng.normal(size=eps.shape)
    lhs = float(np.sum(S.apply_A6(x, eps, h) * y))
    rhs = float(np.sum(x * S.apply_A6T(y, eps, h)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(S.apply_A6(x, eps, h)).sum())


def _smooth_fields(n, L, seed):
    h, x, y, z = _grid(n, L)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 2 * math.pi, size=6)
    eps = 3.0 + np.cos(2 * math.pi * x / L[0] + a[0]) * np.sin(2 * math.pi * z / L[2] + a[1]) \
        + 0.5 * np.sin(2 * math.pi * y / L[1] + a[2])
    rho = np.exp(-((x - 1.0) ** 2 + (y - 1.2) ** 2 + (z - 1.4) ** 2) / 0.3) \
        - np.exp(-((x - 2.0) ** 2 + (y - 1.0) ** 2 + (z - 2.2) ** 2) / 0.2) + 0.1 * np.cos(a[3] + x)
    return h, eps, rho


def test_adjoint_gradients_match_central_differences():
    n, L = (12, 12, 16), (3.0, 3.0, 4.0)
    h, eps, rho = _smooth_fields(n, L, 8)
    phi = S.solve6(rho, eps, h, tol=1e-13)
    lam = S.adjoint6(rho, eps, h, tol=1e-13)
    g = S.eps_gradient6(phi, lam, h)
    psi = S.charge_potential6(phi, lam, h)
    h3 = h[0] * h[1] * h[2]

    def E(e, r):
        return O.energy(r, S.solve6(r, e, h, tol=1e-13), h)

    flat_e, flat_r = eps.reshape(-1), rho.reshape(-1)
    for q in (5, 700, 1800):
        d = 1e-5
        ep, em = flat_e.copy(), flat_e.copy()
        ep[q] += d
        em[q] -= d
        fd = (E(ep.reshape(eps.shape), rho) - E(em.reshape(eps.shape), rho)) / (2 * d)
        assert abs(fd - g.reshape(-1)[q]) <= 1e-6 * np.abs(g).max(), (q, fd, g.reshape(-1)[q])
        rp, rm = flat_r.copy(), flat_r.copy()
        rp[q] += d
        rm[q] -= d
        fd = (E(eps, rp.reshape(rho.shape)) - E(eps, rm.reshape(rho.shape))) / (2 * d)
        assert abs(fd - h3 * psi.reshape(-1)[q]) <= 1e-6 * h3 * np.abs(psi).max(), (q, fd)
    # for a symmetric operator the adjoint is -h^3 phi / 8 pi; here it is close to it
    assert np.abs(lam + h3 * phi / (8 * math.pi)).max() <= 0.05 * np.abs(lam).max()


def test_forces_with_the_sixth_order_operator():
    # three Gaussian charges with erf switches resolved on the grid (delta = 0.4 A
    # at h = 0.25 A): the non-conservative stencils need a permittivity that the
    # grid resolves (with delta = 0.3 A at h = 0.74 A the system is far from
    # solvable, background c ~ 1)
    n, L = (24, 24, 24), (6.0, 6.0, 6.0)
    h = tuple(L[d] / n[d] for d in range(3))
    xyz = np.array([[2.0, 2.5, 3.0], [4.1, 3.6, 2.7], [3.2, 1.1, 4.6]])
    R = np.array([1.4, 1.2, 1.3])
    q = np.array([1.0, -0.6, -0.4])
    sig = np.array([0.5, 0.45, 0.4])
    p = dict(eps_inf=W.EPS_INF, delta=0.4, exclusion=0, z_lim=0.0, delta_z=0.4)

    def run(x):
        eps = O.eps_erf(n, L, x, R, p)
        rho = O.rho_gauss(n, L, x, q, sig)
        phi = S.solve6(rho, eps, h, tol=1e-13)
        return O.energy(rho, phi, h), eps, rho, phi

    E, eps, rho, phi = run(xyz)
    lam = S.adjoint6(rho, eps, h, tol=1e-13)
    g = S.eps_gradient6(phi, lam, h)
    F = O.forces(n, L, xyz, R, q, sig, p, S.charge_potential6(phi, lam, h), g)
    d = 1e-4
    for a in range(3):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, c] += d
            xm[a, c] -= d
            fd = (run(xp)[0] - run(xm)[0]) / (2 * d)
            assert abs(fd - F[a, c]) <= 1e-6 * np.abs(F).max(), (a, c, fd, F[a, c])
