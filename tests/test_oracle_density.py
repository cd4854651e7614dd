"""Pins of the oracle's density-dependent dielectric (Eqs. 5-8, Secs. II.C-II.D).

Checked against what the paper and the mathematics fix, never against a
retyped formula: the closed-form values of Eq. 7 at rho = 0, rho_0 and
rho -> infinity and its step limit for large beta; Eq. 8 against central
differences of Eq. 7; V_eps (Eq. 6) against central differences of the
energy with respect to the density that feeds the permittivity; and Eq. 5,
dE/d rho = phi + V_eps, when one density is both the source and the argument
of the permittivity.
"""
import math

import numpy as np

import oracle as O

EPS_INF, RHO0, BETA = 78.36, 2e-3, 1.3


def test_eps_of_density_limits_and_midpoint():
    e = O.eps_of_density(np.array([0.0, RHO0, 1e6 * RHO0, -1.0]), EPS_INF, RHO0, BETA)
    assert e[0] == EPS_INF                         # no density: bulk solvent
    assert abs(e[1] - 0.5 * (1.0 + EPS_INF)) <= 1e-14 * EPS_INF   # the threshold: halfway
    assert abs(e[2] - 1.0) <= 1e-12                # dense region: vacuum
    assert e[3] == EPS_INF                         # negative density read as none
    rho = np.linspace(0.0, 5 * RHO0, 101)
    assert np.all(np.diff(O.eps_of_density(rho, EPS_INF, RHO0, BETA)) < 0)
    # beta -> infinity: a step at rho_0
    step = O.eps_of_density(np.array([0.9 * RHO0, 1.1 * RHO0]), EPS_INF, RHO0, 200.0)
    assert abs(step[0] - EPS_INF) <= 1e-6 and abs(step[1] - 1.0) <= 1e-6


def test_deps_drho_matches_central_differences():
    rho = np.array([0.05, 0.3, 0.9, 1.0, 1.2, 2.0, 4.0]) * RHO0
    d = 1e-7 * RHO0
    fd = (O.eps_of_density(rho + d, EPS_INF, RHO0, BETA) - O.eps_of_density(rho - d, EPS_INF, RHO0, BETA)) / (2 * d)
    an = O.deps_drho(rho, EPS_INF, RHO0, BETA)
    assert np.all(an < 0)
    assert np.abs(an - fd).max() <= 1e-6 * np.abs(an).max()


def _fields(seed=3):
    n, L = (12, 10, 16), (4.0, 3.6, 6.0)
    h = tuple(L[d] / n[d] for d in range(3))
    rng = np.random.default_rng(seed)
    z = (np.arange(n[2]) + 0.5) * h[2]
    # an electron-like density that falls through rho_0 across the box (an
    # interface) with some in-plane texture
    prof = RHO0 * 3.0 * 0.5 * (1.0 + np.tanh((3.0 - z) / 0.6))
    rho_e = prof[:, None, None] * (1.0 + 0.2 * rng.uniform(-1, 1, size=(n[2], n[1], n[0])))
    src = rng.normal(size=(n[2], n[1], n[0]))
    src -= src.mean()
    return n, h, rho_e, src


def _energy(src, rho_e, h):
    eps = O.eps_of_density(rho_e, EPS_INF, RHO0, BETA)
    phi = O.solve(src, eps, h, tol=1e-13, max_iter=1000)
    return O.energy(src, phi, h), phi


def test_v_eps_is_the_energy_derivative_through_the_permittivity():
    n, h, rho_e, src = _fields()
    E0, phi = _energy(src, rho_e, h)
    V = O.v_eps(phi, rho_e, h, EPS_INF, RHO0, BETA)
    h3 = h[0] * h[1] * h[2]
    flat = rho_e.reshape(-1)
    nodes = np.argsort(-np.abs(V).reshape(-1))[:3]     # where V_eps is largest
    for q in nodes:
        d = 1e-4 * flat[q]
        rp, rm = flat.copy(), flat.copy()
        rp[q] += d
        rm[q] -= d
        Ep, _ = _energy(src, rp.reshape(rho_e.shape), h)
        Em, _ = _energy(src, rm.reshape(rho_e.shape), h)
        fd = (Ep - Em) / (2 * d)
        assert abs(fd - h3 * V.reshape(-1)[q]) <= 1e-5 * abs(fd), (q, fd, h3 * V.reshape(-1)[q])


def test_density_derivative_is_phi_plus_v_eps():
    # one density both as the (neutralised) source and as the permittivity's argument (Eq. 5)
    n, h, rho_e, _ = _fields(4)

    def energy(r):
        eps = O.eps_of_density(r, EPS_INF, RHO0, BETA)
        phi = O.solve(r, eps, h, tol=1e-13, max_iter=1000)
        return O.energy(r, phi, h), phi

    E0, phi = energy(rho_e)
    V = O.v_eps(phi, rho_e, h, EPS_INF, RHO0, BETA)
    h3 = h[0] * h[1] * h[2]
    flat = rho_e.reshape(-1)
    nodes = list(np.argsort(-np.abs(V).reshape(-1))[:2]) + [0]
    for q in nodes:
        d = 1e-4 * flat[q] + 1e-12
        rp, rm = flat.copy(), flat.copy()
        rp[q] += d
        rm[q] -= d
        fd = (energy(rp.reshape(rho_e.shape))[0] - energy(rm.reshape(rho_e.shape))[0]) / (2 * d)
        want = h3 * (phi.reshape(-1)[q] + V.reshape(-1)[q])
        assert abs(fd - want) <= 1e-5 * max(abs(want), h3 * np.abs(phi).max()), (q, fd, want)
