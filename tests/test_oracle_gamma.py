"""Pins of the oracle's atom-defined dielectric (Secs. II.E-II.F: Eqs. 9, 10, 12, 19).

Against what the mathematics fixes, not a retyped formula:
* one atom: Eq. 10 with Eq. 9 is a logistic function of the distance,
  1 + (eps_inf - 1) expit(2 beta (d - R)/a), whose midpoint (1 + eps_inf)/2 sits
  at the van der Waals radius (Fig. 3's transition) and whose width shrinks as
  1/beta;
* Eq. 19: under a buried atom the logistic is mirrored, so eps tends to 1
  away from it; above it (and for atoms that are not buried) nothing changes;
* gamma adds up over atoms, and the whole field moves with the atoms (a shift
  by one node in x or y rolls it);
* d eps/dR against central differences of eps, and its sign: moving an atom
  towards a node lowers eps there (the printed Eq. 12 has the other sign);
* forces against central differences of the oracle energy, both modes.
"""
import math

import numpy as np
import pytest
from scipy.special import expit

import oracle as O
from paper_0904_4887_amd import workloads as W

BETA, A, EPS = 2.4, W.BOHR, W.EPS_INF


def _params(exclusion=0, z_lim=0.0, beta=BETA):
    return dict(eps_inf=EPS, model=1, beta=beta, decay=A, exclusion=exclusion, z_lim=z_lim)


def _one_atom(beta=BETA, exclusion=0, R=1.6):
    n, L = (40, 40, 40), (16.0, 16.0, 16.0)
    xyz = np.array([[8.0, 8.0, 8.0]])
    e = O.eps_gamma(n, L, xyz, [R], _params(exclusion, 9.0, beta))
    h = L[0] / n[0]
    c = np.arange(n[0]) * h - 8.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return e, np.sqrt(x * x + y * y + z * z), z


def test_single_atom_is_a_logistic_of_distance():
    e, d, _ = _one_atom()
    ref = 1.0 + (EPS - 1.0) * expit(2.0 * BETA * (d - 1.6) / A)
    assert np.abs(e - ref).max() <= 1e-12 * EPS
    # the transition is centred at the van der Waals radius
    e_mid = O.eps_gamma((8, 8, 8), (16.0, 16.0, 16.0), np.array([[1.6, 0.0, 0.0]]), [1.6], _params())[0, 0, 0]
    assert abs(e_mid - 0.5 * (1.0 + EPS)) <= 1e-12 * EPS


def test_transition_width_shrinks_as_one_over_beta():
    widths = []
    for beta in (1.2, 2.4, 4.8):
        n, L = (60000, 2, 2), (60.0, 1.0, 1.0)
        nodes = np.arange(0, 6001)          # x in [0, 6] A on a 1 mA grid
        e = O.eps_gamma(n, L, np.zeros((1, 3)), [2.0], _params(beta=beta), nodes=nodes)
        x = nodes * 1e-3
        lo = x[np.argmax(e > 1.0 + 0.1 * (EPS - 1.0))]
        hi = x[np.argmax(e > 1.0 + 0.9 * (EPS - 1.0))]
        widths.append(hi - lo)
        assert np.all(np.diff(e) >= 0.0)
    # 10%-90% width of a logistic in 2 beta d / a is a ln(81) / (2 beta)
    for beta, wd in zip((1.2, 2.4, 4.8), widths):
        assert abs(wd - A * math.log(81.0) / (2.0 * beta)) <= 2e-3


def test_exclusion_mirrors_the_logistic_under_a_buried_atom():
    e, d, z = _one_atom(exclusion=1)
    below = z < 0.0
    up = 1.0 + (EPS - 1.0) * expit(2.0 * BETA * (d - 1.6) / A)
    down = 1.0 + (EPS - 1.0) * expit(-2.0 * BETA * (d - 1.6) / A)
    assert np.abs(e[~below] - up[~below]).max() <= 1e-12 * EPS
    assert np.abs(e[below] - down[below]).max() <= 1e-12 * EPS
    # far below the atom the region is dry
    assert np.all(e[below & (d > 6.0)] - 1.0 <= 1e-12)
    # an atom above z_lim is not buried: no change
    n, L = (40, 40, 40), (16.0, 16.0, 16.0)
    e3 = O.eps_gamma(n, L, np.array([[8.0, 8.0, 8.0]]), [1.6], _params(1, 7.9))
    e0, _, _ = _one_atom()
    assert np.array_equal(e3, e0)


def test_gamma_adds_over_atoms_and_moves_with_them():
    n, L = (24, 20, 32), (7.2, 6.0, 9.6)
    rng = np.random.default_rng(5)
    xyz = rng.uniform(0, 1, size=(5, 3)) * np.array(L)
    R = rng.uniform(1.4, 2.1, size=5)
    p = _params()
    g_all = O.gamma_density(n, L, xyz, R, p)
    g_sum = sum(O.gamma_density(n, L, xyz[i:i + 1], R[i:i + 1], p) for i in range(5))
    assert np.abs(g_all - g_sum).max() <= 1e-13 * np.abs(g_all).max()
    hx = L[0] / n[0]
    shifted = xyz + np.array([hx, 0.0, 0.0])
    e0 = O.eps_gamma(n, L, xyz, R, p)
    e1 = O.eps_gamma(n, L, shifted, R, p)
    assert np.abs(np.roll(e0, 1, axis=2) - e1).max() <= 1e-12 * EPS
    hy = L[1] / n[1]
    e2 = O.eps_gamma(n, L, xyz + np.array([0.0, 3 * hy, 0.0]), R, p)
    assert np.abs(np.roll(e0, 3, axis=1) - e2).max() <= 1e-12 * EPS


@pytest.mark.parametrize("exclusion", [0, 1])
def test_eps_derivative_matches_central_differences_and_has_the_corrected_sign(exclusion):
    n, L = (16, 16, 24), (6.0, 6.0, 9.0)
    xyz = np.array([[2.0, 3.1, 4.05], [4.3, 2.2, 5.6], [3.05, 4.4, 3.3]])   # none at L/2 from a node
    R = np.array([1.6, 2.0, 1.6])
    p = _params(exclusion, 4.5)
    d = 1e-5
    for atom in range(3):
        an = O.deps_gamma_dR_dense(n, L, xyz, R, p, atom)
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[atom, c] += d
            xm[atom, c] -= d
            fd = (O.eps_gamma(n, L, xp, R, p) - O.eps_gamma(n, L, xm, R, p)) / (2 * d)
            assert np.abs(fd - an[c]).max() <= 1e-6 * np.abs(an[c]).max() + 1e-9
    # moving the first atom along +x lowers eps at a node in front of it
    an = O.deps_gamma_dR_dense(n, L, xyz, R, _params(), 0)
    node = (int(round(4.05 / (9.0 / 24))), int(round(3.1 / (6.0 / 16))), int(round(3.9 / (6.0 / 16))))
    assert an[0][node] < 0.0


def _energy(w, xyz, tol=1e-12):
    p = w.eps_params
    eps = O.eps_gamma(w.n, w.L, xyz, w.radius, p)
    rho = O.rho_gauss(w.n, w.L, xyz, w.q, w.sigma)
    phi = O.solve(rho, eps, w.h, tol=tol, max_iter=1000)
    return O.energy(rho, phi, w.h), eps, rho, phi


@pytest.mark.parametrize("exclusion", [False, True])
def test_forces_match_finite_differences(exclusion):
    w = W.slab_gamma((24, 24, 64), exclusion=exclusion, precision=0)
    E, eps, rho, phi = _energy(w, w.xyz)
    g = O.eps_gradient(phi, w.h)
    F = O.forces_gamma(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi, g)
    d = 1e-4
    scale = np.abs(F).max()
    hz = w.h[2]
    checked = 0
    for a in (3, 40, 70):   # a bottom-layer (buried) atom, a middle one, a top one
        for c in range(3):
            if c == 2 and w.buried[a]:
                # Eq. 19 jumps where z_a crosses a grid plane: keep the step inside one cell
                k = (w.xyz[a, 2] % w.L[2]) / hz
                if abs(k - round(k)) * hz <= 2 * d:
                    continue
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[a, c] += d
            xm[a, c] -= d
            fd = (_energy(w, xp)[0] - _energy(w, xm)[0]) / (2 * d)
            assert abs(fd - F[a, c]) <= 2e-6 * scale, (a, c, fd, F[a, c])
            checked += 1
    assert checked >= 8
