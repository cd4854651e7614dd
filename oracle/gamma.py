"""The paper's atom-defined dielectric (Sec. II.E): the dummy density of
Eq. 9, the permittivity of Eq. 10, the solvent exclusion of Eq. 19 and the
permittivity term of the forces (Eqs. 11-12).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Dummy density (Eq. 9), with the exclusion of Eq. 19 for the buried atoms
(z_I <= z_lim):
    gamma_n = sum_I exp(-s_In (d_In - R_I) / a),
    s_In = +1 for an atom that is not buried, and for a buried atom
    s_In = sign(z_n - z_I) (z measured from the bottom of the cell, in [0, Lz);
    +1 where z_n = z_I),
with d_In the minimum-image distance (one term per atom: under a buried atom
the term grows with distance, so a sum over periodic images would diverge),
R_I the van der Waals radius and a the length unit of the exponent (the paper
works in atomic units: a = 1 bohr).

Permittivity (Eq. 10, the form of Eq. 7 fed with gamma):
    eps_n = 1 + (eps_inf - 1)/2 (1 + (1 - gamma^(2 beta)) / (1 + gamma^(2 beta))).

Its derivative with respect to an atom (the corrected Eq. 12; the printed one
has the opposite sign): with p = gamma^(2 beta),
    d eps_n / dR_I = (d eps / d gamma)_n  d gamma_n / dR_I,
    d eps / d gamma = -(eps_inf - 1) 2 beta gamma^(2 beta - 1) / (1 + p)^2,
    d gamma_n / dR_I = exp(-s_In (d_In - R_I) / a) s_In (r_n - R_I) / (a d_In),
(r_n - R_I the minimum-image vector).  The sign of a buried atom's term is
held fixed: where z_I crosses a grid plane the energy jumps (Eq. 19 is
discontinuous), and the derivative here is that of the smooth pieces.

Forces: dE/dR_I = sum_n g_n d eps_n / dR_I + h^3 sum_n phi_n d rho_n / dR_I
(Eq. 11), the charge term from the Gaussian builder of atoms.py.
"""
from __future__ import annotations

import math

import numpy as np

from .atoms import _chunk, _min_image, _node_coords, forces as _charge_forces

BOHR = 0.529177210544   # Angstrom


def _signs(r, xyz, params, L):
    """s_In (natoms, m) for node coordinates r (m, 3)."""
    nat = len(xyz)
    s = np.ones((nat, len(r)))
    if params.get("exclusion", 0):
        buried = xyz[:, 2] <= params["z_lim"]
        zI = np.mod(xyz[:, 2], L[2])
        below = r[None, :, 2] < zI[:, None]
        s = np.where(buried[:, None] & below, -1.0, 1.0)
    return s


def _terms(r, xyz, rvdw, params, L):
    """exp(-s (d - R) / a), s, min-image vectors and distances for nodes r."""
    vec = _min_image(r[None, :, :] - xyz[:, None, :], L)
    d = np.sqrt(np.sum(vec * vec, axis=2))
    s = _signs(r, xyz, params, L)
    a = params["decay"]
    return np.exp(-s * (d - rvdw[:, None]) / a), s, vec, d


def _eps_of_gamma(gam, eps_inf, beta):
    with np.errstate(over="ignore"):
        p = gam ** (2.0 * beta)
    # (1 - p)/(1 + p) written as 2/(1 + p) - 1, which stays finite when p overflows
    return 1.0 + 0.5 * (eps_inf - 1.0) * (1.0 + (2.0 / (1.0 + p) - 1.0))


def _deps_dgamma(gam, eps_inf, beta):
    with np.errstate(over="ignore"):
        p = gam ** (2.0 * beta)
    q = 1.0 / (1.0 + p)
    # gamma^(2 beta - 1) / (1 + p)^2 = q (1 - q) / gamma
    return -(eps_inf - 1.0) * 2.0 * beta * q * (1.0 - q) / gam


def gamma_density(n, L, xyz, rvdw, params, nodes=None):
    """gamma (Eqs. 9 and 19) at every node [nz][ny][nx] (or at flat `nodes`)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    rvdw = np.asarray(rvdw, dtype=np.float64)
    coords = _node_coords(n, L)
    if nodes is not None:
        coords = coords[np.asarray(nodes)]
    out = np.empty(len(coords))
    C = _chunk(len(xyz))
    for c0 in range(0, len(coords), C):
        e, _, _, _ = _terms(coords[c0:c0 + C], xyz, rvdw, params, L)
        out[c0:c0 + C] = e.sum(axis=0)
    return out if nodes is not None else out.reshape(n[2], n[1], n[0])


def eps_gamma(n, L, xyz, rvdw, params, nodes=None):
    """Node permittivity of Eq. 10 [nz][ny][nx] (or at flat `nodes`)."""
    gam = gamma_density(n, L, xyz, rvdw, params, nodes)
    return _eps_of_gamma(gam, params["eps_inf"], params["beta"])


def deps_gamma_dR_dense(n, L, xyz, rvdw, params, atom):
    """d eps_n / dR_atom at every node, shape (3, nz, ny, nx) (test helper)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    rvdw = np.asarray(rvdw, dtype=np.float64)
    coords = _node_coords(n, L)
    e, s, vec, d = _terms(coords, xyz, rvdw, params, L)
    gam = e.sum(axis=0)
    de = _deps_dgamma(gam, params["eps_inf"], params["beta"])
    da = d[atom]
    unit = np.where(da[:, None] > 0, vec[atom] / np.maximum(da[:, None], 1e-300), 0.0)
    out = (de * e[atom] * s[atom] / params["decay"])[:, None] * unit
    return out.T.reshape(3, n[2], n[1], n[0])


def forces_gamma(n, L, xyz, rvdw, q, sigma, params, phi, g):
    """dE/dR (natoms, 3) for the Eq. 10 permittivity: the permittivity term
    sum_n g_n d eps_n/dR_I plus the charge term h^3 sum_n phi_n d rho_n/dR_I."""
    xyz = np.asarray(xyz, dtype=np.float64)
    rvdw = np.asarray(rvdw, dtype=np.float64)
    nat = len(xyz)
    coords = _node_coords(n, L)
    gf = g.ravel()
    acc = [[[] for _ in range(3)] for _ in range(nat)]
    C = _chunk(nat)
    a = params["decay"]
    for c0 in range(0, len(coords), C):
        r = coords[c0:c0 + C]
        e, s, vec, d = _terms(r, xyz, rvdw, params, L)
        gam = e.sum(axis=0)
        de = _deps_dgamma(gam, params["eps_inf"], params["beta"])
        with np.errstate(invalid="ignore", divide="ignore"):
            unit = np.where(d[:, :, None] > 0.0, vec / d[:, :, None], 0.0)
        w = (gf[c0:c0 + C] * de)[None, :] * e * s / a
        part = np.einsum("am,amc->ac", w, unit)
        for i in range(nat):
            for c in range(3):
                acc[i][c].append(part[i, c])
    F = np.array([[math.fsum(acc[i][c]) for c in range(3)] for i in range(nat)])
    return F + _charge_forces(n, L, xyz, None, q, sigma, None, phi, None)
