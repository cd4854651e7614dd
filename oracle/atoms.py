"""Permittivity and charge builders of the oracle, and the atomic forces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Permittivity (the product-of-switches dielectric of the slab workloads; it
plays the role of the paper's atom-defined dielectric, Eqs. 9-10):
    eps_n = 1 + (eps_inf - 1) * prod_i s_i(d_in) * H(z_n)
    s_i(d) = 1/2 [1 + erf((d - r_i) / delta)],  d_in the minimum-image distance.
With the exclusion switch on (the smooth analogue of Eq. 19), every atom with
z_i <= z_lim adds a height factor
    h_i(z) = 1/2 [1 + erf((z - z_i) / delta_z)],   H(z) = prod_buried h_i(z),
so that the solvent is pushed out of the region under the buried atoms; z is the
node height in [0, Lz), measured from the bottom of the cell.

Charge: Gaussians of standard deviation sigma_i,
    rho_n = sum_i q_i (2 pi sigma_i^2)^(-3/2) exp(-d_in^2 / (2 sigma_i^2)).

Forces (Eq. 11, derived in App. B), as the exact derivative of the discrete
energy: dE/dR_I = sum_n g_n d eps_n / dR_I + h^3 sum_n phi_n d rho_n / dR_I,
with g = dE/d eps.  No cutoffs are applied here.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_NODE_ATOM_BUDGET = 1 << 22   # nodes x atoms handled per chunk


def _chunk(natoms):
    return max(1024, _NODE_ATOM_BUDGET // max(1, natoms))


def _node_coords(n, L):
    h = [L[d] / n[d] for d in range(3)]
    z, y, x = np.meshgrid(np.arange(n[2]) * h[2], np.arange(n[1]) * h[1],
                          np.arange(n[0]) * h[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)  # (N, 3)


def _min_image(dx, L):
    Lv = np.asarray(L, dtype=np.float64)
    return dx - Lv * np.round(dx / Lv)


def _buried(xyz, params):
    if not params.get("exclusion", 0):
        return np.zeros(len(xyz), dtype=bool)
    return xyz[:, 2] <= params["z_lim"]


def _switch_factors(r, xyz, radius, params, L):
    """s (natoms, m), ds/dd (natoms, m), min-image vectors (natoms, m, 3) and
    distances (natoms, m) for node coordinates r (m, 3)."""
    vec = _min_image(r[None, :, :] - xyz[:, None, :], L)
    d = np.sqrt(np.sum(vec * vec, axis=2))
    delta = params["delta"]
    t = (d - radius[:, None]) / delta
    s = 0.5 * (1.0 + erf(t))
    ds = np.exp(-t * t) / (delta * math.sqrt(math.pi))
    return s, ds, vec, d


def _height_factors(r, xyz, buried, params):
    """h_i(z) (nb, m) and dh_i/dz (nb, m) for the buried atoms."""
    dz = params["delta_z"]
    zb = xyz[buried, 2]
    t = (r[None, :, 2] - zb[:, None]) / dz
    return 0.5 * (1.0 + erf(t)), np.exp(-t * t) / (dz * math.sqrt(math.pi))


def _exclusive_products(f):
    """P[i] = prod_{j != i} f[j] along axis 0, by prefix and suffix products
    (never by division: a factor may be exactly zero)."""
    k = f.shape[0]
    pre = np.ones_like(f)
    suf = np.ones_like(f)
    for i in range(1, k):
        pre[i] = pre[i - 1] * f[i - 1]
    for i in range(k - 2, -1, -1):
        suf[i] = suf[i + 1] * f[i + 1]
    return pre * suf


def eps_erf(n, L, xyz, radius, params, nodes=None):
    """Node permittivity [nz][ny][nx] (or at the flat node indices `nodes`)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    coords = _node_coords(n, L)
    if nodes is not None:
        coords = coords[np.asarray(nodes)]
    buried = _buried(xyz, params)
    out = np.empty(len(coords))
    C = _chunk(len(xyz))
    for c0 in range(0, len(coords), C):
        r = coords[c0:c0 + C]
        s, _, _, _ = _switch_factors(r, xyz, radius, params, L)
        S = np.prod(s, axis=0)
        if buried.any():
            hz, _ = _height_factors(r, xyz, buried, params)
            S = S * np.prod(hz, axis=0)
        out[c0:c0 + C] = 1.0 + (params["eps_inf"] - 1.0) * S
    if nodes is not None:
        return out
    return out.reshape(n[2], n[1], n[0])


def rho_gauss(n, L, xyz, q, sigma, nodes=None):
    """Sum of normalised Gaussians sampled at the nodes."""
    xyz = np.asarray(xyz, dtype=np.float64)
    coords = _node_coords(n, L)
    if nodes is not None:
        coords = coords[np.asarray(nodes)]
    out = np.zeros(len(coords))
    C = _chunk(len(xyz))
    for c0 in range(0, len(coords), C):
        r = coords[c0:c0 + C]
        vec = _min_image(r[None, :, :] - xyz[:, None, :], L)
        d2 = np.sum(vec * vec, axis=2)
        s2 = np.asarray(sigma, dtype=np.float64)[:, None] ** 2
        g = np.asarray(q)[:, None] * (2.0 * math.pi * s2) ** -1.5 * np.exp(-d2 / (2.0 * s2))
        out[c0:c0 + C] = g.sum(axis=0)
    if nodes is not None:
        return out
    return out.reshape(n[2], n[1], n[0])


def forces(n, L, xyz, radius, q, sigma, params, phi, g):
    """dE/dR (natoms, 3): sum_n g_n d eps_n/dR_I + h^3 sum_n phi_n d rho_n/dR_I.

    `params` may be None when the permittivity does not depend on the atoms
    (then only the charge term is returned).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    nat = len(xyz)
    h = [L[d] / n[d] for d in range(3)]
    h3 = h[0] * h[1] * h[2]
    coords = _node_coords(n, L)
    gf = g.ravel() if g is not None else None
    pf = phi.ravel()
    buried = _buried(xyz, params) if params is not None else np.zeros(nat, dtype=bool)
    bidx = np.nonzero(buried)[0]
    acc = np.zeros((nat, 3, 0)).tolist()  # per atom, per component: list of partial sums
    C = _chunk(nat)
    for c0 in range(0, len(coords), C):
        r = coords[c0:c0 + C]
        # charge term: d rho_n / dR_I = q_I G_I(d) (r_n - R_I) / sigma_I^2
        vec = _min_image(r[None, :, :] - xyz[:, None, :], L)
        d2 = np.sum(vec * vec, axis=2)
        s2 = np.asarray(sigma, dtype=np.float64)[:, None] ** 2
        G = np.asarray(q)[:, None] * (2.0 * math.pi * s2) ** -1.5 * np.exp(-d2 / (2.0 * s2))
        wq = h3 * pf[c0:c0 + C][None, :] * G / s2
        part = np.einsum("am,amc->ac", wq, vec)
        if params is not None and gf is not None:
            s, ds, svec, d = _switch_factors(r, xyz, np.asarray(radius, np.float64), params, L)
            if len(bidx):
                hz, dhz = _height_factors(r, xyz, buried, params)
                H = np.prod(hz, axis=0)
            else:
                H = np.ones(len(r))
            others = _exclusive_products(s)                       # prod_{j != I} s_j
            pref = (params["eps_inf"] - 1.0) * gf[c0:c0 + C][None, :] * H[None, :]
            # d d / dR_I = -(r - R_I) / d  (d > 0 wherever ds is not negligible)
            with np.errstate(invalid="ignore", divide="ignore"):
                unit = np.where(d[:, :, None] > 0.0, svec / d[:, :, None], 0.0)
            part -= np.einsum("am,amc->ac", pref * others * ds, unit)
            if len(bidx):
                S = np.prod(s, axis=0)
                hoth = _exclusive_products(hz)                   # prod_{K != I, buried} h_K
                # d h_I / d z_I = -dh_I/dz
                wz = -(params["eps_inf"] - 1.0) * gf[c0:c0 + C][None, :] * S[None, :] \
                    * hoth * dhz
                part[bidx, 2] += wz.sum(axis=1)
        for a in range(nat):
            for c in range(3):
                acc[a][c].append(part[a, c])
    return np.array([[math.fsum(acc[a][c]) for c in range(3)] for a in range(nat)])


def deps_dR_dense(n, L, xyz, radius, params, atom):
    """d eps_n / dR_atom at every node, shape (3, nz, ny, nx) (test helper)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    coords = _node_coords(n, L)
    buried = _buried(xyz, params)
    s, ds, svec, d = _switch_factors(coords, xyz, np.asarray(radius, np.float64), params, L)
    others = _exclusive_products(s)[atom]
    if buried.any():
        hz, dhz = _height_factors(coords, xyz, buried, params)
        H = np.prod(hz, axis=0)
    else:
        H = np.ones(len(coords))
    unit = np.where(d[atom][:, None] > 0, svec[atom] / np.maximum(d[atom][:, None], 1e-300), 0.0)
    out = -(params["eps_inf"] - 1.0) * (others * ds[atom] * H)[:, None] * unit
    if buried[atom]:
        bidx = list(np.nonzero(buried)[0])
        j = bidx.index(atom)
        hoth = _exclusive_products(hz)[j]
        out[:, 2] -= (params["eps_inf"] - 1.0) * np.prod(s, axis=0) * hoth * dhz[j]
    return out.T.reshape(3, n[2], n[1], n[0])


def drho_dR_dense(n, L, xyz, q, sigma, atom):
    """d rho_n / dR_atom at every node, shape (3, nz, ny, nx) (test helper)."""
    coords = _node_coords(n, L)
    vec = _min_image(coords - np.asarray(xyz, np.float64)[atom][None, :], L)
    s2 = float(sigma[atom]) ** 2
    G = q[atom] * (2.0 * math.pi * s2) ** -1.5 * np.exp(-np.sum(vec * vec, axis=1) / (2.0 * s2))
    return (G[:, None] * vec / s2).T.reshape(3, n[2], n[1], n[0])
