"""Seeded synthetic workloads for the dry/wet generalized-Poisson path.

This module only draws inputs: grids, atom positions, charges, radii, the
planar tanh permittivity that the smallest workload hands over directly, and
the solver options each workload is run with.  It holds none of the method's
arithmetic (no permittivity switch, no Gaussian density, no operator), so the
FP64 oracle and the HIP path can both be fed from it without sharing code.

The paper's own systems are DFT slabs (an anatase (101) slab in a continuum
solvent, Sec. II.A); they are replaced here by synthetic stand-ins of the same
kind: a rutile-like TiO2 slab of Gaussian point charges with solvent above it.

Conventions (Sec. II.B-II.F of the paper, made concrete):
  * lengths in Angstrom, charges in e, energies in e^2/Angstrom;
  * node n = (i*hx, j*hy, k*hz) for 0 <= i < nx etc., arrays are [nz][ny][nx];
  * the wet region W is the periodic z-interval [z_wet_lo, z_wet_hi) (hi may
    exceed Lz, in which case W wraps through z = 0).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

EPS_INF = 78.36          # solvent permittivity used by every workload
DELTA = 0.3              # width of the erf switch, Angstrom
R_TI, R_O = 2.0, 1.6     # switch radii, Angstrom
Q_TI, Q_O = 4.0, -2.0    # Gaussian valence charges, e
SIGMA_SLAB = 0.6         # Gaussian width (standard deviation) for slab charges
RUTILE_U = 0.305         # rutile internal parameter


@dataclasses.dataclass
class Workload:
    name: str
    n: tuple              # (nx, ny, nz)
    L: tuple              # (Lx, Ly, Lz), Angstrom
    xyz: np.ndarray       # (natoms, 3) float64, wrapped into [0, L)
    q: np.ndarray         # (natoms,) charges
    sigma: np.ndarray     # (natoms,) Gaussian standard deviations
    radius: np.ndarray    # (natoms,) switch radii (unused when eps is given)
    eps_kind: str         # "tanh_z" (eps handed over as a grid), "erf", "gamma" or "density"
    eps_params: dict      # eps_inf, delta, exclusion (0/1), z_lim, delta_z (gamma: + model 1, beta,
                          # decay; density: eps_inf, rho0, beta)
    z_wet: tuple          # (z_wet_lo, z_wet_hi) Angstrom
    tol: float            # relative residual tolerance of the solve
    precision: int = 0    # 0 = FP64, 1 = mixed FP32-in-FP64
    buried: np.ndarray = None  # (natoms,) bool, atoms under the exclusion rule
    opts: dict = dataclasses.field(default_factory=dict)  # solver options tuned for this input

    def solver_opts(self, **extra):
        """Options for Solver.set_grid: wet slab, tolerance, precision, tuning."""
        o = dict(z_wet_lo=self.z_wet[0], z_wet_hi=self.z_wet[1], tol=self.tol, precision=self.precision)
        o.update(self.opts)
        o.update(extra)
        return o

    @property
    def N(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def h(self):
        return tuple(self.L[d] / self.n[d] for d in range(3))

    def eps_grid(self):
        """Node permittivity for the 'tanh_z' workload (an input, not a builder)."""
        assert self.eps_kind == "tanh_z"
        p = self.eps_params
        nz = self.n[2]
        z = np.arange(nz, dtype=np.float64) * self.h[2]
        prof = 1.0 + (p["eps_inf"] - 1.0) * 0.5 * (1.0 + np.tanh((z - p["z0"]) / p["width"]))
        return np.ascontiguousarray(
            np.broadcast_to(prof[:, None, None], (nz, self.n[1], self.n[0])))


def _rutile_slab(cells_xy, cell_xy, n_layers, z0, layer_dz):
    """Rutile-like TiO2 slab, c axis along z.

    Conventional cell basis (fractional x, y; layer index): Ti at (0,0) and
    (1/2,1/2); O at (u,u), (-u,-u) in the same layer as Ti(0,0) and at
    (1/2+u, 1/2-u), (1/2-u, 1/2+u) in the layer of Ti(1/2,1/2).
    Returns xyz (unwrapped), species code (0 = Ti, 1 = O) and layer index.
    """
    u = RUTILE_U
    basis_even = [(0, 0.0, 0.0), (1, u, u), (1, -u, -u)]
    basis_odd = [(0, 0.5, 0.5), (1, 0.5 + u, 0.5 - u), (1, 0.5 - u, 0.5 + u)]
    xyz, spec, layer = [], [], []
    for lz in range(n_layers):
        basis = basis_even if lz % 2 == 0 else basis_odd
        for cx in range(cells_xy):
            for cy in range(cells_xy):
                for s, fx, fy in basis:
                    xyz.append(((cx + fx) * cell_xy, (cy + fy) * cell_xy, z0 + lz * layer_dz))
                    spec.append(s)
                    layer.append(lz)
    return np.array(xyz, dtype=np.float64), np.array(spec), np.array(layer)


def _slab_workload(name, n, L, cells_xy, layer_dz, seed, z_cut, tol, precision, exclusion):
    cell_xy = L[0] / cells_xy
    xyz, spec, layer = _rutile_slab(cells_xy, cell_xy, 6, 5.0, layer_dz)
    rng = np.random.default_rng(seed)
    xyz = xyz + rng.normal(0.0, 0.05, size=xyz.shape)
    xyz = np.mod(xyz, np.array(L, dtype=np.float64))
    q = np.where(spec == 0, Q_TI, Q_O).astype(np.float64)
    radius = np.where(spec == 0, R_TI, R_O).astype(np.float64)
    sigma = np.full(len(q), SIGMA_SLAB)
    # Exclusion (the smooth analogue of the paper's Eq. 19): atoms of every
    # layer up to the second one from the top are "buried"; z_lim sits half
    # way between the two top layers so that jitter cannot flip the choice.
    z_top2 = 5.0 + 4 * layer_dz
    z_lim = z_top2 + 0.5 * layer_dz
    buried = layer <= 4
    params = dict(eps_inf=EPS_INF, delta=DELTA, exclusion=int(exclusion),
                  z_lim=z_lim, delta_z=DELTA)
    if exclusion:
        # Below the highest buried atom minus 6 switch widths the permittivity
        # is exactly 1; W starts there and wraps two planes past z = 0 so that
        # every dry row of the operator is a vacuum row.
        zmax = float(xyz[buried, 2].max())
        z_wet = (zmax - 6.0 * DELTA, L[2] + 2.0 * L[2] / n[2])
    else:
        z_wet = (z_cut, L[2])
    # With a really dry region the eps^-1/2-scaled dry update needs fewer
    # coupling iterations; with solvent inside the "dry" region it needs more,
    # and there the coupling, not the multigrid, limits the iteration count, so
    # a lighter V(1,1) cycle with a short coarsest solve (4 sweeps) costs no
    # iterations.
    # For the same reason the literal slab's hierarchy halves z from the first
    # coarsening on (semi_ratio 2 > hz / hx = 1.69): half the points on every
    # coarse level for the same 106 iterations at 192 x 192 x 384; the
    # exclusion slab keeps the semi-coarsened first level (there 26 against
    # 32 iterations).
    # FGMRES restart 16: with float32 Krylov vectors the longer cycle's
    # Gram-Schmidt costs less than the iterations it saves (106 against 120
    # on the literal slab at 192 x 192 x 384)
    opts = (dict(scaled_dry=1, restart=16) if exclusion else
            dict(pre=1, post=1, coarse_sweeps=4, restart=16, semi_ratio=2.0))
    return Workload(name=name, n=n, L=L, xyz=xyz, q=q, sigma=sigma, radius=radius,
                    eps_kind="erf", eps_params=params, z_wet=z_wet, tol=tol,
                    precision=precision, buried=buried, opts=opts)


def tanh_box(n=(32, 32, 64), seed=0):
    """10x10x20 A box, planar tanh permittivity, 8 Gaussians of charge +-1.

    Centres are uniform in [0,10) x [0,10) x [0,8) from the seed; charges
    alternate +1, -1; sigma = 0.5 A; dry z < 8 A.
    """
    L = (10.0, 10.0, 20.0)
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, 1.0, size=(8, 3)) * np.array([10.0, 10.0, 8.0])
    q = np.array([1.0, -1.0] * 4)
    return Workload(name=f"tanh_box_{n[0]}x{n[1]}x{n[2]}", n=tuple(n), L=L, xyz=xyz, q=q,
                    sigma=np.full(8, 0.5), radius=np.zeros(8), eps_kind="tanh_z",
                    eps_params=dict(eps_inf=EPS_INF, z0=10.0, width=1.0),
                    z_wet=(8.0, 20.0), tol=1e-10, precision=0,
                    buried=np.zeros(8, dtype=bool))


def slab(n=(96, 96, 192), exclusion=False, tol=1e-10, precision=0, seed=1, name=None):
    """11.8 x 11.8 x 40 A cell, 72-atom rutile-like slab in z in [5, 12] A.

    Six Ti/O layers 1.4 A apart (2x2x3 conventional cells, in-plane edge
    5.9 A), N(0, 0.05 A) jitter, Ti +4 / O -2 Gaussians of sigma 0.6 A,
    switch radii 2.0 / 1.6 A, dry z < 14 A.
    """
    nm = name or f"slab_{n[0]}x{n[1]}x{n[2]}" + ("_excl" if exclusion else "")
    return _slab_workload(nm, tuple(n), (11.8, 11.8, 40.0), 2, 1.4, seed, 14.0, tol,
                          precision, exclusion)


def big_slab(n=(256, 256, 512), exclusion=False, tol=1e-8, precision=1, seed=5):
    """23.6 x 23.6 x 60 A cell, 288 atoms (2x2 lateral replica of the slab),
    six layers stretched to 2.8 A spacing so that they span z in [5, 19] A;
    dry z < 21 A."""
    nm = f"big_slab_{n[0]}x{n[1]}x{n[2]}" + ("_excl" if exclusion else "")
    return _slab_workload(nm, tuple(n), (23.6, 23.6, 60.0), 4, 2.8, seed, 21.0, tol,
                          precision, exclusion)


BOHR = 0.529177210544   # Angstrom: the length unit of the exponent of Eq. 9
BETA_GAMMA = 2.4         # exponent of Eq. 10 used with the paper's solvation tests


def slab_gamma(n=(192, 192, 384), exclusion=False, tol=1e-8, precision=1, z_wet=None):
    """The slab workload with the paper's own atom-defined dielectric.

    Same cell, atoms and charges as slab(); eps_kind "gamma": the dummy density
    of Eq. 9 (van der Waals radii 2.0 A for Ti and 1.6 A for O, exponent in
    bohr) in Eq. 10 with beta = 2.4; with exclusion, Eq. 19 for the atoms of
    every layer up to the second from the top (z_lim half way between the two
    top layers).  Without exclusion the solvent fills the voids of the slab
    and wraps under it; the dry region is z in [4.0, 13.0] A (W wraps from 13 A
    through z = 0).  With exclusion eps is close to 1 below the top buried layer
    and W starts 0.5 A below that layer's lowest atom.
    """
    nm = f"slab_gamma_{n[0]}x{n[1]}x{n[2]}" + ("_excl" if exclusion else "")
    w = slab(n, exclusion=exclusion, tol=tol, precision=precision, seed=1, name=nm)
    p = dict(eps_inf=EPS_INF, model=1, beta=BETA_GAMMA, decay=BOHR, exclusion=int(exclusion),
             z_lim=w.eps_params["z_lim"], delta=DELTA, delta_z=DELTA)
    w.eps_kind = "gamma"
    w.eps_params = p
    if z_wet is not None:
        w.z_wet = tuple(z_wet)
    elif exclusion:
        top_buried = w.xyz[w.buried, 2]
        z4 = top_buried[top_buried > top_buried.max() - 0.7]
        w.z_wet = (float(z4.min()) - 0.5, w.L[2] + 2.0 * w.L[2] / n[2])
    else:
        w.z_wet = (13.0, w.L[2] + 4.0)
    # measured at 192 x 192 x 384, mixed: the eps^-1/2-scaled dry update with the
    # default V(2,2) cycle takes 29 (exclusion) and 39 (literal) coupling
    # iterations against 82 and 93 with the literal slab's V(1,1)
    w.opts = dict(scaled_dry=1)
    return w


RHO0 = 0.0027            # density threshold of Eq. 7, e/A^3 (4e-4 e/bohr^3)
BETA = 1.3               # transition exponent of Eq. 7


def density_slab(n=(192, 192, 384), tol=1e-8, precision=1, seed=7):
    """The slab workload with eps taken from an electron density (Eq. 7).

    Same cell, atoms and charges as slab(); eps_kind "density" with
    eps_inf = 78.36, rho0 = 0.0027 e/A^3, beta = 1.3.  The electron density
    is electron_density(); it is at least 0.35 e/A^3 (so eps - 1 < 3e-4) for
    z in [4.5, 12.5] A, which is the dry region; W wraps from 12.5 A through
    z = 0 to 4.5 A.
    """
    w = slab(n, tol=tol, precision=precision, seed=1, name=f"density_slab_{n[0]}x{n[1]}x{n[2]}")
    w.eps_kind = "density"
    w.eps_params = dict(eps_inf=EPS_INF, rho0=RHO0, beta=BETA, seed=seed)
    w.z_wet = (12.5, w.L[2] + 4.5)
    # measured at 192 x 192 x 384, mixed: 15 coupling iterations with the
    # eps^-1/2-scaled dry update and V(2,2), 73 with the literal slab's V(1,1)
    w.opts = dict(scaled_dry=1)
    return w


def electron_density(w):
    """Synthetic valence density of the density_slab workload, e/A^3.

    A planar slab of height 0.5 e/A^3 on z in [4.5, 12.5] A, corrugated in
    plane by a factor 1 + 0.3 cos(2 pi (x - x0)/a) cos(2 pi (y - y0)/a) with the
    lattice period a = 5.9 A and a seeded phase (x0, y0), decaying as
    exp(-d/0.45 A) at distance d outside the slab; it crosses rho0 about 2.2 A
    from either face, the solid-solvent interfaces where V_eps peaks.
    """
    nx, ny, nz = w.n
    hx, hy, hz = w.h
    rng = np.random.default_rng(w.eps_params["seed"])
    x0, y0 = rng.uniform(0.0, 5.9, size=2)
    x = np.arange(nx) * hx
    y = np.arange(ny) * hy
    z = np.arange(nz) * hz
    d = np.maximum(np.maximum(4.5 - z, z - 12.5), 0.0)
    prof = 0.5 * np.exp(-d / 0.45)
    corr = 1.0 + 0.3 * np.cos(2 * np.pi * (y[:, None] - y0) / 5.9) * np.cos(2 * np.pi * (x[None, :] - x0) / 5.9)
    return prof[:, None, None] * corr[None, :, :]


def md_displacements(natoms, steps, seed=6, scale=0.02):
    """Per-step Gaussian displacements N(0, 0.02 A), applied cumulatively."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(steps, natoms, 3))


def fd_atoms(natoms, seed=2, count=6):
    """Atoms whose forces are checked by central finite differences."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(natoms, size=count, replace=False))


def random_fields(n, seed, eps_lo=1.0, eps_hi=EPS_INF):
    """Random permittivity in [eps_lo, eps_hi] and a random neutral density."""
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    eps = rng.uniform(eps_lo, eps_hi, size=shape)
    rho = rng.normal(size=shape)
    rho -= rho.mean()
    return eps, rho


# The five workloads the solver is specified on.
def configs():
    return {
        "C1": tanh_box(),
        "C2": slab((96, 96, 192), tol=1e-10),
        "C3": slab((128, 128, 256), tol=1e-12),
        "C4": slab((192, 192, 384), tol=1e-8, precision=1),
        "C5": big_slab(),
    }


def wet_planes(n_z, L_z, z_wet):
    """First wet plane ceil(z_lo/hz) and one-past-last plane ceil(z_hi/hz)."""
    hz = L_z / n_z
    k0 = int(math.ceil(z_wet[0] / hz - 1e-9))
    k1 = int(math.ceil(z_wet[1] / hz - 1e-9))
    return k0, k1
