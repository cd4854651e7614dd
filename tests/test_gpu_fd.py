"""dE/dR at the 128 x 128 x 256 slab against central differences of the
energy, both computed on the GPU through the C ABI.

The forces are the exact derivative of the discrete energy (the grid
permittivity and density are analytic functions of the positions), so central
differences with a 1e-4 A step agree up to O(step^2) and the solve tolerance
(1e-12 relative residual): about 1e-6 of the largest force.  Six atoms drawn
with seed 2 (all in buried layers) plus one top-layer atom, all three
directions, both permittivity modes; in the exclusion mode buried atoms also
carry the height-factor term.
"""
import numpy as np
import pytest

from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("exclusion", [False, True])
def test_forces_match_central_differences(exclusion):
    import torch  # noqa: F401
    from paper_0904_4887_amd.binding import Solver
    w = W.slab((128, 128, 256), tol=1e-12, exclusion=exclusion)
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts())
    rho, phi = s.empty(), s.empty()

    def energy(xyz):
        s.build_epsilon(xyz, w.radius, w.eps_params)
        s.build_rho(xyz, w.q, w.sigma, out=rho)
        _, E, info = s.solve(rho, phi)
        assert info["rel_res"] <= 1e-12
        return E

    energy(w.xyz)
    F = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    step = 1e-4
    # the seeded six, plus the first atom of the top (never buried) layer
    atoms = np.append(W.fd_atoms(len(w.q)), int(np.flatnonzero(~w.buried)[0]))
    fd = np.zeros((len(atoms), 3))
    for n, a in enumerate(atoms):
        for d in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[a, d] += step
            xm[a, d] -= step
            fd[n, d] = (energy(xp) - energy(xm)) / (2 * step)
    s.close()
    err = np.abs(F[atoms] - fd).max()
    assert err <= 1e-5 * np.abs(F).max(), (err, np.abs(F).max(), F[atoms], fd)
    assert w.buried[atoms].any() and (~w.buried[atoms]).any()


@pytest.mark.parametrize("exclusion", [False, True])
def test_gamma_model_forces_match_central_differences(exclusion):
    """The same check for the paper's own permittivity (Eqs. 9, 10, 19).  With
    the exclusion of Eq. 19 the energy jumps where a buried atom's z crosses a
    grid plane, so a z step that would cross one is left out."""
    import torch  # noqa: F401
    from paper_0904_4887_amd.binding import Solver
    w = W.slab_gamma((128, 128, 256), exclusion=exclusion, tol=1e-12, precision=0)
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts())
    rho, phi = s.empty(), s.empty()

    def energy(xyz):
        s.build_epsilon(xyz, w.radius, w.eps_params)
        s.build_rho(xyz, w.q, w.sigma, out=rho)
        _, E, info = s.solve(rho, phi)
        assert info["rel_res"] <= 1e-12
        return E

    energy(w.xyz)
    F = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    step = 1e-4
    hz = w.h[2]
    atoms = np.append(W.fd_atoms(len(w.q)), int(np.flatnonzero(~w.buried)[0]))
    errs = []
    for a in atoms:
        for d in range(3):
            if d == 2 and exclusion and w.buried[a]:
                k = (w.xyz[a, 2] % w.L[2]) / hz
                if abs(k - round(k)) * hz <= 2 * step:
                    continue
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[a, d] += step
            xm[a, d] -= step
            errs.append(abs((energy(xp) - energy(xm)) / (2 * step) - F[a, d]))
    s.close()
    assert len(errs) >= 18
    assert max(errs) <= 1e-5 * np.abs(F).max(), (max(errs), np.abs(F).max())
