"""The paper's atom-defined dielectric on the GPU (Secs. II.E-II.F: Eqs. 9, 10, 12, 19),
through the C ABI (dwp_eps_params.model = 1).

* eps against the oracle node by node (both exclusion modes, a ragged grid,
  atoms across the periodic boundary), and at sampled nodes of the full
  192 x 192 x 384 grid;
* the solve, dE/d eps and dE/dR against the oracle's own solution, and the
  force kernels alone against the oracle's forces of the device's phi;
* argument and state errors.

Tolerance of eps: the device evaluates gamma^(2 beta) as exp(2 beta log gamma)
and Eq. 10 in its simplified form, the oracle as a power and in the printed
form; with |2 beta log gamma| up to ~300 the rounding of the exponent is up to
~3e-13 relative in gamma^(2 beta), i.e. up to (eps_inf - 1)/4 * 3e-13 ~ 6e-12
in eps.
"""
import numpy as np
import pytest

import oracle as O
from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS_TOL = 1e-11


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _solver(w, **extra):
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts(**extra))
    return s


@pytest.mark.parametrize("n,exclusion", [((48, 48, 128), False), ((48, 48, 128), True), ((36, 24, 96), True)])
def test_eps_matches_oracle(torch, n, exclusion):
    w = W.slab_gamma(n, exclusion=exclusion, precision=0)
    s = _solver(w)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    eps = s.get_epsilon().cpu().numpy()
    ref = O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params)
    assert np.abs(eps - ref).max() <= EPS_TOL
    assert eps.min() >= 1.0
    s.close()


def test_eps_with_atoms_across_the_boundary(torch):
    n, L = (24, 24, 48), (6.0, 6.0, 12.0)
    xyz = np.array([[0.02, 5.97, 0.01], [5.99, 0.03, 11.98], [3.0, 3.0, 6.0], [1.5, 4.4, 2.2]])
    R = np.array([1.6, 2.0, 1.6, 1.8])
    p = dict(eps_inf=W.EPS_INF, model=1, beta=2.4, decay=W.BOHR, exclusion=1, z_lim=3.0)
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(n, L, z_wet_lo=4.0, z_wet_hi=12.0)
    s.build_epsilon(xyz, R, p)
    eps = s.get_epsilon().cpu().numpy()
    ref = O.eps_gamma(n, L, np.mod(xyz, L), R, p)
    assert np.abs(eps - ref).max() <= EPS_TOL
    s.close()


def test_eps_full_size_sampled(torch):
    w = W.slab_gamma((192, 192, 384), exclusion=True)
    s = _solver(w)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rng = np.random.default_rng(7)
    nodes = np.sort(rng.choice(w.N, size=4096, replace=False))
    eps = s.get_epsilon().reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy()
    ref = O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params, nodes=nodes)
    assert np.abs(eps - ref).max() <= EPS_TOL
    s.close()


@pytest.mark.parametrize("exclusion", [False, True])
def test_solve_gradient_and_forces_match_oracle(torch, exclusion):
    w = W.slab_gamma((48, 48, 128), exclusion=exclusion, tol=1e-11, precision=0)
    s = _solver(w)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho = s.build_rho(w.xyz, w.q, w.sigma)
    phi, E, info = s.solve(rho)
    assert info["rel_res"] <= w.tol
    F = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    ph = phi.cpu().numpy()
    # the force kernels alone: the oracle's forces of the device's phi
    F_same = O.forces_gamma(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, ph, O.eps_gradient(ph, w.h))
    assert np.abs(F - F_same).max() <= 1e-10 * np.abs(F_same).max()
    # the whole path against the oracle's own solution
    eps = O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho_o = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    ref = O.solve(rho_o, eps, w.h, tol=1e-13, max_iter=1000)
    assert np.abs(ph - ref).max() <= 1e-8 * np.abs(ref).max()
    assert abs(E - O.energy(rho_o, ref, w.h)) <= 1e-10 * abs(E)
    g = s.eps_gradient().cpu().numpy()
    g_ref = O.eps_gradient(ref, w.h)
    assert np.abs(g - g_ref).max() <= 1e-7 * np.abs(g_ref).max()
    F_ref = O.forces_gamma(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, ref, g_ref)
    assert np.abs(F - F_ref).max() <= 1e-7 * np.abs(F_ref).max()
    s.close()


def test_mixed_precision_solve_matches_oracle(torch):
    w = W.slab_gamma((48, 48, 128), exclusion=True, tol=1e-9, precision=1)
    s = _solver(w)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho = s.build_rho(w.xyz, w.q, w.sigma)
    phi, E, info = s.solve(rho)
    eps = O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho_o = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    ref = O.solve(rho_o, eps, w.h, tol=1e-13, max_iter=1000)
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref).max()
    assert abs(E - O.energy(rho_o, ref, w.h)) <= 1e-8 * abs(E)
    s.close()


def test_gamma_model_errors(torch):
    from paper_0904_4887_amd.binding import DWPError, DWP_EINVAL, DWP_ESTATE
    w = W.slab_gamma((16, 16, 32), exclusion=True, precision=0)
    s = _solver(w)
    for bad in (dict(model=2), dict(beta=0.5), dict(beta=101.0), dict(decay=0.0), dict(decay=float("nan"))):
        with pytest.raises(DWPError) as e:
            s.build_epsilon(w.xyz, w.radius, dict(w.eps_params, **bad))
        assert e.value.status == DWP_EINVAL, bad
    with pytest.raises(DWPError) as e:        # 600 decay lengths at most across the half-diagonal
        s.build_epsilon(w.xyz, w.radius, dict(w.eps_params, decay=0.03))
    assert e.value.status == DWP_EINVAL
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    s.solve(s.build_rho(w.xyz, w.q, w.sigma))
    with pytest.raises(DWPError) as e:        # forces with the other model than the build
        s.forces(w.xyz, w.q, w.sigma, w.radius, dict(w.eps_params, model=0))
    assert e.value.status == DWP_ESTATE
    with pytest.raises(DWPError) as e:        # or another beta
        s.forces(w.xyz, w.q, w.sigma, w.radius, dict(w.eps_params, beta=2.0))
    assert e.value.status == DWP_ESTATE
    s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    s.close()


@pytest.mark.parametrize("exclusion", [0, 1])
def test_atom_on_a_node(torch, exclusion):
    # an atom exactly on a grid node (d = 0 there: that node adds no force) next
    # to one off the grid; with exclusion the first is buried
    n, L = (16, 16, 24), (6.0, 6.0, 9.0)
    h = (L[0] / n[0], L[1] / n[1], L[2] / n[2])
    xyz = np.array([[5 * h[0], 7 * h[1], 10 * h[2]], [3.9, 3.1, 5.3]])
    R, q, sig = np.array([1.6, 1.4]), np.array([1.0, -1.0]), np.array([0.3, 0.3])
    p = dict(eps_inf=W.EPS_INF, model=1, beta=2.4, decay=W.BOHR, exclusion=exclusion, z_lim=5.0)
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(n, L, z_wet_lo=0.5, z_wet_hi=8.5, tol=1e-11, scaled_dry=1)
    s.build_epsilon(xyz, R, p)
    eps = s.get_epsilon().cpu().numpy()
    assert np.abs(eps - O.eps_gamma(n, L, xyz, R, p)).max() <= EPS_TOL
    phi, E, info = s.solve(s.build_rho(xyz, q, sig))
    F = s.forces(xyz, q, sig, R, p)
    ph = phi.cpu().numpy()
    F_same = O.forces_gamma(n, L, xyz, R, q, sig, p, ph, O.eps_gradient(ph, s.h))
    assert np.abs(F - F_same).max() <= 1e-10 * np.abs(F_same).max()
    s.close()
