"""Gradients through torch.autograd: the hand-written adjoint against the
oracle's gradient and against central finite differences of the oracle."""
import math

import numpy as np
import pytest

import oracle as O
from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _solver(n, L, **opts):
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(n, L, **opts)
    return s


def test_energy_gradients_wrt_rho_and_eps(torch):
    from paper_0904_4887_amd.autograd import dielectric_poisson
    n, L = (16, 16, 32), (6.0, 6.0, 12.0)
    eps_np, rho_np = W.random_fields(n, 41, eps_hi=20.0)
    s = _solver(n, L, z_wet_lo=4.0, z_wet_hi=12.0, tol=1e-12)
    rho = torch.tensor(rho_np, device="cuda", requires_grad=True)
    eps = torch.tensor(eps_np, device="cuda", requires_grad=True)
    phi, E = dielectric_poisson(rho, eps, s)
    E.backward()
    h = s.h
    phi_o = O.solve(rho_np, eps_np, h, tol=1e-13)
    assert abs(E.item() - O.energy(rho_np, phi_o, h)) <= 1e-10 * abs(E.item())
    h3 = float(np.prod(h))
    gr = rho.grad.cpu().numpy()
    assert np.abs(gr - h3 * phi_o).max() <= 1e-9 * np.abs(h3 * phi_o).max()
    ge = eps.grad.cpu().numpy()
    ge_o = O.eps_gradient(phi_o, h)
    assert np.abs(ge - ge_o).max() <= 1e-9 * np.abs(ge_o).max()


def test_gradient_through_phi_matches_finite_differences(torch):
    """L = sum w * phi: needs the adjoint solve and the face-product kernel."""
    from paper_0904_4887_amd.autograd import dielectric_poisson
    n, L = (16, 16, 32), (6.0, 6.0, 12.0)
    eps_np, rho_np = W.random_fields(n, 43, eps_hi=20.0)
    wts = np.random.default_rng(44).normal(size=eps_np.shape)
    s = _solver(n, L, z_wet_lo=4.0, z_wet_hi=12.0, tol=1e-12)
    rho = torch.tensor(rho_np, device="cuda", requires_grad=True)
    eps = torch.tensor(eps_np, device="cuda", requires_grad=True)
    phi, E = dielectric_poisson(rho, eps, s)
    loss = (torch.tensor(wts, device="cuda") * phi).sum()
    loss.backward()
    gr, ge = rho.grad.cpu().numpy(), eps.grad.cpu().numpy()
    h = s.h

    def Lval(r, e):
        return float(np.sum(wts * O.solve(r, e, h, tol=1e-13, max_iter=1500)))

    for node in [(3, 5, 7), (20, 2, 11), (31, 15, 0)]:
        d = 1e-3 * eps_np[node]
        ep, em = eps_np.copy(), eps_np.copy()
        ep[node] += d
        em[node] -= d
        fd = (Lval(rho_np, ep) - Lval(rho_np, em)) / (2 * d)
        assert abs(fd - ge[node]) <= 1e-5 * np.abs(ge).max(), (node, fd, ge[node])
        rp, rm = rho_np.copy(), rho_np.copy()
        rp[node] += 1e-3
        rm[node] -= 1e-3
        fd = (Lval(rp, eps_np) - Lval(rm, eps_np)) / 2e-3
        assert abs(fd - gr[node]) <= 1e-6 * np.abs(gr).max(), (node, fd, gr[node])


@pytest.mark.parametrize("exclusion", [False, True])
def test_slab_energy_backward_is_the_oracle_force(torch, exclusion):
    from paper_0904_4887_amd.autograd import slab_energy
    w = W.slab(n=(48, 48, 96), exclusion=exclusion)
    s = _solver(w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-12)
    xyz = torch.tensor(w.xyz, device="cuda", requires_grad=True)
    E = slab_energy(xyz, s, w)
    E.backward()
    eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    phi = O.solve(rho, eps, s.h, tol=1e-13)
    F_o = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi, O.eps_gradient(phi, s.h))
    g = xyz.grad.cpu().numpy()
    assert np.abs(g - F_o).max() <= 1e-8 * np.abs(F_o).max()
