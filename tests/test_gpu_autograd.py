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


def test_backward_uses_the_forward_pass_state(torch):
    """Two forward passes on one solver, then the backward of the first: the
    gradients are those of the first pass's permittivity, not of whatever the
    solver holds when backward runs; warm_start on the solver does not make a
    new solve read an uninitialised initial guess."""
    from paper_0904_4887_amd.autograd import dielectric_poisson
    n, L = (16, 16, 32), (6.0, 6.0, 12.0)
    eps1, rho1 = W.random_fields(n, 51, eps_hi=20.0)
    eps2, rho2 = W.random_fields(n, 52, eps_hi=40.0)
    wts = np.random.default_rng(53).normal(size=eps1.shape)
    s = _solver(n, L, z_wet_lo=4.0, z_wet_hi=12.0, tol=1e-12, warm_start=1)
    r1 = torch.tensor(rho1, device="cuda", requires_grad=True)
    e1 = torch.tensor(eps1, device="cuda", requires_grad=True)
    phi1, E1 = dielectric_poisson(r1, e1, s)
    r2 = torch.tensor(rho2, device="cuda", requires_grad=True)
    e2 = torch.tensor(eps2, device="cuda", requires_grad=True)
    phi2, E2 = dielectric_poisson(r2, e2, s)
    s.set_opts(tol=1e-3)  # a later change of options must not leak into the first backward
    loss = E1 + (torch.tensor(wts, device="cuda") * phi1).sum()
    loss.backward()
    h = s.h
    h3 = float(np.prod(h))
    phi_o = O.solve(rho1, eps1, h, tol=1e-13)
    assert abs(E1.item() - O.energy(rho1, phi_o, h)) <= 1e-10 * abs(E1.item())
    assert abs(E2.item() - O.energy(rho2, O.solve(rho2, eps2, h, tol=1e-13), h)) <= 1e-10 * abs(E2.item())
    # the adjoint: A lam = w - mean(w), zero mean (A symmetric)
    lam_o = O.solve(-wts / (4.0 * math.pi), eps1, h, tol=1e-13)
    gr_o = h3 * phi_o - 4.0 * math.pi * lam_o
    gr = r1.grad.cpu().numpy()
    assert np.abs(gr - gr_o).max() <= 1e-9 * np.abs(gr_o).max()
    # dL/d eps_n = dE/d eps_n + sum_d 1/2 [(D+ lam)(D+ phi) + (D- lam)(D- phi)]_n, by
    # central differences of the oracle's loss in three node permittivities
    ge = e1.grad.cpu().numpy()

    def Lval(e):
        p = O.solve(rho1, e, h, tol=1e-13, max_iter=1500)
        return O.energy(rho1, p, h) + float(np.sum(wts * p))

    for node in [(3, 5, 7), (20, 2, 11), (31, 15, 0)]:
        d = 1e-3 * eps1[node]
        ep, em = eps1.copy(), eps1.copy()
        ep[node] += d
        em[node] -= d
        fd = (Lval(ep) - Lval(em)) / (2 * d)
        assert abs(fd - ge[node]) <= 1e-5 * np.abs(ge).max(), (node, fd, ge[node])
    s.close()


def test_library_backward_leaves_the_last_solution(torch):
    """dwp_backward runs its adjoint solve on buffers of its own: the
    permittivity gradient of the last solve is unchanged by it."""
    n, L = (16, 16, 32), (6.0, 6.0, 12.0)
    eps_np, rho_np = W.random_fields(n, 61, eps_hi=20.0)
    s = _solver(n, L, z_wet_lo=4.0, z_wet_hi=12.0, tol=1e-12)
    s.set_epsilon(torch.tensor(eps_np, device="cuda"))
    phi, E, _ = s.solve(torch.tensor(rho_np, device="cuda"))
    g0 = s.eps_gradient().cpu().numpy()
    g_phi = torch.tensor(np.random.default_rng(62).normal(size=eps_np.shape), device="cuda")
    gr, ge, info = s.backward(phi, 1.0, g_phi)
    assert info["outer_iters"] > 0 and info["rel_res"] <= 1e-12
    assert info["t_fft_ms"] > 0 and info["t_mg_ms"] > 0 and info["t_krylov_ms"] > 0
    g1 = s.eps_gradient().cpu().numpy()
    assert np.array_equal(g0, g1)
    # g_E alone (no g_phi): the energy gradients of the hand-written adjoint
    gr, ge, info = s.backward(phi, 2.0, None)
    h3 = float(np.prod(s.h))
    assert np.abs(gr.cpu().numpy() - 2.0 * h3 * phi.cpu().numpy()).max() <= 1e-15 * np.abs(gr.cpu().numpy()).max() + 1e-300
    assert np.abs(ge.cpu().numpy() - 2.0 * g0).max() <= 1e-13 * np.abs(g0).max()
    assert info["outer_iters"] == 0
    s.close()
