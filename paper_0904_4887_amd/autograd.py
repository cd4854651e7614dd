"""torch.autograd wrappers around the library's solve and its adjoint.

DielectricPoisson: (rho, eps) -> (phi, E) for a solver whose grid is set.
  E = 1/2 h^3 sum rho phi (the Hartree energy of Sec. II.C); phi the zero-mean
  solution of A(eps) phi = -4 pi (rho - mean rho).
  Backward (Eq. 11 and App. A-B in discrete form):
    dE/drho = h^3 phi,   dE/deps = -(h^3/8 pi) sum_d 1/2[(D+ phi)^2 + (D- phi)^2]
  (the hand-written adjoint kernel), and for a gradient g_phi flowing into phi
  one adjoint solve A lam = P g_phi (A is symmetric; P removes the mean):
    dL/drho = -4 pi lam,  dL/deps_n = sum_d 1/2[(D+ lam)(D+ phi) + (D- lam)(D- phi)].

SlabEnergy: atom positions -> E for the atom-built permittivity and Gaussian
  charges; backward = dE/dR from the library's force kernel, the permittivity
  gradient chained through the switching functions plus the charge term (with
  the sixth-order operator the library solves the adjoint problem for it).

Every step runs in libdwp; this module only moves tensors and scalars.
"""
from __future__ import annotations

import math

import numpy as np
import torch


class DielectricPoisson(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, eps, solver):
        if solver.opts.order != 2:
            raise ValueError("DielectricPoisson's backward relies on a symmetric operator: use order = 2 "
                             "(the sixth-order operator's gradients come from eps_gradient and forces)")
        solver.set_epsilon(eps.detach().contiguous())
        phi, E, info = solver.solve(rho.detach().contiguous())
        ctx.solver = solver
        ctx.save_for_backward(phi)
        return phi.clone(), torch.tensor(E, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, g_phi, g_E):
        (phi,) = ctx.saved_tensors
        s = ctx.solver
        h3 = float(np.prod(s.h))
        grad_rho = torch.zeros_like(phi)
        grad_eps = torch.zeros_like(phi)
        if g_E is not None:
            ge = float(g_E)
            if ge != 0.0:
                grad_rho += ge * h3 * phi
                grad_eps += ge * s.eps_pair_gradient(phi, phi, -h3 / (8.0 * math.pi))
        if g_phi is not None and bool(torch.any(g_phi != 0)):
            # A lam = P g_phi  <=>  solve with rho' = -g_phi / (4 pi)
            lam, _, _ = s.solve((-g_phi / (4.0 * math.pi)).contiguous())
            grad_rho += -4.0 * math.pi * lam
            grad_eps += s.eps_pair_gradient(lam, phi, 1.0)
        return grad_rho, grad_eps, None


class SlabEnergy(torch.autograd.Function):
    """E(R) for a workload: build eps and rho from the atoms, solve, return E;
    backward returns dE/dR (the negative of the forces)."""

    @staticmethod
    def forward(ctx, xyz, solver, workload):
        w = workload
        x = xyz.detach().cpu().numpy().astype(np.float64)
        solver.build_epsilon(x, w.radius, w.eps_params)
        rho = solver.build_rho(x, w.q, w.sigma)
        phi, E, info = solver.solve(rho)
        ctx.solver, ctx.workload, ctx.x = solver, w, x
        return torch.tensor(E, dtype=torch.float64, device=xyz.device)

    @staticmethod
    def backward(ctx, g_E):
        w = ctx.workload
        dEdR = ctx.solver.forces(ctx.x, w.q, w.sigma, w.radius, w.eps_params)
        g = torch.from_numpy(dEdR).to(dtype=torch.float64, device=g_E.device)
        return g_E * g, None, None


def dielectric_poisson(rho, eps, solver):
    return DielectricPoisson.apply(rho, eps, solver)


def slab_energy(xyz, solver, workload):
    return SlabEnergy.apply(xyz, solver, workload)
