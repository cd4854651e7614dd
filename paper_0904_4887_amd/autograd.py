"""torch.autograd wrappers around the library's solve and its adjoint.

DielectricPoisson: (rho, eps) -> (phi, E) for a solver whose grid is set.
  E = 1/2 h^3 sum rho phi (the Hartree energy of Sec. II.C); phi the zero-mean
  solution of A(eps) phi = -4 pi (rho - mean rho).
  Backward (Eq. 11 and App. A-B in discrete form) is one library call,
  dwp_backward: dE/drho = h^3 phi, dE/deps from the hand-written adjoint
  kernel, and for a gradient g_phi flowing into phi one adjoint solve
  A lam = P g_phi (A is symmetric; P removes the mean) with
  dL/drho = -4 pi lam and dL/deps from the face-product kernel.  The forward
  pass's permittivity, options and phi are kept, so a later forward call or
  set_epsilon on the same solver does not change the gradients.

SlabEnergy: atom positions -> E for the atom-built permittivity and Gaussian
  charges; backward = dE/dR from the library's force kernel, the permittivity
  gradient chained through the switching functions plus the charge term (with
  the sixth-order operator the library solves the adjoint problem for it).

Every step runs in libdwp; this module only moves tensors and scalars.
"""
from __future__ import annotations

import numpy as np
import torch


class DielectricPoisson(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, eps, solver):
        if solver.opts.order != 2:
            raise ValueError("DielectricPoisson's backward relies on a symmetric operator: use order = 2 "
                             "(the sixth-order operator's gradients come from eps_gradient and forces)")
        eps_c = eps.detach().contiguous()
        solver.set_epsilon(eps_c)
        phi, E, info = solver.solve(rho.detach().contiguous())
        ctx.solver = solver
        ctx.epoch = solver.epoch
        ctx.opts = bytes(solver.opts)
        ctx.save_for_backward(phi, eps_c)
        return phi.clone(), torch.tensor(E, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, g_phi, g_E):
        phi, eps = ctx.saved_tensors
        s = ctx.solver
        if s.epoch != ctx.epoch or bytes(s.opts) != ctx.opts:
            # the solver was used for something else since the forward pass:
            # restore the forward's options and permittivity
            saved = type(s.opts).from_buffer_copy(ctx.opts)
            s.set_opts(**{k: getattr(saved, k) for k, _ in saved._fields_})
            s.set_epsilon(eps)
            ctx.epoch = s.epoch
        ge = 0.0 if g_E is None else float(g_E)
        if g_phi is not None and not bool(torch.any(g_phi != 0)):
            g_phi = None
        if g_phi is not None:
            g_phi = g_phi.detach().to(torch.float64).contiguous()
        grad_rho, grad_eps, _ = s.backward(phi, ge, g_phi)
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
