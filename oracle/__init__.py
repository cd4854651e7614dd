"""FP64 CPU oracle for the dry/wet generalized-Poisson path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library or its binding;
both sides take their inputs from the seeded generators, which hold none of the
method's arithmetic.

What it computes (paper, Sec. II.B-II.F and Appendix B):
  * the 7-point conservative discretisation of div(eps grad phi) (Eq. 3);
  * the periodic vacuum Poisson solve by FFT with the discrete 7-point symbol
    (the discrete counterpart of Eq. 15);
  * the unique zero-mean solution of A phi = -4 pi (rho - mean rho) on the full
    periodic box, by conjugate gradients preconditioned with that FFT solve
    (a different algorithm from the GPU's dry/wet coupling, on purpose);
  * the Hartree energy 1/2 int phi rho and its permittivity form (Eq. 4);
  * dE/d eps at every node and dE/dR for every atom (Eq. 11, App. B) through
    the product-of-erf switches and the Gaussian charges;
  * the paper's one-pass split (vacuum FFT, then a Dirichlet solve in the wet
    slab with the vacuum potential as boundary data, Sec. II.F) as a
    diagnostic;
  * the density-dependent permittivity (Eq. 7), its derivative (Eq. 8) and the
    potential term V_eps (Eq. 6) of Secs. II.C-II.D;
  * the paper's atom-defined permittivity: dummy density (Eq. 9), Eq. 10, the
    solvent exclusion of Eq. 19, and its force term (Eqs. 11-12, with the sign
    that differentiating Eqs. 9-10 gives);
  * the paper's sixth-order non-conservative operator (Eqs. 16-18), its solve
    (GMRES preconditioned with the second-order solve), the adjoint solve and
    the energy gradients that need it.

Every pin of these functions lives in the CPU test-suite.  Parity unpinned:
none of the functions above (the one-pass split is pinned only by its epsilon
= 1 special case, where it reduces to the vacuum solve).
"""
from .poisson import (apply_A, vacuum_symbol, vacuum_solve, solve, energy,
                      energy_eps_form, eps_gradient, residual_norm)
from .atoms import eps_erf, rho_gauss, forces, deps_dR_dense, drho_dR_dense
from .split import one_pass_split
from .density import eps_of_density, deps_drho, v_eps
from .gamma import gamma_density, eps_gamma, deps_gamma_dR_dense, forces_gamma
from .sixth import (apply_A6, apply_A6T, symbol6, vacuum_solve6, solve6, residual_norm6, adjoint6,
                    eps_gradient6, charge_potential6)

__all__ = ["apply_A", "vacuum_symbol", "vacuum_solve", "solve", "energy",
           "energy_eps_form", "eps_gradient", "residual_norm", "eps_erf",
           "rho_gauss", "forces", "deps_dR_dense", "drho_dR_dense", "one_pass_split",
           "eps_of_density", "deps_drho", "v_eps", "gamma_density", "eps_gamma",
           "deps_gamma_dR_dense", "forces_gamma", "apply_A6", "apply_A6T", "symbol6", "vacuum_solve6",
           "solve6", "residual_norm6", "adjoint6", "eps_gradient6", "charge_potential6"]
