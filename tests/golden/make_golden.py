"""Write the oracle's reference results for the full-size workloads.

Calls only the FP64 oracle (and the seeded input generators).  Output: one
JSON file per workload in this directory, holding the energy in both forms,
the oracle's PCG iteration counts, phi and dE/d eps at 64 seeded nodes, the
mean of phi^2, and dE/dR of every atom (atom-built permittivities only).

With "one_pass" first, it writes instead the error of the paper's one-pass
split for the five headline configurations (or the names given).

Usage: python tests/golden/make_golden.py [name ...]
       python tests/golden/make_golden.py one_pass [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_0904_4887_amd import workloads as W  # noqa: E402


def workloads():
    return {
        "tanh_box_32x32x64": W.tanh_box(),
        "slab_96x96x192": W.slab((96, 96, 192)),
        "slab_96x96x192_excl": W.slab((96, 96, 192), exclusion=True),
        "slab_128x128x256": W.slab((128, 128, 256), tol=1e-12),
        "slab_192x192x384": W.slab((192, 192, 384), tol=1e-8, precision=1),
        "slab_192x192x384_excl": W.slab((192, 192, 384), exclusion=True, tol=1e-8, precision=1),
        "big_slab_256x256x512": W.big_slab(),
        "density_slab_192x192x384": W.density_slab((192, 192, 384)),
        "slab_gamma_192x192x384": W.slab_gamma((192, 192, 384)),
        "slab_gamma_192x192x384_excl": W.slab_gamma((192, 192, 384), exclusion=True),
        "slab6_96x96x192": W.slab((96, 96, 192), tol=1e-10),
        "big_slab_256x256x512_md3": md_workload(W.big_slab(), 3),
    }


def md_workload(w, steps):
    """The workload after `steps` MD-like displacements: R += N(0, 0.02 A) per
    step, cumulative, the same draws as the warm-started MD loop."""
    disp = W.md_displacements(len(w.q), steps + 1)
    xyz = w.xyz.copy()
    for t in range(1, steps + 1):
        xyz = np.mod(xyz + disp[t], np.array(w.L))
    w.xyz = xyz
    w.name = f"{w.name}_md{steps}"
    return w


def first_below(history, tol):
    for i, r in enumerate(history):
        if r <= tol:
            return i + 1
    return None


def make_sixth(name, w):
    """The sixth-order operator (Eqs. 16-18) on an atom-built slab: energy,
    background constant, phi and dE/d eps (adjoint) at 64 nodes, dE/dR."""
    from oracle import sixth as S
    t0 = time.time()
    eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    phi, info = S.solve6(rho, eps, w.h, tol=1e-12, return_info=True)
    t1 = time.time()
    lam = S.adjoint6(rho, eps, w.h, tol=1e-12)
    g = S.eps_gradient6(phi, lam, w.h)
    F = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, S.charge_potential6(phi, lam, w.h), g)
    rng = np.random.default_rng(12345)
    nodes = np.sort(rng.choice(w.N, size=64, replace=False))
    out = dict(name=name, n=list(w.n), L=list(w.L), order=6, energy=O.energy(rho, phi, w.h),
               background=info["background"], oracle_gmres_iters=info["iters"], oracle_rel_res=info["rel_res"],
               nodes=nodes.tolist(), phi=phi.ravel()[nodes].tolist(), g=g.ravel()[nodes].tolist(),
               forces=F.tolist(), t_solve_s=t1 - t0, t_total_s=time.time() - t0)
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "E", out["energy"], "gmres", info["iters"], "s", round(time.time() - t0, 1), flush=True)


def make(name, w):
    if name.startswith("slab6_"):
        return make_sixth(name, w)
    t0 = time.time()
    rho_e = None
    if w.eps_kind == "tanh_z":
        eps = w.eps_grid()
        params = None
    elif w.eps_kind == "gamma":
        eps = O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params)
        params = w.eps_params
    elif w.eps_kind == "density":
        p = w.eps_params
        rho_e = W.electron_density(w)
        eps = O.eps_of_density(rho_e, p["eps_inf"], p["rho0"], p["beta"])
        params = None
    else:
        eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
        params = w.eps_params
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    t1 = time.time()
    phi, info = O.solve(rho, eps, w.h, tol=1e-12, max_iter=1000, return_info=True)
    t2 = time.time()
    E = O.energy(rho, phi, w.h)
    Ee = O.energy_eps_form(phi, eps, w.h)
    g = O.eps_gradient(phi, w.h)
    rng = np.random.default_rng(12345)
    nodes = np.sort(rng.choice(w.N, size=64, replace=False))
    out = dict(name=name, n=list(w.n), L=list(w.L), energy=E, energy_eps_form=Ee,
               oracle_iters=info["iters"], oracle_rel_res=info["rel_res"],
               oracle_iters_to=dict((f"{t:.0e}", first_below(info["history"], t)) for t in (1e-8, 1e-10, 1e-12)),
               nodes=nodes.tolist(), phi=phi.ravel()[nodes].tolist(), g=g.ravel()[nodes].tolist(),
               phi2_mean=float(np.mean(phi * phi)), t_build_s=t1 - t0, t_solve_s=t2 - t1)
    del g
    if rho_e is not None:
        p = w.eps_params
        out["v_eps"] = O.v_eps(phi, rho_e, w.h, p["eps_inf"], p["rho0"], p["beta"]).ravel()[nodes].tolist()
        # the charge term of dE/dR (eps does not move with the atoms here)
        F = O.forces(w.n, w.L, w.xyz, None, w.q, w.sigma, None, phi, None)
        out["forces"] = F.tolist()
    if params is not None:
        t3 = time.time()
        if w.eps_kind == "gamma":
            F = O.forces_gamma(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, params, phi, O.eps_gradient(phi, w.h))
        else:
            F = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, params, phi, O.eps_gradient(phi, w.h))
        out["forces"] = F.tolist()
        out["t_forces_s"] = time.time() - t3
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "E", E, "iters", info["iters"], "solve s", round(t2 - t1, 1), flush=True)


# the five headline configurations, smallest first
ONE_PASS = ("tanh_box_32x32x64", "slab_96x96x192", "slab_128x128x256", "slab_192x192x384",
            "big_slab_256x256x512")


def make_one_pass(name, w):
    """The error of the paper's one-pass dry/wet split (Sec. II.F) against the
    exact solution of the same discrete problem, on the configured wet slab:
    relative energy error, relative L2 and max-norm errors of phi."""
    t0 = time.time()
    eps = w.eps_grid() if w.eps_kind == "tanh_z" else O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    phi = O.solve(rho, eps, w.h, tol=1e-12, max_iter=3000)
    k0, k1 = W.wet_planes(w.n[2], w.L[2], w.z_wet)
    phi_a = O.one_pass_split(rho, eps, w.h, k0, k1, tol=1e-12)
    E, E_a = O.energy(rho, phi, w.h), O.energy(rho, phi_a, w.h)
    d = phi_a - phi
    out = dict(name=name, n=list(w.n), L=list(w.L), z_wet=list(w.z_wet), wet_planes=[int(k0), int(k1)],
               energy=E, energy_one_pass=E_a, rel_energy_error=(E_a - E) / abs(E),
               rel_l2_phi_error=float(np.linalg.norm(d) / np.linalg.norm(phi)),
               rel_max_phi_error=float(np.abs(d).max() / np.abs(phi).max()), t_s=time.time() - t0)
    with open(os.path.join(HERE, f"oracle_one_pass_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("one-pass", name, "rel E", out["rel_energy_error"], "rel L2 phi", out["rel_l2_phi_error"],
          "s", round(out["t_s"], 1), flush=True)


if __name__ == "__main__":
    ws = workloads()
    args = sys.argv[1:]
    if args and args[0] == "one_pass":
        for nm in args[1:] or ONE_PASS:
            make_one_pass(nm, ws[nm])
        sys.exit(0)
    for nm in args or list(ws):
        make(nm, ws[nm])
