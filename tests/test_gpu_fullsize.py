"""Parity at the full workload sizes, in the configuration the benchmark runs.

The oracle's results for these sizes take minutes to hours of CPU time, so
they are stored under tests/golden/ (written by tests/golden/make_golden.py,
which calls only the oracle): the energy in both forms, phi and dE/d eps at 64
seeded nodes (V_eps too for a density-built permittivity), and dE/dR of every
atom.
"""
import json
import os

import numpy as np
import pytest

from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# the mixed-precision configuration the benchmark runs: float32 dry update,
# float32 Krylov vectors with the Arnoldi basis in float16, around the float32
# multigrid
HEADLINE = dict(fft_fp32=1, krylov_fp32=1, krylov_fp16=1)

# name -> (workload, E tol, phi tol (x max|phi| at the samples), force tol (x max|F|)[, stored result
# [, extra solver options]])
CASES = {
    "tanh_box_32x32x64": (lambda: W.tanh_box(), 1e-10, 1e-8, None),
    "slab_96x96x192": (lambda: W.slab((96, 96, 192)), 1e-10, 1e-8, 1e-7),
    "slab_96x96x192_excl": (lambda: W.slab((96, 96, 192), exclusion=True), 1e-10, 1e-8, 1e-7),
    "slab_128x128x256": (lambda: W.slab((128, 128, 256), tol=1e-12), 1e-10, 1e-9, 1e-8),
    "slab_192x192x384": (lambda: W.slab((192, 192, 384), tol=1e-8, precision=1), 1e-8, 1e-6, 1e-5),
    # the same slab solved entirely in float64 at the same tolerance
    "slab_192x192x384_fp64": (lambda: W.slab((192, 192, 384), tol=1e-8, precision=0), 1e-8, 1e-6, 1e-5,
                              "slab_192x192x384"),
    "slab_192x192x384_excl": (lambda: W.slab((192, 192, 384), exclusion=True, tol=1e-8, precision=1),
                              1e-8, 1e-6, 1e-5),
    "slab_192x192x384_headline": (lambda: W.slab((192, 192, 384), tol=1e-8, precision=1), 1e-8, 1e-6, 1e-5,
                                  "slab_192x192x384", HEADLINE),
    "big_slab_256x256x512": (lambda: W.big_slab(), 1e-8, 1e-6, 1e-5),
    "big_slab_256x256x512_headline": (lambda: W.big_slab(), 1e-8, 1e-6, 1e-5, "big_slab_256x256x512", HEADLINE),
    "density_slab_192x192x384": (lambda: W.density_slab((192, 192, 384)), 1e-8, 1e-6, 1e-5),
    "slab_gamma_192x192x384": (lambda: W.slab_gamma((192, 192, 384)), 1e-8, 1e-6, 1e-5),
    "slab_gamma_192x192x384_excl": (lambda: W.slab_gamma((192, 192, 384), exclusion=True), 1e-8, 1e-6, 1e-5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_matches_stored_oracle(name):
    case = CASES[name]
    make, tol_E, tol_phi, tol_F = case[:4]
    stored = case[4] if len(case) > 4 else name
    extra = case[5] if len(case) > 5 else {}
    path = os.path.join(GOLDEN, f"oracle_{stored}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result for {stored}")
    import torch
    from paper_0904_4887_amd.binding import Solver
    w = make()
    with open(path) as f:
        ref = json.load(f)
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts(**extra))
    if w.eps_kind == "tanh_z":
        s.set_epsilon(torch.from_numpy(w.eps_grid()).cuda())
    elif w.eps_kind == "density":
        p = w.eps_params
        s.build_epsilon_density(torch.from_numpy(W.electron_density(w)).cuda(), p["eps_inf"], p["rho0"], p["beta"])
    else:
        s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho = s.build_rho(w.xyz, w.q, w.sigma)
    phi, E, info = s.solve(rho)
    assert info["rel_res"] <= w.tol
    assert abs(E - ref["energy"]) <= tol_E * abs(ref["energy"]), (E, ref["energy"])
    nodes = np.array(ref["nodes"])
    ph = phi.reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy()
    ref_phi = np.array(ref["phi"])
    assert np.abs(ph - ref_phi).max() <= tol_phi * np.abs(ref_phi).max()
    g = s.eps_gradient().reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy()
    ref_g = np.array(ref["g"])
    assert np.abs(g - ref_g).max() <= 10 * tol_phi * np.abs(ref_g).max()
    if "v_eps" in ref:
        v = s.v_eps().reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy()
        ref_v = np.array(ref["v_eps"])
        assert np.abs(v - ref_v).max() <= 10 * tol_phi * np.abs(ref_v).max()
    if tol_F is not None and "forces" in ref:
        density = w.eps_kind == "density"
        F = s.forces(w.xyz, w.q, w.sigma, None if density else w.radius, None if density else w.eps_params)
        F_ref = np.array(ref["forces"])
        assert np.abs(F - F_ref).max() <= tol_F * np.abs(F_ref).max()
    s.close()


@pytest.mark.parametrize("extra", [{}, HEADLINE], ids=["mixed", "headline"])
def test_big_slab_md_steps_match_stored_oracle(extra):
    """The 256 x 256 x 512 slab through the warm-started MD loop: a cold solve
    at the initial atoms, then three steps of cumulative N(0, 0.02 A)
    displacements, each solved from the previous phi; after the third step
    the energy, phi at the stored nodes and dE/dR match the oracle's solution
    at the displaced positions."""
    path = os.path.join(GOLDEN, "oracle_big_slab_256x256x512_md3.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle result for big_slab_256x256x512_md3")
    import torch
    from paper_0904_4887_amd.binding import Solver
    with open(path) as f:
        ref = json.load(f)
    w = W.big_slab()
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts(**extra))
    disp = W.md_displacements(len(w.q), 4)
    xyz = w.xyz.copy()
    rho, phi = s.empty(), s.empty().zero_()
    iters = []
    for t in range(4):
        if t:
            xyz = np.mod(xyz + disp[t], np.array(w.L))
        s.set_opts(warm_start=1 if t else 0)
        s.build_epsilon(xyz, w.radius, w.eps_params)
        s.build_rho(xyz, w.q, w.sigma, out=rho)
        _, E, info = s.solve(rho, phi)
        assert info["rel_res"] <= w.tol
        iters.append(info["outer_iters"])
    assert abs(E - ref["energy"]) <= 1e-8 * abs(ref["energy"]), (E, ref["energy"])
    nodes = torch.from_numpy(np.array(ref["nodes"])).cuda()
    ref_phi = np.array(ref["phi"])
    assert np.abs(phi.reshape(-1)[nodes].cpu().numpy() - ref_phi).max() <= 1e-6 * np.abs(ref_phi).max()
    F = s.forces(xyz, w.q, w.sigma, w.radius, w.eps_params)
    F_ref = np.array(ref["forces"])
    assert np.abs(F - F_ref).max() <= 1e-5 * np.abs(F_ref).max()
    assert max(iters[1:]) <= iters[0]  # the warm start never costs iterations
    s.close()
