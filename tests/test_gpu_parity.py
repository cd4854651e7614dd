"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes are chosen so the oracle finishes in seconds while the grids span
several tiles of every kernel and have ragged edges (x extents that are not
multiples of the 64-wide stencil tiles, radix-3 FFT lengths, a wet slab that
wraps through z = 0).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu

FOUR_PI = 4.0 * math.pi


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _solver(torch, n, L, **opts):
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(n, L, **opts)
    return s


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ---------------------------------------------------------------- building blocks

@pytest.mark.parametrize("n", [(24, 36, 48), (32, 32, 64), (96, 16, 18)])
def test_apply_operator_matches_oracle(torch, n):
    L = (0.3 * n[0], 0.25 * n[1], 0.4 * n[2])
    eps, _ = W.random_fields(n, 7)
    rng = np.random.default_rng(8)
    phi = rng.normal(size=eps.shape)
    s = _solver(torch, n, L, z_wet_lo=0.3 * L[2], z_wet_hi=L[2])
    s.set_epsilon(_dev(torch, eps))
    out = _host(s.apply_operator(_dev(torch, phi)))
    ref = O.apply_A(phi, eps, s.h)
    assert _rel(out, ref) <= 1e-13


@pytest.mark.parametrize("n", [(24, 36, 48), (32, 32, 64), (96, 96, 192), (16, 8, 512), (12, 18, 384)])
def test_vacuum_solve_matches_oracle(torch, n):
    L = (0.2 * n[0], 0.3 * n[1], 0.1 * n[2])
    rng = np.random.default_rng(9)
    r = rng.normal(size=(n[2], n[1], n[0]))
    s = _solver(torch, n, L, z_wet_lo=0.3 * L[2], z_wet_hi=L[2])
    out = _host(s.vacuum_solve(_dev(torch, r)))
    ref = O.vacuum_solve(r, s.h)
    assert _rel(out, ref) <= 1e-12


def test_build_rho_matches_oracle(torch):
    w = W.slab(n=(48, 48, 96))
    s = _solver(torch, w.n, w.L)
    rho = _host(s.build_rho(w.xyz, w.q, w.sigma))
    ref = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    assert np.abs(rho - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("exclusion", [False, True])
def test_build_epsilon_matches_oracle(torch, exclusion):
    w = W.slab(n=(48, 48, 96), exclusion=exclusion)
    s = _solver(torch, w.n, w.L)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    eps = _host(s.get_epsilon())
    ref = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    assert np.abs(eps - ref).max() <= 1e-12 * 78.36


# ---------------------------------------------------------------- full solve

def _check_solution(torch, s, rho, eps, phi, E, info, tol_E, tol_phi):
    ref_phi = O.solve(rho, eps, s.h, tol=1e-13)
    ref_E = O.energy(rho, ref_phi, s.h)
    assert info["rel_res"] <= s.opts.tol
    assert abs(E - ref_E) <= tol_E * abs(ref_E), (E, ref_E)
    assert _rel(phi, ref_phi) <= tol_phi
    assert abs(info["energy_eps_form"] - E) <= 1e-9 * abs(E)
    return ref_phi


def test_solve_tanh_box_fp64(torch):
    w = W.tanh_box()
    eps = w.eps_grid()
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    s = _solver(torch, w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-10)
    s.set_epsilon(_dev(torch, eps))
    phi, E, info = s.solve(_dev(torch, rho))
    _check_solution(torch, s, rho, eps, _host(phi), E, info, 1e-10, 1e-8)


@pytest.mark.parametrize("exclusion,precision", [(False, 0), (True, 0), (True, 1), (False, 1)])
def test_solve_small_slab(torch, exclusion, precision):
    w = W.slab(n=(48, 48, 96), exclusion=exclusion)
    s = _solver(torch, w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-10, precision=precision)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho_d = s.build_rho(w.xyz, w.q, w.sigma)
    phi, E, info = s.solve(rho_d)
    eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    _check_solution(torch, s, rho, eps, _host(phi), E, info, 1e-10, 1e-8)


@pytest.mark.parametrize("exclusion", [False, True])
def test_solve_small_slab_float32_dry_update(torch, exclusion):
    """Mixed precision with the float32 FFT dry update: the preconditioner
    changes, the float64 coupling still reaches the same solution."""
    w = W.slab(n=(48, 48, 96), exclusion=exclusion)
    s = _solver(torch, w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-10, precision=1, fft_fp32=1)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho_d = s.build_rho(w.xyz, w.q, w.sigma)
    phi, E, info = s.solve(rho_d)
    eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    _check_solution(torch, s, rho, eps, _host(phi), E, info, 1e-10, 1e-8)


@pytest.mark.parametrize("exclusion", [False, True])
def test_forces_and_eps_gradient_match_oracle(torch, exclusion):
    w = W.slab(n=(48, 48, 96), exclusion=exclusion)
    s = _solver(torch, w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-12)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho_d = s.build_rho(w.xyz, w.q, w.sigma)
    phi_d, E, info = s.solve(rho_d)
    g = _host(s.eps_gradient())
    F = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    phi = _host(phi_d)
    # oracle gradient and forces evaluated on the GPU solution (isolates the kernels)
    g_ref = O.eps_gradient(phi, s.h)
    assert _rel(g, g_ref) <= 1e-12
    eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params)
    F_ref = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi, g_ref)
    assert np.abs(F - F_ref).max() <= 1e-10 * np.abs(F_ref).max()
    # and against the oracle's own solution
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    phi_o = O.solve(rho, eps, s.h, tol=1e-13)
    F_o = O.forces(w.n, w.L, w.xyz, w.radius, w.q, w.sigma, w.eps_params, phi_o, O.eps_gradient(phi_o, s.h))
    assert np.abs(F - F_o).max() <= 1e-8 * np.abs(F_o).max()
    # the switch term needs the atoms eps was built from
    from paper_0904_4887_amd.binding import DWPError, DWP_ESTATE
    moved = w.xyz.copy()
    moved[3, 0] += 0.01
    with pytest.raises(DWPError) as e:
        s.forces(moved, w.q, w.sigma, w.radius, w.eps_params)
    assert e.value.status == DWP_ESTATE


# ---------------------------------------------------------------- error paths

def test_error_paths(torch):
    from paper_0904_4887_amd.binding import DWPError, DWP_ESTATE, DWP_EINVAL, DWP_ENONFINITE, DWP_ENOCONV
    w = W.tanh_box(n=(16, 16, 32))
    s = _solver(torch, w.n, w.L, z_wet_lo=8.0, z_wet_hi=20.0)
    rho = O.rho_gauss(w.n, w.L, w.xyz, w.q, w.sigma)
    with pytest.raises(DWPError) as e:
        s.solve(_dev(torch, rho))
    assert e.value.status == DWP_ESTATE
    bad = w.eps_grid()
    bad[3, 2, 1] = 0.5
    with pytest.raises(DWPError) as e:
        s.set_epsilon(_dev(torch, bad))
    assert e.value.status == DWP_EINVAL
    s.set_epsilon(_dev(torch, w.eps_grid()))
    nan_rho = rho.copy()
    nan_rho[1, 1, 1] = np.nan
    with pytest.raises(DWPError) as e:
        s.solve(_dev(torch, nan_rho))
    assert e.value.status == DWP_ENONFINITE
    s.set_opts(max_outer=1)
    with pytest.raises(DWPError) as e:
        s.solve(_dev(torch, rho))
    assert e.value.status == DWP_ENOCONV
    s.set_opts(max_outer=600)
    phi, E, info = s.solve(_dev(torch, rho))
    assert info["rel_res"] <= 1e-10


@pytest.mark.parametrize("smoother", [1, 2])
@pytest.mark.parametrize("precision,cycles,pre,post", [(0, 1, 2, 2), (1, 1, 2, 2), (1, 2, 2, 2), (0, 1, 0, 1),
                                                    (1, 2, 0, 2)])
def test_fused_sweep_equals_colour_passes(torch, precision, cycles, pre, post, smoother):
    """The fused out-of-place sweep and the two in-place colour passes are the
    same Gauss-Seidel sweep: one application of the split agrees to rounding.
    The fine wet level of this grid (96 x 96 x 151) is above the size from
    which the fused kernel takes over, so both kernels really run: the fused
    one on bands of 12 whole rows (smoother 1) or on 32 x 16 tiles (smoother
    2).  Without pre-sweeps the first fused sweep follows the coarse-grid
    correction and must read it (its zero-input variant would drop it)."""
    from paper_0904_4887_amd.binding import plan
    w = W.slab(n=(96, 96, 192), exclusion=True)
    fine = plan(w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1])["levels"][0]
    assert fine[0] * fine[1] * fine[2] >= 1 << 20
    s = _solver(torch, w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], precision=precision, smoother=smoother,
                cycles=cycles, pre=pre, post=post)
    s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rng = np.random.default_rng(3)
    r = _dev(torch, rng.normal(size=s.shape))
    z1 = _host(s.apply_split(r))
    s.set_opts(smoother=0)
    z0 = _host(s.apply_split(r))
    assert _rel(z1, z0) <= (1e-12 if precision == 0 else 2e-5)


@pytest.mark.parametrize("smoother", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [(216, 216, 48), (162, 108, 96)])
def test_fused_sweep_equals_colour_passes_ragged_tiles(torch, n, precision, smoother):
    """The fused sweep against the two colour passes on grids whose x and y
    extents are not multiples of its 32 x 16 tile (tiles overhang the
    periodic wrap in x and y).  On 162 x 108 nx is 2 mod 4, so the float32
    variant loads 8-byte vectors; x cannot be halved there, so that grid has
    a single multigrid level, smoothed by the grid-wide kernels.  With
    smoother 1 the row-band kernel takes these levels with bands of 12 rows
    (216, float32), 4 rows (216, float64) and 6 rows (108), with 4- and
    2-wide vectors."""
    from paper_0904_4887_amd.binding import plan
    L = (0.07 * n[0], 0.07 * n[1], 0.1 * n[2])
    opts = dict(z_wet_lo=0.3 * L[2], z_wet_hi=L[2], precision=precision, smoother=smoother, coarse_sweeps=3)
    lv = plan(n, L, **opts)["levels"]
    assert lv[0][0] * lv[0][1] * lv[0][2] >= 1 << 20
    s = _solver(torch, n, L, **opts)
    eps, _ = W.random_fields(n, 17)
    s.set_epsilon(_dev(torch, eps))
    rng = np.random.default_rng(4)
    r = _dev(torch, rng.normal(size=s.shape))
    z1 = _host(s.apply_split(r))
    s.set_opts(smoother=0)
    z0 = _host(s.apply_split(r))
    assert np.isfinite(z1).all()
    assert _rel(z1, z0) <= (1e-12 if precision == 0 else 2e-5)


def test_bottom_vcycle_out_of_lds_matches_the_global_memory_one(torch):
    """The levels at the bottom of the hierarchy (12 x 12 x 37 and 6 x 6 x 18
    here) run in one workgroup; in float32 they fit its LDS (96 KB) and run out
    of it, in float64 (192 KB) they run from global memory.  One application
    of the split agrees between the two precisions to float32 rounding, while
    dropping the bottom levels changes it a hundred times more, so an error in
    either bottom kernel would show."""
    from paper_0904_4887_amd.binding import plan
    w = W.slab(n=(96, 96, 192), exclusion=True)
    opts = dict(z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], pre=2, post=2, coarse_sweeps=8)
    lv = plan(w.n, w.L, **opts)["levels"]
    assert [tuple(x) for x in lv[-2:]] == [(12, 12, 37), (6, 6, 18)]
    rng = np.random.default_rng(5)
    r = rng.normal(size=(w.n[2], w.n[1], w.n[0]))
    z = {}
    for key, kw in (("lds", dict(precision=1)), ("global", dict(precision=0)),
                    ("no_bottom", dict(precision=0, max_levels=len(lv) - 2))):
        s = _solver(torch, w.n, w.L, **opts, **kw)
        s.build_epsilon(w.xyz, w.radius, w.eps_params)
        z[key] = _host(s.apply_split(_dev(torch, r)))
        s.close()
    d_lds, d_drop = _rel(z["lds"], z["global"]), _rel(z["no_bottom"], z["global"])
    assert d_lds <= 1e-4 and d_drop >= 100 * d_lds, (d_lds, d_drop)


@pytest.mark.parametrize("n", [(24, 36, 48), (96, 96, 192), (192, 192, 384), (256, 256, 32), (18, 54, 48),
                               (16, 8, 512)])
def test_float32_vacuum_solve_matches_oracle(torch, n):
    """The dry update with its spectrum in float32 (fft_fp32), as the
    building block runs it: agrees with the float64 oracle to float32
    rounding on grids with radix-2, 3, 4 and 8 stages and long z."""
    L = (0.2 * n[0], 0.3 * n[1], 0.1 * n[2])
    rng = np.random.default_rng(19)
    r = rng.normal(size=(n[2], n[1], n[0]))
    s = _solver(torch, n, L, z_wet_lo=0.3 * L[2], z_wet_hi=L[2], precision=1, fft_fp32=1)
    out = _host(s.vacuum_solve(_dev(torch, r)))
    ref = O.vacuum_solve(r, s.h)
    assert _rel(out, ref) <= 2e-5


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("n", [(4096, 8, 8), (8, 4096, 8), (8, 8, 4096)])
def test_vacuum_solve_at_the_longest_axis(torch, n, fp32):
    """The largest extent the planner accepts (4096) along each axis in turn: a
    line of 4096 values is one FFT block by itself (the x pass then stages 4097
    complex values in LDS).  The smallest eigenvalue of the 4096-long axis,
    (2 pi / 4096)^2 / h^2, amplifies rounding about 64 times more than on the
    512-long axes of the other tests, and the bars scale with it."""
    L = (0.05 * n[0], 0.05 * n[1], 0.05 * n[2])
    rng = np.random.default_rng(23)
    r = rng.normal(size=(n[2], n[1], n[0]))
    s = _solver(torch, n, L, z_wet_lo=0.3 * L[2], z_wet_hi=L[2], precision=fp32, fft_fp32=fp32)
    out = _host(s.vacuum_solve(_dev(torch, r)))
    ref = O.vacuum_solve(r, s.h)
    assert _rel(out, ref) <= (5e-4 if fp32 else 1e-10)
