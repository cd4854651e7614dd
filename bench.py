#!/usr/bin/env python
"""Throughput of the dry/wet generalized-Poisson path on one MI355X.

One step = the whole hot path on one synthetic slab-plus-solvent input:
build eps from the atoms, build the Gaussian charge density, solve
div(eps grad phi) = -4 pi rho to a relative residual of 1e-8 (cold start from
phi = 0, FFT dry update + multigrid wet solve coupled by FGMRES), the energy,
dE/d eps (the adjoint) and dE/dR for every atom.  value = steps per second =
solves per second.

Default workload: the 192 x 192 x 384 slab (72 Ti/O atoms in an
11.8 x 11.8 x 40 A cell, dry z < 14 A), mixed precision (float32 multigrid
inside float64 coupling).  The line also reports the same step in float64,
the same step with the exclusion rule (a really dry region), the dominant
kernel's roofline and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--precision mixed|fp64] [--exclusion] [--no-cpu]
                       [--no-compare]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_0904_4887_amd import workloads as W  # noqa: E402

METRIC = "generalized-Poisson solves/s to 1e-8 residual + smoother HBM GB/s, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0


def make_workload(name, exclusion):
    n = tuple(int(x) for x in name.split("_")[-1].split("x"))
    if name.startswith("big_slab"):
        return W.big_slab(n=n, exclusion=exclusion, tol=1e-8)
    return W.slab(n=n, exclusion=exclusion, tol=1e-8)


def run_steps(s, w, steps, warmup, torch, keep=None):
    """Time `steps` whole steps after `warmup` untimed ones; returns seconds per
    step, the last energy, the per-step infos, the last dE/dR and the profile
    groups; with keep (a dict), also keep["phi"] (the last solution)."""
    rho = s.empty()
    phi = s.empty()
    infos = []

    def step():
        s.build_epsilon(w.xyz, w.radius, w.eps_params)
        s.build_rho(w.xyz, w.q, w.sigma, out=rho)
        _, E, info = s.solve(rho, phi)
        F = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
        return E, info, F

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s.profile_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        E, info, F = step()
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile()
    if keep is not None:
        keep["phi"] = phi
    return (t1 - t0) / steps, E, infos, F, prof


def solver_for(w, precision, torch, profile=0, **extra):
    """A solver for workload w at tol 1e-8.  Mixed precision runs the dry
    update in float32 (fft_fp32) and, where the library supports it (second
    order, or sixth order with the FFT dry update alone; restart <= 16), keeps
    the Krylov vectors in float32 (krylov_fp32), and with the second-order
    operator the Arnoldi basis in float16 (krylov_fp16), unless the workload or
    extra says otherwise."""
    from paper_0904_4887_amd.binding import Solver
    order = extra.get("order", w.opts.get("order", 2))
    if precision == "mixed":
        # the whole preconditioner in float32: the dry update too (unless the
        # workload's own options say otherwise)
        if "fft_fp32" not in w.opts:
            extra.setdefault("fft_fp32", 1)
        cycles = extra.get("cycles", w.opts.get("cycles", 1))
        restart = extra.get("restart", w.opts.get("restart", 10))
        if (order == 2 or cycles == 0) and restart <= 16 and "krylov_fp32" not in w.opts:
            extra.setdefault("krylov_fp32", 1)
        if order == 2 and extra.get("krylov_fp32", w.opts.get("krylov_fp32", 0)) == 1 and "krylov_fp16" not in w.opts:
            extra.setdefault("krylov_fp16", 1)
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts(tol=1e-8, precision=1 if precision == "mixed" else 0, profile=profile,
                                         **extra))
    return s


def sweep_source_digest():
    """sha256 of the fine-level sweep's source: band_sweep.h (the row-band
    kernel's per-thread code), then the text of kern_grid.hip from the row-band
    kernel (`// Row-band variant of the fused sweep`) to the banner of the next
    kernel (`// ---...--- residual + restriction`), then the text of its
    launchers, from `// Row-band sweep: returns false` to the end of
    `launch_sweep_fused<double>`.  Edits elsewhere leave it alone."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_0904_4887_amd", "csrc")
    src, hdr = os.path.join(csrc, "kern_grid.hip"), os.path.join(csrc, "band_sweep.h")
    if not (os.path.exists(src) and os.path.exists(hdr)):
        return None
    text = open(src).read()
    try:
        a = text.index("// Row-band variant of the fused sweep")
        b = text.index("residual + restriction", a)
        c = text.index("// Row-band sweep: returns false")
        d = text.index("launch_sweep_fused<double>(", c)
        d = text.index("\n}\n", d) + 3
    except ValueError:
        return None
    return hashlib.sha256((open(hdr).read() + text[a:b] + text[c:d]).encode()).hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary,
    if that summary was taken on the current source of the kernel and its
    launchers (sweep_source_digest), else None."""
    summ = os.path.join(ROOT, "profiles", "sweep_band_slab_192x192x384_mixed.md")
    digest = sweep_source_digest()
    if digest is None or not os.path.exists(summ):
        return None
    vals = {}
    for line in open(summ):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source sha256") != digest or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_small=(96, 96, 192)):
    """The FP64 oracle's whole step, timed on the host: permittivity and charge
    density from the workload's atoms, the solve to a 1e-8 residual (PCG with
    the vacuum FFT preconditioner, cold start), dE/d eps and dE/dR of every
    atom, on the same slab recipe at a grid that finishes in tens of seconds
    (96 x 96 x 192, same cell and atoms); scaled to the workload's grid by its
    point count (the builds and the force sums grow with the atom-node pairs,
    the solve with points x iterations, the oracle's own iteration count at the
    workload size being taken from its stored run)."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    ws = W.slab(n_small, tol=1e-8)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        eps = O.eps_erf(ws.n, ws.L, ws.xyz, ws.radius, ws.eps_params)
        rho = O.rho_gauss(ws.n, ws.L, ws.xyz, ws.q, ws.sigma)
        t1 = time.perf_counter()
        phi, info = O.solve(rho, eps, ws.h, tol=1e-8, return_info=True)
        t2 = time.perf_counter()
        O.energy(rho, phi, ws.h)
        O.forces(ws.n, ws.L, ws.xyz, ws.radius, ws.q, ws.sigma, ws.eps_params, phi, O.eps_gradient(phi, ws.h))
        t3 = time.perf_counter()
    ratio = (w.n[0] * w.n[1] * w.n[2]) / (ws.n[0] * ws.n[1] * ws.n[2])
    it_big = golden_iters(w.name) or info["iters"]
    t_est = ratio * ((t1 - t0) + (t3 - t2) + (t2 - t1) * it_big / info["iters"])
    return {"value": round(1.0 / t_est, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"the oracle's whole step (eps and rho from the atoms, PCG solve to 1e-8, dE/d eps, dE/dR) "
                      f"on the same slab recipe at {ws.n[0]}x{ws.n[1]}x{ws.n[2]}, measured "
                      f"{t3 - t0:.1f} s ({t1 - t0:.1f} build, {t2 - t1:.1f} solve in {info['iters']} iterations, "
                      f"{t3 - t2:.1f} forces); scaled x{ratio:g} in points and x{it_big}/{info['iters']} in "
                      f"iterations to {w.n[0]}x{w.n[1]}x{w.n[2]}; NumPy/SciPy, one thread",
            "measured_small": {"grid": list(ws.n), "s_per_step": round(t3 - t0, 2), "build_s": round(t1 - t0, 2),
                               "solve_s": round(t2 - t1, 2), "iters": info["iters"], "forces_s": round(t3 - t2, 2)},
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def errors_vs_oracle(name, E, info, phi, F, torch):
    """Per-result errors against the stored FP64 oracle solution: relative
    energy error (E = 1/2 h^3 sum rho phi, and the variational form 2E - E_eps,
    whose error is second order in the residual), max |phi - phi_o| / max |phi_o|
    over the stored nodes, and max |dE/dR - dE/dR_o| / max |dE/dR_o|."""
    p = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        ref = json.load(f)
    Eo = ref["energy"]
    nodes = torch.from_numpy(np.array(ref["nodes"])).to(phi.device)
    ph = phi.reshape(-1)[nodes].cpu().numpy()
    po = np.array(ref["phi"])
    out = {"rel_energy_err": abs(E - Eo) / abs(Eo),
           "rel_energy_err_variational": abs(2.0 * E - info["energy_eps_form"] - Eo) / abs(Eo),
           "max_phi_err_rel": float(np.abs(ph - po).max() / np.abs(po).max()),
           "phi_nodes": len(po), "rel_res": info["rel_res"]}
    if F is not None and "forces" in ref:
        Fo = np.array(ref["forces"])
        out["max_force_err_rel"] = float(np.abs(F - Fo).max() / np.abs(Fo).max())
    return out


def one_pass_errors():
    """The stored error of the paper's one-pass dry/wet split (the FFT, then
    one wet solve with the FFT potential as boundary data) against the exact
    discrete solution, for the five headline configurations: written by the
    oracle alone (tests/golden/make_golden.py one_pass)."""
    out = {}
    for name in ("tanh_box_32x32x64", "slab_96x96x192", "slab_128x128x256", "slab_192x192x384",
                 "big_slab_256x256x512"):
        p = os.path.join(ROOT, "tests", "golden", f"oracle_one_pass_{name}.json")
        if os.path.exists(p):
            with open(p) as f:
                d = json.load(f)
            out[name] = {k: d[k] for k in ("rel_energy_error", "rel_l2_phi_error", "rel_max_phi_error")}
    return out


def cpu_widened(gpu_ms):
    """The oracle beside the widened paths, on bounded samples (one thread):
    the dummy-density permittivity at 1/64 of the 192x192x384 nodes, scaled to
    the grid; the density permittivity and V_eps on the full grid; one
    application of the sixth-order operator on the full grid.  Each is set
    against the GPU's time for the same work (kernel means from the profile
    groups of the timed entries, passed in as gpu_ms)."""
    import oracle as O
    from oracle import sixth as S
    from threadpoolctl import threadpool_limits
    out = {}
    with threadpool_limits(limits=1):
        w = W.slab_gamma((192, 192, 384))
        nodes = np.arange(0, w.N, 64)
        t0 = time.perf_counter()
        O.eps_gamma(w.n, w.L, w.xyz, w.radius, w.eps_params, nodes=nodes)
        t_gamma = (time.perf_counter() - t0) * 64
        out["gamma_eps_build"] = {"oracle_s": round(t_gamma, 2), "sample": "1/64 of the nodes, x64",
                                  "gpu_ms": gpu_ms.get("gamma_build")}
        wd = W.density_slab((192, 192, 384))
        rho_e = W.electron_density(wd)
        p = wd.eps_params
        phi = np.random.default_rng(0).normal(size=rho_e.shape)
        t0 = time.perf_counter()
        O.eps_of_density(rho_e, p["eps_inf"], p["rho0"], p["beta"])
        O.v_eps(phi, rho_e, wd.h, p["eps_inf"], p["rho0"], p["beta"])
        out["density_eps_and_v_eps"] = {"oracle_s": round(time.perf_counter() - t0, 2), "sample": "full grid",
                                        "gpu_ms": gpu_ms.get("density")}
        eps = np.full(rho_e.shape, 2.0)
        t0 = time.perf_counter()
        S.apply_A6(phi, eps, wd.h)
        out["sixth_order_apply"] = {"oracle_s": round(time.perf_counter() - t0, 2), "sample": "full grid",
                                    "gpu_ms": gpu_ms.get("sixth_apply")}
    out["cores"] = 1
    return out


def md_loop(w, steps, torch, precision="mixed"):
    """MD-like steps: R += N(0, 0.02 A) per step (cumulative), eps and rho
    rebuilt, phi warm-started from the previous step, forces every step."""
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    mixed = precision == "mixed"
    s.set_grid(w.n, w.L, **w.solver_opts(tol=1e-8, precision=1 if mixed else 0, krylov_fp32=1 if mixed else 0,
                                         fft_fp32=1 if mixed else 0))
    disp = W.md_displacements(len(w.q), steps)
    rho, phi = s.empty(), s.empty()
    xyz = w.xyz.copy()
    per = []
    for t in range(steps):
        if t > 0:
            xyz = np.mod(xyz + disp[t], np.array(w.L))
        s.set_opts(warm_start=1 if t > 0 else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.build_epsilon(xyz, w.radius, w.eps_params)
        s.build_rho(xyz, w.q, w.sigma, out=rho)
        _, E, info = s.solve(rho, phi)
        F = s.forces(xyz, w.q, w.sigma, w.radius, w.eps_params)
        torch.cuda.synchronize()
        per.append(dict(ms=round(1e3 * (time.perf_counter() - t0), 2), iters=info["outer_iters"], energy=E,
                        max_force=float(np.abs(F).max())))
    s.close()
    return per


def gpu_wall_ms(torch, fn, reps=3):
    """Median wall time of fn() in ms, with the device synchronised around it."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return round(float(np.median(ts)), 3)


def density_steps(torch, n=(192, 192, 384), steps=4, warmup=1, precision="mixed"):
    """Density-dependent permittivity (Eq. 7): eps and d eps/d rho from an
    electron-density grid, the solve, and V_eps (Eq. 6), per step; the density
    and the source are resident before timing."""
    w = W.density_slab(n)
    p = w.eps_params
    s = solver_for(w, precision, torch)
    rho_e = torch.from_numpy(W.electron_density(w)).cuda()
    src = s.build_rho(w.xyz, w.q, w.sigma)
    phi = s.empty()
    v = s.empty()
    infos = []

    def step():
        s.build_epsilon_density(rho_e, p["eps_inf"], p["rho0"], p["beta"])
        _, E, info = s.solve(src, phi)
        s.v_eps(out=v)
        return E, info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        E, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    vmax = float(v.abs().max())
    pmax = float(phi.abs().max())
    # the permittivity and V_eps alone (no solve), for the oracle comparison
    t_eps = gpu_wall_ms(torch, lambda: s.build_epsilon_density(rho_e, p["eps_inf"], p["rho0"], p["beta"]))
    s.solve(src, phi)
    t_v = gpu_wall_ms(torch, lambda: s.v_eps(out=v))
    s.close()
    return {"ms_per_step": round(1e3 * sec, 2), "steps_per_s": round(1.0 / sec, 3),
            "iters": [i["outer_iters"] for i in infos], "energy": E, "z_wet": list(w.z_wet),
            "rho0": p["rho0"], "beta": p["beta"], "max_abs_v_eps": vmax, "max_abs_phi": pmax,
            "v_eps_over_phi": round(vmax / pmax, 3), "eps_build_ms": t_eps, "v_eps_ms": t_v}


def gamma_steps(torch, exclusion, n=(192, 192, 384), steps=4, warmup=1, precision="mixed"):
    """The full step with the paper's own permittivity (Eqs. 9, 10, 19):
    eps from the dummy density, rho, the solve, the adjoint and the forces;
    plus the per-group kernel times of one instrumented step."""
    w = W.slab_gamma(n, exclusion=exclusion)
    s = solver_for(w, precision, torch)
    sec, E, infos, _, _ = run_steps(s, w, steps, warmup, torch)
    t_build = gpu_wall_ms(torch, lambda: s.build_epsilon(w.xyz, w.radius, w.eps_params))
    s.close()
    sp = solver_for(w, precision, torch, profile=1)
    _, _, _, _, prof = run_steps(sp, w, 1, 1, torch)
    sp.close()
    return {"ms_per_step": round(1e3 * sec, 2), "steps_per_s": round(1.0 / sec, 3),
            "iters": [i["outer_iters"] for i in infos], "energy": E, "z_wet": list(w.z_wet),
            "beta": w.eps_params["beta"], "builders_ms": round(prof.get("builders", {}).get("ms", 0.0), 3),
            "forces_ms": round(prof.get("forces", {}).get("ms", 0.0), 3), "eps_build_ms": t_build}


def sixth_order_steps(torch, n=(192, 192, 384), steps=2, warmup=1, precision="mixed"):
    """The full step with the paper's sixth-order operator (Eqs. 16-18) on the
    literal slab: eps, rho, the solve, and the forces, which need the adjoint
    solve of the non-symmetric operator."""
    w = W.slab(n, tol=1e-8)
    # the FFT dry update alone, unscaled: with A6 as the outer operator the
    # 7-point wet V-cycle slows the coupling down (the entry "with_wet_vcycle")
    w.opts = dict(order=6, cycles=0, scaled_dry=0, restart=16)
    s = solver_for(w, precision, torch)
    sec, E, infos, _, _ = run_steps(s, w, steps, warmup, torch)
    x = s.empty().normal_()
    t_apply = gpu_wall_ms(torch, lambda: s.apply_operator(x), reps=5)
    s.close()
    out = {"ms_per_step": round(1e3 * sec, 2), "steps_per_s": round(1.0 / sec, 3),
           "iters": [i["outer_iters"] for i in infos], "energy": E, "background": infos[-1]["background"],
           "opts": dict(w.opts), "apply_ms": t_apply}
    w.opts = dict(order=6, scaled_dry=1, pre=1, post=1, coarse_sweeps=4)
    s = solver_for(w, precision, torch, max_outer=1000)
    sec, E, infos, _, _ = run_steps(s, w, 1, 0, torch)
    s.close()
    out["with_wet_vcycle"] = {"ms_per_step": round(1e3 * sec, 2), "iters": infos[-1]["outer_iters"],
                              "energy": E, "opts": dict(w.opts)}
    # the exclusion slab: every setting with the wet V-cycle stalls; the FFT
    # dry update alone converges, and with restart 60 so does the adjoint
    # solve, in float64 (with the float32 dry update the coupling stalls)
    from paper_0904_4887_amd.binding import DWPError
    we = W.slab(n, exclusion=True, tol=1e-8)
    we.opts = dict(order=6, cycles=0, scaled_dry=0, restart=60, fft_fp32=0)
    s = solver_for(we, precision, torch, max_outer=3000)
    try:
        sec, E, infos, _, _ = run_steps(s, we, 1, 1, torch)
        out["exclusion"] = {"ms_per_step": round(1e3 * sec, 2), "iters": infos[-1]["outer_iters"], "energy": E,
                            "opts": dict(we.opts), "z_wet": list(we.z_wet)}
    except DWPError as e:
        out["exclusion"] = {"error": str(e), "opts": dict(we.opts)}
    s.close()
    return out


def copy_ceiling(torch):
    """Measured device copy bandwidth (1 GiB read + 1 GiB written per copy)."""
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del x, y
    return round(2.0 * (1 << 30) / dt / 1e9, 1)


def hbm_resident_smoother(torch, n=(512, 512, 512), reps=4):
    """The fine-level fused sweep on a grid whose wet field set is far larger
    than the 256 MB last-level cache: the 512^3 box with the planar tanh
    permittivity of the smallest workload stretched to it, wet region the top
    70 %; the split preconditioner is applied `reps` times and only the
    fine-level sweeps are timed (HIP events on the library's stream)."""
    from paper_0904_4887_amd.binding import Solver
    L = (0.1 * n[0], 0.1 * n[1], 0.1 * n[2])
    z = np.arange(n[2]) * L[2] / n[2]
    prof = 1.0 + (W.EPS_INF - 1.0) * 0.5 * (1.0 + np.tanh((z - 0.5 * L[2]) / 1.0))
    eps = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(prof[:, None, None], (n[2], n[1], n[0])))).cuda()
    out = {}
    for prec in ("mixed", "fp64"):
        s = Solver(0)
        s.set_grid(n, L, z_wet_lo=0.3 * L[2], z_wet_hi=L[2], precision=1 if prec == "mixed" else 0, profile=2,
                   restart=1)
        s.set_epsilon(eps)
        r = torch.randn(n[2], n[1], n[0], dtype=torch.float64, device="cuda")
        s.apply_split(r)
        torch.cuda.synchronize()
        s.profile_reset()
        for _ in range(reps):
            s.apply_split(r)
        torch.cuda.synchronize()
        p = s.profile().get("rbgs_fine")
        s.close()
        if p and p["ms"] > 0:
            out[prec] = {"GB/s": round(p["bytes"] / p["ms"] / 1e6, 1), "avg_launch_us": round(1e3 * p["ms"] / p["launches"], 2),
                         "launches": p["launches"], "algorithmic_bytes_per_launch": p["bytes"] / p["launches"]}
    del eps
    torch.cuda.empty_cache()
    return {"grid": list(n), "wet_fraction": 0.7, **out}


def coupling_variants(w, precision, torch, steps=3):
    """The literal slab's coupling under other solver parameters at the same
    tolerance (the wet cut and the cycle change the preconditioner, not the
    result): (i) the FFT dry update alone (no wet correction); (ii) the wet
    region extended from the top of the slab through the solvent above it and
    across the periodic wrap to the bottom of the slab, so that the FFT's dry
    region is the slab's interior; (iii) that cut with V(2,2) cycles and a
    64-sweep coarsest solve."""
    top = float(w.xyz[:, 2].max())
    bot = float(w.xyz[:, 2].min())
    cut = (top + 0.5, w.L[2] + bot)
    out = {}
    for key, kw in [("fft_only", dict(cycles=0)),
                    ("slab_interior_dry", dict(z_wet_lo=cut[0], z_wet_hi=cut[1])),
                    ("slab_interior_dry_v22", dict(z_wet_lo=cut[0], z_wet_hi=cut[1], pre=2, post=2,
                                                   coarse_sweeps=64))]:
        sv = solver_for(w, precision, torch, **kw)
        keep = {}
        sec, E, infos, F, _ = run_steps(sv, w, steps, 1, torch, keep=keep)
        out[key] = {"ms_per_step": round(1e3 * sec, 2), "iters": infos[-1]["outer_iters"], "energy": E,
                    "z_wet": [kw.get("z_wet_lo", w.z_wet[0]), kw.get("z_wet_hi", w.z_wet[1])],
                    "phases_ms": {k: round(infos[-1][k], 2) for k in ("t_fft_ms", "t_mg_ms", "t_krylov_ms")},
                    "vs_oracle": errors_vs_oracle(w.name, E, infos[-1], keep["phi"], F, torch)}
        sv.close()
    return out


def golden_iters(name):
    p = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if os.path.exists(p):
        with open(p) as f:
            d = json.load(f)
        v = d.get("oracle_iters_to", {}).get("1e-08")
        if v:
            return int(v)
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slab_192x192x384")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--exclusion", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--md-steps", type=int, default=10,
                    help="MD-like warm-started steps on the 256x256x512 slab (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling hardware traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              f"supported (multi-GPU z-slab sharding is design only)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 1 << 30, "copy_calibration_bytes_written": 1 << 30,
                          "launches": 3}), flush=True)
        return

    w = make_workload(args.workload, args.exclusion)
    # the timed run instruments only the fine-level smoother (HIP events around
    # each of its launches on the library's stream)
    s = solver_for(w, args.precision, torch, profile=2)
    print(f"# bench: {w.name} {args.precision} exclusion={args.exclusion} steps={args.steps} "
          f"warmup={args.warmup}", file=sys.stderr, flush=True)
    keep = {}
    sec, E, infos, F, prof = run_steps(s, w, args.steps, args.warmup, torch, keep=keep)
    iters = [i["outer_iters"] for i in infos]
    solve_ms = float(np.median([i["t_total_ms"] for i in infos]))
    phases = {k: round(float(np.median([i[k] for i in infos])), 3) for k in ("t_fft_ms", "t_mg_ms", "t_krylov_ms")}
    print(f"# main: {1e3 * sec:.2f} ms/step, iters {iters}, E {E:.12f}, phases {phases}", file=sys.stderr, flush=True)
    err_main = errors_vs_oracle(w.name, E, infos[-1], keep["phi"], F, torch)

    # roofline of the fine-level smoother (the dominant kernel of the wet solve),
    # from the HIP events that each of its launches in the timed steps records
    # at the kernel's start and end (hipExtLaunchKernel)
    roof = None
    dom = prof.get("rbgs_fine")
    smoother_gbs = None
    if dom and dom["ms"] > 0:
        avg_ms = dom["ms"] / dom["launches"]
        per_launch = dom["bytes"] / dom["launches"]
        gbs = per_launch / (avg_ms * 1e-3) / 1e9
        smoother_gbs = round(gbs, 1)
        roof = {"kernel": "k_sweep_band (fine-level red-black Gauss-Seidel sweep on bands of whole rows)", "bound": "hbm",
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic("k_sweep_band<float, 4, *>") if args.precision == "mixed" and w.n == (192, 192, 384) else None,
                "avg_launch_us": round(1e3 * avg_ms, 2), "launches": dom["launches"],
                "algorithmic_bytes_per_launch": per_launch}
    # the headline: the same steps with no instrumentation at all
    s0 = solver_for(w, args.precision, torch, profile=0)
    sec0, _, _, _, _ = run_steps(s0, w, args.steps, args.warmup, torch)
    s0.close()
    print(f"# main, no instrumentation: {1e3 * sec0:.2f} ms/step", file=sys.stderr, flush=True)
    # per-kernel-group breakdown from a separate, fully instrumented short run
    sb = solver_for(w, args.precision, torch, profile=1)
    secb, _, _, _, profb = run_steps(sb, w, 2, 0, torch)
    sb.close()
    kernels = {k: {"ms_per_step": round(v["ms"] / 2, 3), "launches_per_step": v["launches"] / 2,
                   "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in profb.items()}

    extra = {"smoother_instrumented_ms_per_step": round(1e3 * sec, 3),
             "one_pass_split_error_oracle": one_pass_errors()}
    if not args.no_compare:
        other = "fp64" if args.precision == "mixed" else "mixed"
        s2 = solver_for(w, other, torch)
        keep2 = {}
        sec2, E2, inf2, F2, prof2 = run_steps(s2, w, max(2, args.steps // 2), 1, torch, keep=keep2)
        extra[other] = {"steps_per_s": round(1.0 / sec2, 3), "ms_per_step": round(1e3 * sec2, 2),
                        "iters": inf2[-1]["outer_iters"], "energy": E2,
                        "rel_energy_diff_vs_main": abs(E2 - E) / abs(E),
                        "vs_oracle": errors_vs_oracle(w.name, E2, inf2[-1], keep2["phi"], F2, torch)}
        s2.close()
        print(f"# {other}: {1e3 * sec2:.2f} ms/step", file=sys.stderr, flush=True)
        if args.precision == "mixed":
            s4 = solver_for(w, "mixed", torch, fft_fp32=0)
            keep4 = {}
            sec4, E4, inf4, F4, _ = run_steps(s4, w, max(2, args.steps // 2), 1, torch, keep=keep4)
            extra["mixed_fft_fp64"] = {"steps_per_s": round(1.0 / sec4, 3), "ms_per_step": round(1e3 * sec4, 2),
                                       "iters": inf4[-1]["outer_iters"], "energy": E4,
                                       "rel_energy_diff_vs_main": abs(E4 - E) / abs(E),
                                       "vs_oracle": errors_vs_oracle(w.name, E4, inf4[-1], keep4["phi"], F4, torch)}
            s4.close()
            print(f"# mixed with a float64 dry update: {1e3 * sec4:.2f} ms/step", file=sys.stderr, flush=True)
            s6 = solver_for(w, "mixed", torch, krylov_fp16=0)
            keep6 = {}
            sec6, E6, inf6, F6, _ = run_steps(s6, w, max(2, args.steps // 2), 1, torch, keep=keep6)
            extra["mixed_fp32_krylov_basis"] = {
                "steps_per_s": round(1.0 / sec6, 3), "ms_per_step": round(1e3 * sec6, 2),
                "iters": inf6[-1]["outer_iters"], "energy": E6, "rel_energy_diff_vs_main": abs(E6 - E) / abs(E),
                "vs_oracle": errors_vs_oracle(w.name, E6, inf6[-1], keep6["phi"], F6, torch)}
            s6.close()
            print(f"# mixed with a float32 Arnoldi basis: {1e3 * sec6:.2f} ms/step", file=sys.stderr, flush=True)
            s5 = solver_for(w, "mixed", torch, krylov_fp32=0)
            keep5 = {}
            sec5, E5, inf5, F5, _ = run_steps(s5, w, max(2, args.steps // 2), 1, torch, keep=keep5)
            extra["mixed_fp64_krylov_basis"] = {
                "steps_per_s": round(1.0 / sec5, 3), "ms_per_step": round(1e3 * sec5, 2),
                "iters": inf5[-1]["outer_iters"], "energy": E5, "rel_energy_diff_vs_main": abs(E5 - E) / abs(E),
                "phases_ms": {k: round(inf5[-1][k], 2) for k in ("t_fft_ms", "t_mg_ms", "t_krylov_ms")},
                "vs_oracle": errors_vs_oracle(w.name, E5, inf5[-1], keep5["phi"], F5, torch)}
            s5.close()
            print(f"# mixed with a float64 Arnoldi basis: {1e3 * sec5:.2f} ms/step", file=sys.stderr, flush=True)
        we = make_workload(args.workload, not args.exclusion)
        s3 = solver_for(we, args.precision, torch)
        keep3 = {}
        sec3, E3, inf3, F3, _ = run_steps(s3, we, max(2, args.steps // 2), 1, torch, keep=keep3)
        extra["exclusion" if not args.exclusion else "no_exclusion"] = {
            "steps_per_s": round(1.0 / sec3, 3), "ms_per_step": round(1e3 * sec3, 2),
            "iters": inf3[-1]["outer_iters"], "energy": E3, "z_wet": list(we.z_wet),
            "vs_oracle": errors_vs_oracle(we.name, E3, inf3[-1], keep3["phi"], F3, torch)}
        s3.close()
        print(f"# other mode: {1e3 * sec3:.2f} ms/step", file=sys.stderr, flush=True)
        if not args.exclusion:
            extra["coupling_variants"] = coupling_variants(w, args.precision, torch)
            print(f"# coupling variants: {extra['coupling_variants']}", file=sys.stderr, flush=True)

    if not args.no_compare and args.md_steps > 0:
        wb = W.big_slab(exclusion=args.exclusion, tol=1e-8)
        per = md_loop(wb, args.md_steps, torch, args.precision)
        extra["md_256x256x512"] = {"steps": per, "ms_per_step_warm": round(float(np.mean([p["ms"] for p in per[1:]])), 2),
                                   "iters_cold": per[0]["iters"],
                                   "iters_warm_mean": round(float(np.mean([p["iters"] for p in per[1:]])), 2)}
        print(f"# md: {[p['ms'] for p in per]} ms, iters {[p['iters'] for p in per]}", file=sys.stderr, flush=True)

    if not args.no_compare and w.n == (192, 192, 384):
        for ex in (False, True):
            key = "gamma_eps_192x192x384" + ("_excl" if ex else "")
            extra[key] = gamma_steps(torch, ex, precision=args.precision)
            print(f"# {key}: {extra[key]}", file=sys.stderr, flush=True)
        extra["density_eps_192x192x384"] = density_steps(torch, precision=args.precision)
        print(f"# density eps: {extra['density_eps_192x192x384']}", file=sys.stderr, flush=True)
        extra["sixth_order_192x192x384"] = sixth_order_steps(torch, precision=args.precision)
        print(f"# sixth order: {extra['sixth_order_192x192x384']}", file=sys.stderr, flush=True)

    if not args.no_compare:
        extra["hbm_resident_smoother_512"] = hbm_resident_smoother(torch)
        print(f"# smoother 512^3: {extra['hbm_resident_smoother_512']}", file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling(torch)
    if roof:
        roof["copy_ceiling_gbs"] = copy_gbs
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w)
        if "sixth_order_192x192x384" in extra:
            dd = extra["density_eps_192x192x384"]
            gpu_ms = {"gamma_build": extra["gamma_eps_192x192x384"]["eps_build_ms"],
                      "density": round(dd["eps_build_ms"] + dd["v_eps_ms"], 3),
                      "sixth_apply": extra["sixth_order_192x192x384"]["apply_ms"]}
            extra["oracle_beside_widened"] = cpu_widened(gpu_ms)
            print(f"# oracle beside widened paths: {extra['oracle_beside_widened']}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(1.0 / sec0, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * sec0, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32+f16" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {len(w.q)}-atom TiO2-like slab, {w.L[0]}x{w.L[1]}x{w.L[2]} A cell, "
                               f"{'exclusion rule' if args.exclusion else 'literal product-erf eps'}, "
                               f"dry z<{w.z_wet[0]:.2f} A, tol 1e-8, cold start",
                   "grid": list(w.n), "precision": args.precision, "step": "build_eps+build_rho+solve+adjoint+forces",
                   "preconditioner": "f32 (dry FFT update and wet multigrid)" if args.precision == "mixed" else "f64",
                   "krylov_basis": ("V in f16 (f32 in a solve's first cycle and after one that cut the residual over 100x) and Z "
                                    "in f32 storage, f64 products and residual" if args.precision == "mixed" else "f64")},
        "solve_iters": iters[-1], "solve_ms_median": round(solve_ms, 3), "solve_phases_ms": phases,
        "energy": E, "vs_oracle": err_main,
        "smoother_hbm_gbs": smoother_gbs, "kernels": kernels,
        "roofline": roof, "cpu_baseline": cpu, "compare": extra,
    }
    print(json.dumps(line), flush=True)
    s.close()


if __name__ == "__main__":
    main()
