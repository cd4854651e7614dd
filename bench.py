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


def run_steps(s, w, steps, warmup, torch):
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
    return (t1 - t0) / steps, E, infos, F, prof


def solver_for(w, precision, torch, profile=0, **extra):
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(w.n, w.L, **w.solver_opts(tol=1e-8, precision=1 if precision == "mixed" else 0, profile=profile,
                                         **extra))
    return s


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary,
    if that summary was taken on the current source of the kernel, else None."""
    import hashlib
    src = os.path.join(ROOT, "paper_0904_4887_amd", "csrc", "kern_grid.hip")
    summ = os.path.join(ROOT, "profiles", "sweep_fused_slab_192x192x384_mixed.md")
    if not (os.path.exists(src) and os.path.exists(summ)):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    vals = {}
    for line in open(summ):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kern_grid.hip sha256") != digest or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, golden_iters):
    """The FP64 oracle's solve, timed on a bounded sample: a few PCG iterations
    of the full-size problem, scaled by the iteration count the oracle needs
    for a 1e-8 residual on this workload."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        eps = O.eps_erf(w.n, w.L, w.xyz, w.radius, w.eps_params, nodes=np.arange(0, w.N, 997))
        del eps
        rho = np.zeros((w.n[2], w.n[1], w.n[0]))
        rho[::7, ::5, ::3] = 1.0
        eps = np.ones_like(rho)
        its = 3
        t0 = time.perf_counter()
        O.solve(rho, eps, w.h, tol=1e-300, max_iter=its)
        dt = (time.perf_counter() - t0) / its
    n_iters = golden_iters
    t_solve = dt * n_iters
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{its} PCG iterations of the oracle's full-grid {w.n[0]}x{w.n[1]}x{w.n[2]} solve "
                      f"({dt:.2f} s each), scaled by its {n_iters} iterations to a 1e-8 residual on this "
                      f"workload; eps/rho builds and forces not included (NumPy, one thread)"}


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
    s.set_grid(w.n, w.L, **w.solver_opts(tol=1e-8, precision=1 if precision == "mixed" else 0))
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
    w.opts = dict(scaled_dry=1, order=6)
    s = solver_for(w, precision, torch)
    sec, E, infos, _, _ = run_steps(s, w, steps, warmup, torch)
    x = s.empty().normal_()
    t_apply = gpu_wall_ms(torch, lambda: s.apply_operator(x), reps=5)
    s.close()
    return {"ms_per_step": round(1e3 * sec, 2), "steps_per_s": round(1.0 / sec, 3),
            "iters": [i["outer_iters"] for i in infos], "energy": E, "background": infos[-1]["background"],
            "opts": w.opts, "apply_ms": t_apply}


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
    sec, E, infos, F, prof = run_steps(s, w, args.steps, args.warmup, torch)
    iters = [i["outer_iters"] for i in infos]
    solve_ms = float(np.median([i["t_total_ms"] for i in infos]))
    print(f"# main: {1e3 * sec:.2f} ms/step, iters {iters}, E {E:.12f}", file=sys.stderr, flush=True)

    # roofline of the fine-level smoother (the dominant kernel of the wet solve),
    # from the HIP events recorded around each of its launches in the timed steps
    roof = None
    dom = prof.get("rbgs_fine")
    smoother_gbs = None
    if dom and dom["ms"] > 0:
        avg_ms = dom["ms"] / dom["launches"]
        per_launch = dom["bytes"] / dom["launches"]
        gbs = per_launch / (avg_ms * 1e-3) / 1e9
        smoother_gbs = round(gbs, 1)
        roof = {"kernel": "k_sweep_fused (fine-level red-black Gauss-Seidel sweep)", "bound": "hbm",
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic("k_sweep_fused<float, 4, *>") if args.precision == "mixed" and w.n == (192, 192, 384) else None,
                "avg_launch_us": round(1e3 * avg_ms, 2), "launches": dom["launches"],
                "algorithmic_bytes_per_launch": per_launch}
    # per-kernel-group breakdown from a separate, fully instrumented short run
    sb = solver_for(w, args.precision, torch, profile=1)
    secb, _, _, _, profb = run_steps(sb, w, 2, 0, torch)
    sb.close()
    kernels = {k: {"ms_per_step": round(v["ms"] / 2, 3), "launches_per_step": v["launches"] / 2,
                   "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in profb.items()}

    extra = {}
    if not args.no_compare:
        other = "fp64" if args.precision == "mixed" else "mixed"
        s2 = solver_for(w, other, torch)
        sec2, E2, inf2, _, prof2 = run_steps(s2, w, max(2, args.steps // 2), 1, torch)
        extra[other] = {"steps_per_s": round(1.0 / sec2, 3), "ms_per_step": round(1e3 * sec2, 2),
                        "iters": inf2[-1]["outer_iters"], "energy": E2,
                        "rel_energy_diff_vs_main": abs(E2 - E) / abs(E)}
        s2.close()
        print(f"# {other}: {1e3 * sec2:.2f} ms/step", file=sys.stderr, flush=True)
        if args.precision == "mixed":
            s4 = solver_for(w, "mixed", torch, fft_fp32=1)
            sec4, E4, inf4, _, _ = run_steps(s4, w, max(2, args.steps // 2), 1, torch)
            extra["mixed_fft_fp32"] = {"steps_per_s": round(1.0 / sec4, 3), "ms_per_step": round(1e3 * sec4, 2),
                                       "iters": inf4[-1]["outer_iters"], "energy": E4,
                                       "rel_energy_diff_vs_main": abs(E4 - E) / abs(E)}
            s4.close()
            print(f"# mixed with float32 dry update: {1e3 * sec4:.2f} ms/step", file=sys.stderr, flush=True)
        we = make_workload(args.workload, not args.exclusion)
        s3 = solver_for(we, args.precision, torch)
        sec3, E3, inf3, _, _ = run_steps(s3, we, max(2, args.steps // 2), 1, torch)
        extra["exclusion" if not args.exclusion else "no_exclusion"] = {
            "steps_per_s": round(1.0 / sec3, 3), "ms_per_step": round(1e3 * sec3, 2),
            "iters": inf3[-1]["outer_iters"], "energy": E3, "z_wet": list(we.z_wet)}
        s3.close()
        print(f"# other mode: {1e3 * sec3:.2f} ms/step", file=sys.stderr, flush=True)

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
        gi = golden_iters(w.name if not args.exclusion else w.name)
        if gi is None:
            gi = 130
        cpu = cpu_baseline(w, gi)
        if "sixth_order_192x192x384" in extra:
            dd = extra["density_eps_192x192x384"]
            gpu_ms = {"gamma_build": extra["gamma_eps_192x192x384"]["eps_build_ms"],
                      "density": round(dd["eps_build_ms"] + dd["v_eps_ms"], 3),
                      "sixth_apply": extra["sixth_order_192x192x384"]["apply_ms"]}
            extra["oracle_beside_widened"] = cpu_widened(gpu_ms)
            print(f"# oracle beside widened paths: {extra['oracle_beside_widened']}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(1.0 / sec, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * sec, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {len(w.q)}-atom TiO2-like slab, {w.L[0]}x{w.L[1]}x{w.L[2]} A cell, "
                               f"{'exclusion rule' if args.exclusion else 'literal product-erf eps'}, "
                               f"dry z<{w.z_wet[0]:.2f} A, tol 1e-8, cold start",
                   "grid": list(w.n), "precision": args.precision, "step": "build_eps+build_rho+solve+adjoint+forces"},
        "solve_iters": iters[-1], "solve_ms_median": round(solve_ms, 3), "energy": E,
        "smoother_hbm_gbs": smoother_gbs, "kernels": kernels,
        "roofline": roof, "cpu_baseline": cpu, "compare": extra,
    }
    print(json.dumps(line), flush=True)
    s.close()


if __name__ == "__main__":
    main()
