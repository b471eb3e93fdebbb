#!/usr/bin/env python3
"""Throughput of the KFBI hot path on one MI355X: grid unknowns per second per K_D apply.

Workload: the 2D modified Helmholtz problem (kappa = 1) on the star
r(t) = 0.6 + 0.15 sin 5t in the box [-1.2, 1.2]^2, 2048 x 2048 grid
(2047^2 unknowns), 1024 equal-arc-length boundary samples, synthetic data.
One step is one GMRES iteration on the boundary density (Alg. 5): a K_D apply
(jumps + correction, sparse fast solve, interpolation: Alg. 1-4) plus the
device-side Gram-Schmidt / Givens update.  The steps run back to back on the
device with no convergence stop, so the timed work is fixed.

The timed region replays the captured GMRES steps (the production path).  A
second region of the same length launches the same steps one by one, each
apply kernel recording a start and an end HIP event from its own dispatch packet
on the library's stream: the dominant kernel's average duration (roofline) and
the per-stage times come from there.  The roofline's ``traffic`` is the HBM
bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, null when
that summary was taken on other kernel sources.

Also reported, outside the timed region:
  solve     one full Dirichlet solve of the workload (FP64), error vs exact;
  convergence  full FP64 solves of the star workload at 512^2, 1024^2 and 2048^2:
            L-infinity error against the exact solution and the observed order;
  three_d   the ellipsoid Poisson problem at 64^3 and 128^3: GMRES steps per
            second and a full solve with its error against the exact solution;
  mixed     the circle r = 0.8, M = N, kappa = 1 problem at the same grid:
            full solves with FP64 and with FP32-refined grid solves, their
            times and the L-infinity difference between the two;
  serving   a seeded stream of mixed-size requests through the continuous
            batching scheduler: solves/s at saturation and p50/p99 latency at
            50 % and 90 % of that rate (``--mode serving`` runs a longer stream).
The CPU baseline is the FP64 oracle timed on a bounded sample of the same
workload (rank 0, one GPU only).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X, dense FP64 vector
HBM_PEAK_BYTES = 8.0e12             # MI355X HBM3E, bytes/s

# HBM traffic of k_modes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by
# what the same counters read for a plain copy (``--mode copy``); valid only for
# the kernel sources, grid and launch shape it was taken with
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "k_modes_star2048_counters.md")
KERNEL_SOURCES = ("device.h", "kernels.h", "kernels.hip", "api.hip", "plan.cpp")


def modes_flops(n_grid: int, n_irr: int, m: int) -> float:
    """Algorithmic FP64 flops of one sparse fast-solve launch (k_modes).

    Per sine mode (n-1 of them): 2 flops per irregular node for the sparse sine
    sum, 14 flops per grid point for the two chunked recurrences with their
    carry fixes and the rank-one fix, 16 flops per boundary sample for the
    weighted six-point gather.
    """
    return (n_grid - 1) * (2.0 * n_irr + 14.0 * n_grid + 16.0 * m)


def kernel_source_hash() -> str:
    """sha256 over the sources that decide what k_modes reads and writes."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2404_15249_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(n_grid: int, modes_per_group: int):
    """HBM bytes per k_modes launch from the committed counter summary, or None
    when it is missing or was taken on other kernel sources, grid or shape."""
    try:
        with open(COUNTER_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    try:
        rec = json.loads(m.group(1))
    except ValueError:
        return None
    if (rec.get("source_sha256") != kernel_source_hash() or rec.get("grid") != n_grid
            or rec.get("modes_per_group") != modes_per_group):
        return None
    return float(rec["hbm_bytes_per_launch"])


def copy_calibration() -> dict:
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = 32 << 20
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"mode": "copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8, "copies": 5}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_workers() -> int:
    """Threads this process may use on the host: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of the machine it was given)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def _time_oracle_applies(plan, phi, kappa, seconds: float, workers: int):
    """K_D applies of the oracle, back to back for about `seconds`, with scipy's
    FFT given `workers` threads (the oracle's own code is unchanged)."""
    from scipy import fft as sfft
    from oracle import kfbi_oracle as O
    with sfft.set_workers(workers):
        O.apply_KD(plan, phi, kappa)                    # warm-up
        t0 = time.perf_counter()
        k = 0
        while True:
            O.apply_KD(plan, phi, kappa)
            k += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return k, time.perf_counter() - t0


def cpu_baseline(p, seconds: float):
    """The oracle's K_D apply on the same workload, timed on the host cores:
    once with the FFTs on every thread the process may use (the reported
    baseline), once on one thread."""
    from oracle import kfbi_oracle as O
    import synth
    plan = O.build_plan(p.xy, p.n, p.lo, p.hi)
    phi = synth.smooth_density(plan.M, 1234)
    unknowns = (p.n - 1) ** 2
    nw = host_workers()
    legs = {}
    for w in (nw, 1):
        k, dt = _time_oracle_applies(plan, phi, p.kappa, seconds, w)
        legs[w] = {"value": unknowns * k / dt, "applies": k, "seconds": dt}
    top = legs[nw]
    return {"value": top["value"], "unit": "grid unknowns/s", "cores": nw, "kind": "oracle",
            "sample": f"{top['applies']} oracle K_D applies (scipy DST-I with workers={nw}, NumPy) on the same "
                      f"{p.n}^2 star problem, {top['seconds']:.1f} s on {cpu_model()}",
            "one_core": {"value": legs[1]["value"], "unit": "grid unknowns/s", "cores": 1,
                         "sample": f"{legs[1]['applies']} applies with workers=1, {legs[1]['seconds']:.1f} s"}}


def mixed_precision(ctx, n: int) -> dict:
    """Full solves of the circle problem (r = 0.8, M = N, kappa = 1, u = e^x sin y)
    with FP64 and with FP32-refined grid solves."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    p = synth.circle_problem(n=n, m=n, kappa=1.0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    f, fg, g = dev(p.f_grid), dev(p.f_gamma), dev(p.g)
    c = p.lo + np.arange(p.n + 1) * p.h
    X, Y = np.meshgrid(c, c, indexing="xy")
    exact = p.exact.u(X, Y)
    res = {"workload": f"circle r=0.8, {n}x{n} grid, M={n}, kappa=1, u=e^x sin y, GMRES tol 1e-12"}
    base = None
    for prec in ("fp64", "fp32"):
        prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12, precision=prec, refine_steps=1)
        prob.solve(f, fg, g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 3
        for _ in range(reps):
            u, ug, phi, it, rel, conv = prob.solve(f, fg, g)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / reps
        # the grid solve alone (volume potential form), averaged
        zero = torch.zeros(prob.M, dtype=torch.float64, device="cuda:0")
        prob.interface_solve(zero, f, fg)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            prob.interface_solve(zero, f, fg)
        torch.cuda.synchronize()
        gs_ms = 1e3 * (time.perf_counter() - t) / 10
        uh = u.cpu().numpy()
        mask = prob.mask()
        entry = {"solve_ms": ms, "interface_solve_ms": gs_ms, "gmres_iters": it, "converged": conv,
                 "linf_err_vs_exact": float(np.max(np.abs(uh - exact)[mask]))}
        if base is None:
            base = uh
        else:
            entry["linf_diff_vs_fp64_path"] = float(np.max(np.abs(uh - base)[mask]))
            entry["refine_steps"] = 1
        res[prec] = entry
        prob.close()
    return res


def dense_solves(ctx, n: int, calls: int = 20) -> dict:
    """The dense path alone: interface solves (volume potential form: right-hand
    side with its corrections, the grid solve, interpolation at the samples) of
    the circle problem (r = 0.8, M = N, kappa = 1) with FP64 and with FP32 grid
    solves (0 and 1 refinement steps), timed with events on the library's stream.
    One FP64 grid solve is two column sine transforms (``k_dst_cols``, in place)
    around the row solves; each transform reads N - 1 rows and writes N rows of
    N doubles."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    p = synth.circle_problem(n=n, m=n, kappa=1.0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    f, fg = dev(p.f_grid), dev(p.f_gamma)
    res = {"mode": "dense", "workload": f"circle r=0.8, {n}x{n} grid, M={n}, kappa=1: interface solves",
           "grid": n, "calls": calls, "transform_bytes_per_launch": 8 * (2 * n - 1) * n}
    base = None
    for name, prec, rs in (("fp64", "fp64", 1), ("fp32_refine0", "fp32", 0), ("fp32_refine1", "fp32", 1)):
        prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12, precision=prec, refine_steps=rs)
        zero = torch.zeros(prob.M, dtype=torch.float64, device="cuda:0")
        _, vz = prob.interface_solve(zero, f, fg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            prob.interface_solve(zero, f, fg)
        e1.record()
        torch.cuda.synchronize()
        entry = {"interface_solve_us": 1e3 * e0.elapsed_time(e1) / calls, "dst_tile": prob.tiles()["dst_cols"]}
        v = vz.cpu().numpy()
        if base is None:
            base = v
        else:
            entry["linf_diff_vs_fp64_at_samples"] = float(np.max(np.abs(v - base)))
        res[name] = entry
        prob.close()
    return res


def convergence(ctx, sizes=(512, 1024, 2048)) -> dict:
    """Full FP64 solves of the star workload (kappa = 1, M = N/2,
    u = sin(pi x) cos(pi y) + x^2) at several grids: L-infinity error against the
    exact solution on the grid nodes in Omega and on Gamma, and the observed order."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    rows = []
    for n in sizes:
        p = synth.star_problem(n=n, kappa=1.0)
        prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-10)
        u, ug, phi, it, rel, conv = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        c = p.lo + np.arange(p.n + 1) * p.h
        X, Y = np.meshgrid(c, c, indexing="xy")
        mask = prob.mask()
        e_grid = float(np.max(np.abs(u.cpu().numpy() - p.exact.u(X, Y))[mask]))
        e_gam = float(np.max(np.abs(ug.cpu().numpy() - p.exact.u(p.xy[:, 0], p.xy[:, 1]))))
        rows.append({"n": n, "samples": prob.M, "gmres_iters": it, "converged": conv,
                     "linf_err_grid": e_grid, "linf_err_gamma": e_gam})
        prob.close()
    for a, b in zip(rows, rows[1:]):
        b["order_grid"] = float(np.log2(a["linf_err_grid"] / b["linf_err_grid"]))
    return {"workload": "star r=0.6+0.15 sin 5t, kappa=1, M=N/2, u=sin(pi x)cos(pi y)+x^2, GMRES tol 1e-10",
            "rows": rows}


def three_d(ctx, sizes=(64, 128), steps: int = 200) -> dict:
    """The ellipsoid (0.9, 0.7, 0.5) Poisson problem, u = e^(x+y+z): per size,
    graphed GMRES steps with no convergence stop (grid unknowns per second per
    step), and a full FP64 solve to 1e-10 with its error against the exact
    solution."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    rows = []
    for n in sizes:
        pr = synth.ellipsoid_problem(n=n)
        prob = kfbi.Problem3(ctx, n, pr.axes, kappa=pr.kappa, tol=1e-10, max_iter=1500)
        pts, _ = prob.points()
        fg, g = pr.boundary_data(pts)
        rhs = dev(g)
        prob.gmres(rhs, tol=0.0, max_iter=16)                  # warm-up (records the step graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.gmres(rhs, tol=0.0, max_iter=steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f_grid, fgd, gd = dev(pr.f_grid), dev(fg), dev(g)
        prob.solve(f_grid, fgd, gd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, ug, phi, it, rel, conv = prob.solve(f_grid, fgd, gd)
        torch.cuda.synchronize()
        solve_ms = 1e3 * (time.perf_counter() - t1)
        err = float(np.max(np.abs(u.cpu().numpy() - pr.exact_grid())[prob.mask()]))
        unknowns = (n - 1) ** 3
        rows.append({"n": n, "unknowns": unknowns, "control_points": prob.M, "irregular_nodes": prob.I,
                     "us_per_step": 1e6 * dt / steps, "unknowns_per_s": unknowns * steps / dt,
                     "solve_ms": solve_ms, "gmres_iters": it, "converged": conv, "linf_err_vs_exact": err})
        prob.close()
    for a, b in zip(rows, rows[1:]):
        b["order"] = float(np.log2(a["linf_err_vs_exact"] / b["linf_err_vs_exact"]))
    return {"workload": "ellipsoid (0.9,0.7,0.5) in [-1.2,1.2]^3, kappa=0, u=e^(x+y+z), 7-point grid, "
                        "control points = grid-edge crossings; step = one GMRES iteration", "rows": rows}


def neumann(ctx, n: int = 2048, steps: int = 400, sizes=(512, 1024, 2048), cpu: bool = True) -> dict:
    """The Neumann problem d_n u = g_n on the star workload (kappa = 1, M = N/2,
    u = sin(pi x) cos(pi y) + x^2): graphed GMRES steps on K_N (grid unknowns per
    second per step, as the headline's K_D step), a full FP64 solve to 1e-10,
    and the L-infinity error against the exact solution at several grids."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    p = synth.star_neumann_problem(n=n, kappa=1.0)
    prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, restart=50)
    rhs = dev(p.g_n)
    prob.gmres_neumann(rhs, tol=0.0, max_iter=50)              # warm-up (records the step graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters, _, _, _ = prob.gmres_neumann(rhs, tol=0.0, max_iter=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert iters == steps
    prob.close()
    unknowns = (n - 1) ** 2
    res = {"workload": f"Neumann problem on the star r=0.6+0.15 sin 5t, kappa=1, M=N/2, "
                       f"u=sin(pi x)cos(pi y)+x^2; step = one GMRES iteration on K_N at {n}x{n}",
           "us_per_step": 1e6 * dt / steps, "unknowns_per_s": unknowns * steps / dt}
    if cpu:
        # the oracle's K_N apply on the same problem, beside it (one host core)
        from oracle import kfbi_oracle as O
        plan = O.build_plan(p.xy, p.n, p.lo, p.hi)
        psi = synth.smooth_density(plan.M, 5)
        O.apply_KN(plan, psi, p.kappa)
        t0 = time.perf_counter()
        for _ in range(3):
            O.apply_KN(plan, psi, p.kappa)
        res["cpu_oracle"] = {"us_per_apply": 1e6 * (time.perf_counter() - t0) / 3, "cores": 1, "kind": "oracle",
                             "sample": f"3 oracle K_N applies at {n}x{n}"}
    rows = []
    for m in sizes:
        q = synth.star_neumann_problem(n=m, kappa=1.0)
        pr = kfbi.Problem(ctx, q.xy, q.n, q.kappa, tol=1e-10)
        args = (dev(q.f_grid), dev(q.f_gamma), dev(q.g_n))
        pr.solve_neumann(*args)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, ug, dn, psi, it, rel, conv = pr.solve_neumann(*args)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1)
        c = q.lo + np.arange(q.n + 1) * q.h
        X, Y = np.meshgrid(c, c, indexing="xy")
        mask = pr.mask()
        rows.append({"n": m, "samples": pr.M, "solve_ms": ms, "gmres_iters": it, "converged": conv,
                     "linf_err_grid": float(np.max(np.abs(u.cpu().numpy() - q.exact.u(X, Y))[mask])),
                     "linf_err_trace": float(np.max(np.abs(ug.cpu().numpy() - q.g))),
                     "linf_dn_minus_g_n": float(np.max(np.abs(dn.cpu().numpy() - q.g_n)))})
        pr.close()
    for a, b in zip(rows, rows[1:]):
        b["order_grid"] = float(np.log2(a["linf_err_grid"] / b["linf_err_grid"]))
    res["rows"] = rows
    return res


# Table 2: the paper's GPU times in seconds of the Example 1 solve with each
# outer iteration, on its own machine (context only)
PAPER_ITER_GPU_S = {"richardson": {512: 0.19, 1024: 0.27, 2048: 0.66, 4096: 1.65},
                    "gmres": {512: 0.13, 1024: 0.16, 2048: 0.18, 4096: 0.25},
                    "bicgstab": {512: 0.45, 1024: 0.45, 2048: 0.63, 4096: 1.01}}


def iterations(ctx, sizes=(512, 1024, 2048, 4096), cpu: bool = True) -> dict:
    """Table 2: the Dirichlet problem of Example 1 (Laplace on the circle r = 1 in
    (-1.2, 1.2)^2, u = e^x cos y + e^y sin x, M = n samples) solved with GMRES,
    BiCGSTAB and Richardson (gamma = 1) to the paper's tolerance 1e-8: the time
    of one full solve (volume potential, iteration, final solve) and the
    iteration counts."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    rows = []
    for n in sizes:
        p = synth.make_problem(f"circle r=1 n={n}", synth.circle_points(n, 1.0), n, 0.0, synth.PAPER_EX1)
        prob = kfbi.Problem(ctx, p.xy, p.n, 0.0, tol=1e-8)
        args = (dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        c = p.lo + np.arange(n + 1) * p.h
        X, Y = np.meshgrid(c, c, indexing="xy")
        exact = p.exact.u(X, Y)
        mask = prob.mask()
        for method in ("gmres", "bicgstab", "richardson"):
            prob.solve_method(method, *args)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, ug, phi, it, rel, conv = prob.solve_method(method, *args)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            rows.append({"n": n, "method": method, "solve_ms": ms, "iters": it, "relres": rel, "converged": conv,
                         "linf_err": float(np.max(np.abs(u.cpu().numpy() - exact)[mask])),
                         "paper_gpu_s": PAPER_ITER_GPU_S[method][n]})
        prob.close()
    out = {}
    if cpu:
        # the oracle's solves of the smallest size with each method, beside them (one host core)
        from oracle import kfbi_oracle as O
        n = sizes[0]
        p = synth.make_problem(f"circle r=1 n={n}", synth.circle_points(n, 1.0), n, 0.0, synth.PAPER_EX1)
        ms = {}
        for method in ("gmres", "bicgstab", "richardson"):
            t0 = time.perf_counter()
            O.solve_bvp(p.xy, p.n, p.lo, p.hi, 0.0, p.f_grid, p.f_gamma, p.g, tol=1e-8, method=method)
            ms[method] = 1e3 * (time.perf_counter() - t0)
        out["cpu_oracle"] = {"solve_ms": ms, "cores": 1, "kind": "oracle", "sample": f"one oracle solve per method at {n}x{n}"}
    return {**out, "workload": "Example 1: Laplace on the circle r=1 in (-1.2,1.2)^2, u=e^x cos y+e^y sin x, M=n, "
                        "tol 1e-8; iters: GMRES and Richardson count K_D applies, BiCGSTAB its iterations "
                        "(two applies each); paper_gpu_s is the paper's own machine (context)",
            "rows": rows}


# Table of Example 3 (Neumann row): the paper's GPU times in seconds on its own
# machine, for context only
PAPER_GS_GPU_S = {128: 0.40, 256: 1.04, 512: 3.29, 1024: 12.07}


def gray_scott(ctx, grid_steps=((128, 8), (256, 16), (512, 32), (1024, 64)), T: float = 1.0, cpu: bool = True) -> dict:
    """Example 3: Gray-Scott on the disk r = 1.8 in (-2, 2)^2 with the paper's
    parameters, Strang splitting, GMRES tol 1e-8, at the grid sizes and step
    counts of the paper's table (final time T = 1).  The timed region is the time
    stepping alone, with the state resident on the device."""
    import torch
    import synth
    from paper_2404_15249_amd import kfbi
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    lo, hi = synth.GS_LO, synth.GS_HI
    rows = []
    for n, steps in grid_steps:
        xy = synth.gray_scott_samples(n)
        dt = T / steps
        mask = kfbi.Problem(ctx, xy, n, 1.0, lo=lo, hi=hi).mask()
        c = lo + np.arange(n + 1) * (hi - lo) / n
        X, Y = np.meshgrid(c, c, indexing="xy")
        u0, v0 = synth.gray_scott_initial(X, Y)
        ug0, vg0 = synth.gray_scott_initial(xy[:, 0], xy[:, 1])
        init = (dev(np.where(mask, u0, 0.0)), dev(np.where(mask, v0, 0.0)), dev(ug0), dev(vg0))
        gs = kfbi.GrayScott(ctx, xy, n, dt, lo=lo, hi=hi, tol=1e-8)
        gs.set_state(*init)
        gs.step(1)                                   # warm-up (first launches, allocations)
        gs.set_state(*init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs.step(steps)
        torch.cuda.synchronize()
        run_s = time.perf_counter() - t0
        u, v, ug, vg = [t.cpu().numpy() for t in gs.state()]
        info = gs.info()
        gs.close()
        row = {"n": n, "steps": steps, "dt": dt, "samples": int(xy.shape[0]), "run_s": run_s,
               "ms_per_step": 1e3 * run_s / steps, "gmres_iters": info["gmres_iters"],
               "u_max": float(u[mask].max()), "u_min": float(u[mask].min()), "v_max": float(v[mask].max()),
               "u_trace_max": float(ug.max())}
        if n in PAPER_GS_GPU_S:
            row["paper_gpu_s"] = PAPER_GS_GPU_S[n]
            row["paper_gpu_s_over_this"] = PAPER_GS_GPU_S[n] / run_s
        rows.append(row)
    out = {}
    if cpu:
        # the oracle's Strang steps on the smallest configuration, beside it (one host core)
        from oracle import gray_scott as G
        from oracle import kfbi_oracle as O
        n, steps = grid_steps[0]
        xy = synth.gray_scott_samples(n)
        plan = O.build_plan(xy, n, lo, hi)
        st = G.initial_state(plan, synth.gray_scott_initial)
        t0 = time.perf_counter()
        G.run(plan, st, T / steps, steps, synth.GrayScottParams(), tol=1e-8)
        out["cpu_oracle"] = {"ms_per_step": 1e3 * (time.perf_counter() - t0) / steps, "cores": 1, "kind": "oracle",
                             "sample": f"{steps} oracle steps at {n}x{n} (T = {T})"}
    return {**out, "workload": "Gray-Scott (Example 3): disk r=1.8 in (-2,2)^2, gamma=0.024, kill=0.06, eps0=0.01, "
                        "eps1=0.008, eps2=0.004, T=1, Strang splitting (RK4 reaction half steps, Crank-Nicolson "
                        "diffusion as two warm-started Neumann solves per step), GMRES tol 1e-8; "
                        "paper_gpu_s is the paper's own machine (context)",
            "rows": rows}


def run_stream(ctx, reqs, budget_gib: float = 64.0, max_slots: int = 32, time_scale: float = 1.0, keep_ids=(),
               label: str = ""):
    import synth
    from paper_2404_15249_amd.serving import GpuExecutor, Scheduler, summarize
    ex = GpuExecutor(ctx, max_slots=max_slots, m_max=8192, budget_bytes=0,
                     make_spec=lambda r: synth.serving_spec(r.seed, r.n), tol=1e-10, keep_ids=keep_ids)
    sch = Scheduler(ex, int(budget_gib * (1 << 30)), max_slots, steps_per_poll=8, prepare_workers=8,
                    prepare_ahead=16, keep_results=True)
    recs, span = sch.run(reqs, time_scale=time_scale)
    out = summarize(recs, span)
    solved = [r for r in recs if not r.rejected]
    flagged = [r for r in solved if r.result["under_resolved"]]
    out["under_resolved"] = len(flagged)
    out["resolved_converged"] = sum(r.converged for r in solved if not r.result["under_resolved"])
    out["resolved"] = len(solved) - len(flagged)
    out["peak_live"] = sch.peak_live
    out["peak_reserved_gib"] = sch.peak_reserved / (1 << 30)
    # the byte model of a dense-formulation solve: (iterations + 2) applies of
    # 48 B per grid unknown (three read+write passes), summed over the solves
    model = sum((r.iters + 2) * 48.0 * (r.n - 1) ** 2 for r in solved)
    out["byte_model_gbps"] = model / span / 1e9
    out["byte_model_frac_of_hbm"] = model / span / HBM_PEAK_BYTES
    ex.batch.close()
    kept = {r.rid: r.result for r in solved if r.result and "u_host" in r.result}
    print(f"serving {label}: {len(solved)} solved in {span:.1f} s ({out['solves_per_s']:.1f}/s), "
          f"p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    return out, kept


def oracle_check(kept, stream) -> dict:
    """The served solutions of a seeded subsample against FP64 oracle solves of
    the same requests: L-infinity over the grid nodes in Omega and the trace."""
    import synth
    from oracle import kfbi_oracle as O
    rows = []
    for rid in sorted(kept):
        _, n, seed = stream[rid]
        p = synth.serving_request(seed, n)
        t0 = time.perf_counter()
        ref = O.solve_bvp(p.xy, p.n, p.lo, p.hi, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-12)
        plan = O.build_plan(p.xy, p.n, p.lo, p.hi)
        e_grid = float(np.max(np.abs(kept[rid]["u_host"] - ref.u_grid)[plan.inside]))
        e_gam = float(np.max(np.abs(kept[rid]["u_gamma_host"] - ref.u_gamma)))
        rows.append({"request": rid, "n": n, "linf_grid": e_grid, "linf_trace": e_gam,
                     "oracle_s": time.perf_counter() - t0})
        print(f"oracle check: request {rid} n={n}: Linf grid {e_grid:.2e} trace {e_gam:.2e}", file=sys.stderr,
              flush=True)
    worst = max([max(r["linf_grid"], r["linf_trace"]) for r in rows], default=0.0)
    return {"requests": len(rows), "worst_linf": worst, "within_1e-6": worst <= 1e-6, "rows": rows}


def oracle_subsample(stream, k: int, seed: int):
    """A seeded choice of k resolved requests for the oracle check, weighted
    toward the smaller grids the host solves quickly (at most one 2048^2)."""
    import synth
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(stream))
    quota = {256: (k + 2) // 3, 512: (k + 2) // 3, 1024: max(1, k // 5), 2048: 1}
    out = []
    for i in order:
        _, n, s = stream[int(i)]
        if quota.get(n, 0) > 0 and not synth.serving_spec(s, n).under_resolved:
            quota[n] -= 1
            out.append(int(i))
        if len(out) >= k:
            break
    return out


def serving(ctx, n_requests: int, seed: int, oracle_requests: int = 0) -> dict:
    """Saturation throughput, then Poisson arrivals at 50 % and 90 % of it;
    with oracle_requests > 0 a seeded subsample of the saturation run is
    checked against the FP64 oracle."""
    import synth
    from paper_2404_15249_amd.serving import Request
    stream = synth.serving_stream(n_requests, seed=seed, qps=1.0)
    keep = oracle_subsample(stream, oracle_requests, seed + 1) if oracle_requests > 0 else ()
    sat, kept = run_stream(ctx, [Request(i, 0.0, n, s) for i, (_, n, s) in enumerate(stream)], keep_ids=keep,
                           label="saturation")
    rate = sat["solves_per_s"]
    res = {"requests": n_requests, "seed": seed, "sizes": "256/512/1024/2048 with p=.4/.3/.2/.1",
           "tol": 1e-10, "saturation": sat}
    for frac in (0.5, 0.9):
        qps = frac * rate
        # the stream's arrival times are drawn at 1 request/s: stretch them to the target rate
        reqs = [Request(i, t, n, s) for i, (t, n, s) in enumerate(stream)]
        r, _ = run_stream(ctx, reqs, time_scale=1.0 / qps, label=f"{int(frac * 100)}% load")
        res[f"at_{int(frac * 100)}pct"] = dict(r, qps=qps)
    if kept:
        res["oracle_check"] = oracle_check(kept, stream)
    return res


def serving_line(ctx, args) -> dict:
    s = serving(ctx, args.serving_requests, args.serving_seed, args.oracle_requests)
    return {"metric": "solves/s (p99 latency beside)", "value": s["saturation"]["solves_per_s"],
            "unit": "solves/s", "n_gpus": 1, "steps": args.serving_requests, "warmup": 0,
            "ms_per_step": 1e3 / max(s["saturation"]["solves_per_s"], 1e-9), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{args.serving_requests} seeded Dirichlet solve requests, random stars "
                                   "r=0.6+a sin(k t), grids 256..2048, kappa~U(0,10), GMRES tol 1e-10"},
            "serving": s}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=2048, help="grid intervals per axis")
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--mixed", choices=["on", "off"], default="on")
    ap.add_argument("--convergence", choices=["on", "off"], default="on")
    ap.add_argument("--three-d", choices=["on", "off"], default="on")
    ap.add_argument("--neumann", choices=["on", "off"], default="on")
    ap.add_argument("--gray-scott", choices=["on", "off"], default="on")
    ap.add_argument("--iterations", choices=["on", "off"], default="on")
    ap.add_argument("--serving-requests", type=int, default=300)
    ap.add_argument("--serving-seed", type=int, default=2404)
    ap.add_argument("--oracle-requests", type=int, default=0,
                    help="--mode serving: served requests checked against the FP64 oracle")
    ap.add_argument("--mode", choices=["apply", "serving", "copy", "dense", "3d", "neumann", "gray_scott", "iterations"],
                    default="apply",
                    help="serving: only the request stream (metric solves/s), e.g. with --serving-requests 10000; "
                         "copy: a 256 MiB device copy to calibrate the HBM byte counters; "
                         "dense: only the dense path (interface solves at --n, --steps calls); "
                         "3d: only the ellipsoid section; neumann: only the Neumann section; "
                         "gray_scott: only the Gray-Scott section; iterations: only Table 2's comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the KFBI path here has no multi-GPU mode "
              "(no sharding, no collectives); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2404_15249_amd import kfbi

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.mode == "copy":
        print(json.dumps(copy_calibration()), flush=True)
        return
    # one stream, current for torch and the library's: nothing to order between two
    stream = torch.cuda.Stream(device=0)
    torch.cuda.set_stream(stream)
    ctx = kfbi.Context(0, stream=stream)
    if args.mode == "dense":
        print(json.dumps(dense_solves(ctx, args.n, calls=min(args.steps, 50))), flush=True)
        return
    if args.mode == "3d":
        print(json.dumps(three_d(ctx)), flush=True)
        return
    cpu = args.cpu_baseline == "on"
    if args.mode == "neumann":
        print(json.dumps(neumann(ctx, args.n, cpu=cpu)), flush=True)
        return
    if args.mode == "gray_scott":
        print(json.dumps(gray_scott(ctx, cpu=cpu)), flush=True)
        return
    if args.mode == "iterations":
        print(json.dumps(iterations(ctx, cpu=cpu)), flush=True)
        return
    if args.mode == "serving":
        print(json.dumps(serving_line(ctx, args)), flush=True)
        return
    p = synth.star_problem(n=args.n, kappa=1.0)
    prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, restart=50)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    rhs = dev(p.g)

    # warm-up (untimed): also records the step graphs.  A graph's first launch
    # uploads it, so one more untimed call of exactly the timed call's length
    # launches every graph the timed call replays (the library splits a call
    # into graphs of 32, 16, 8, 4, 2 and 1 steps).
    phi = torch.zeros(prob.M, dtype=torch.float64, device="cuda:0")
    prob.gmres(rhs, tol=0.0, max_iter=max(args.warmup, 1), out=phi)
    phi.zero_()
    prob.gmres(rhs, tol=0.0, max_iter=args.steps, out=phi)
    # timed region: graphed steps from the zero initial guess (set before the clock starts)
    phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters, applies, _, _ = prob.gmres(rhs, tol=0.0, max_iter=args.steps, out=phi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert iters == args.steps

    # the fixed cost of one kfbi_gmres call (start launch, graph launches, the
    # final wait, the Python call), outside the timed region: medians of calls
    # of 10 and 20 steps (11 and 21 applies, no restart), per step the difference
    def call_us(k):
        ts = []
        for _ in range(7):
            phi.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            prob.gmres(rhs, tol=0.0, max_iter=k, out=phi)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return 1e6 * sorted(ts)[3]
    t10, t20 = call_us(10), call_us(20)
    marginal = (t20 - t10) / 10.0
    per_call = {"overhead_us": t10 - 11.0 * marginal, "us_per_apply_marginal": marginal,
                "call_10_steps_us": t10, "call_20_steps_us": t20,
                "basis": "t(10 steps) - 11 x (t(20) - t(10))/10; a call of K steps makes K + 1 applies "
                         "(the last one the true residual) below the restart length"}

    # instrumented region: the same steps launched one by one with HIP events per stage
    prob.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.gmres(rhs, tol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    dt_ev = time.perf_counter() - t1
    tim = prob.apply_timing()
    prob.set_timing(False)

    unknowns = (p.n - 1) ** 2
    value = unknowns * args.steps / dt
    fl = modes_flops(p.n, prob.I, prob.M)
    achieved = fl / (tim["modes_us"] * 1e-6) / 1e12

    # full Dirichlet solves of the same problem (volume potential, GMRES to 1e-10,
    # final solve), the data already on the device: the median of five after two
    prob_s = kfbi.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-10)
    fs, fgs, gs = dev(p.f_grid), dev(p.f_gamma), dev(p.g)
    for _ in range(2):
        prob_s.solve(fs, fgs, gs)
    solve_ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        u, ug, phi, it, rel, conv = prob_s.solve(fs, fgs, gs)
        torch.cuda.synchronize()
        solve_ts.append(1e3 * (time.perf_counter() - ts))
    solve_ms = sorted(solve_ts)[2]
    c = p.lo + np.arange(p.n + 1) * p.h
    X, Y = np.meshgrid(c, c, indexing="xy")
    mask = prob_s.mask()
    err = np.max(np.abs(u.cpu().numpy() - p.exact.u(X, Y))[mask])
    prob_s.close()

    out = {
        "metric": "grid unknowns/s per KFBI apply",
        "value": value,
        "unit": "grid unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D modified Helmholtz (kappa=1) on the star r=0.6+0.15 sin 5t, {p.n}x{p.n} grid "
                        f"({unknowns} unknowns), {prob.M} boundary samples; step = one GMRES iteration "
                        f"(K_D apply + Gram-Schmidt + Givens)",
            "grid": p.n, "unknowns": unknowns, "samples": prob.M, "irregular_nodes": prob.I,
            "crossings": prob.Q, "kappa": p.kappa, "restart": 50,
        },
        "roofline": {
            "kernel": "k_modes (sparse fast solve)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": counter_traffic(p.n, prob.tiles()["modes_per_group"]),
            "flops_per_launch": fl,
            "avg_us": tim["modes_us"],
        },
        # the method's own floor: one write and one read of a half-transformed
        # FP64 grid per apply (16 bytes per unknown) at the 8 TB/s HBM peak
        "method_ceiling": {"value": HBM_PEAK_BYTES / 16.0, "unit": "grid unknowns/s",
                           "frac": value / (HBM_PEAK_BYTES / 16.0),
                           "basis": "16 B per unknown (one FP64 write + read of the half-transformed grid) at 8 TB/s"},
        "stages_us": {"correct": tim["correct_us"], "modes": tim["modes_us"], "interp": tim["interp_us"],
                      "gmres_step_and_gaps": 1e6 * dt_ev / args.steps - tim["correct_us"] - tim["modes_us"]
                      - tim["interp_us"], "timed_applies": tim["count"], "all_applies": applies,
                      "us_per_step_ungraphed": 1e6 * dt_ev / args.steps},
        "solve": {"ms": solve_ms, "gmres_iters": it, "relres": rel, "converged": conv,
                  "linf_err_vs_exact": float(err)},
        "per_call": per_call,
    }
    if args.convergence == "on":
        out["convergence"] = convergence(ctx)
    if args.mixed == "on":
        out["mixed"] = mixed_precision(ctx, args.n)
    if args.three_d == "on":
        out["three_d"] = three_d(ctx)
    cpu = args.cpu_baseline == "on"
    if args.neumann == "on":
        out["neumann"] = neumann(ctx, args.n, cpu=cpu)
    if args.gray_scott == "on":
        out["gray_scott"] = gray_scott(ctx, cpu=cpu)
    if args.iterations == "on":
        out["iterations"] = iterations(ctx, cpu=cpu)
    if args.serving_requests > 0:
        out["serving"] = serving(ctx, args.serving_requests, args.serving_seed)
    if args.cpu_baseline == "on":
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
