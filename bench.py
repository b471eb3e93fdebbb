#!/usr/bin/env python3
"""Throughput of the KFBI hot path on one MI355X: grid unknowns per second per K_D apply.

Workload: the 2D modified Helmholtz problem (kappa = 1) on the star
r(t) = 0.6 + 0.15 sin 5t in the box [-1.2, 1.2]^2, 2048 x 2048 grid
(2047^2 unknowns), 1024 equal-arc-length boundary samples, synthetic data.
One step is one GMRES iteration on the boundary density (Alg. 5): a K_D apply
(jumps + correction, sparse fast solve, interpolation: Alg. 1-4) plus the
device-side Gram-Schmidt / Givens update.  The steps run back to back on the
device with no convergence stop, so the timed work is fixed.

Prints one JSON line.  The dominant kernel's duration comes from HIP events
recorded around every launch on the library's stream inside the timed region.
The CPU baseline is the FP64 oracle timed on a bounded sample of the same
workload (rank 0, one GPU only).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X, dense FP64 vector


def modes_flops(n_grid: int, n_irr: int, m: int) -> float:
    """Algorithmic FP64 flops of one sparse fast-solve launch (k_modes).

    Per sine mode (n-1 of them): 2 flops per irregular node for the sparse sine
    sum, 14 flops per grid point for the two chunked recurrences with their
    carry fixes and the rank-one fix, 16 flops per boundary sample for the
    weighted six-point gather.
    """
    return (n_grid - 1) * (2.0 * n_irr + 14.0 * n_grid + 16.0 * m)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(p, seconds: float):
    """The oracle's K_D apply on the same workload, timed on the host cores."""
    from oracle import kfbi_oracle as O
    import synth
    plan = O.build_plan(p.xy, p.n, p.lo, p.hi)
    phi = synth.smooth_density(plan.M, 1234)
    O.apply_KD(plan, phi, p.kappa)                      # warm-up
    t0 = time.perf_counter()
    k = 0
    while True:
        O.apply_KD(plan, phi, p.kappa)
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    unknowns = (p.n - 1) ** 2
    return {"value": unknowns * k / dt, "unit": "grid unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} oracle K_D applies (scipy DST-I with workers=1, NumPy) on the same "
                      f"{p.n}^2 star problem, {dt:.1f} s on {cpu_model()}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=2048, help="grid intervals per axis")
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
    p = synth.star_problem(n=args.n, kappa=1.0)
    ctx = kfbi.Context(0)
    prob = kfbi.Problem(ctx, p.xy, p.n, p.kappa, restart=50)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    rhs = dev(p.g)

    # warm-up (untimed)
    prob.gmres(rhs, tol=0.0, max_iter=max(args.warmup, 1))
    torch.cuda.synchronize()

    prob.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters, applies, _, _ = prob.gmres(rhs, tol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = prob.apply_timing()
    prob.set_timing(False)
    assert iters == args.steps

    unknowns = (p.n - 1) ** 2
    value = unknowns * args.steps / dt
    fl = modes_flops(p.n, prob.I, prob.M)
    achieved = fl / (tim["modes_us"] * 1e-6) / 1e12

    # one full Dirichlet solve of the same problem (volume potential, GMRES to 1e-10, final solve)
    prob_s = kfbi.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-10)
    prob_s.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    u, ug, phi, it, rel, conv = prob_s.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - ts)
    c = p.lo + np.arange(p.n + 1) * p.h
    X, Y = np.meshgrid(c, c, indexing="xy")
    mask = prob_s.mask()
    err = np.max(np.abs(u.cpu().numpy() - p.exact.u(X, Y))[mask])

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
            "traffic": None,
            "flops_per_launch": fl,
            "avg_us": tim["modes_us"],
        },
        "stages_us": {"correct": tim["correct_us"], "modes": tim["modes_us"], "interp": tim["interp_us"],
                      "gmres_step_and_gaps": 1e6 * dt / args.steps - tim["correct_us"] - tim["modes_us"]
                      - tim["interp_us"], "timed_applies": tim["count"], "all_applies": applies},
        "solve": {"ms": solve_ms, "gmres_iters": it, "relres": rel, "converged": conv,
                  "linf_err_vs_exact": float(err)},
    }
    if args.cpu_baseline == "on":
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
