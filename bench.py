"""Benchmark: V-ASMG-PCG time-to-rtol on one MI355X.

A step is one whole solve phase (PCG to ||F - A x|| / ||F|| < 1e-6 with the
V-ASMG V-cycle preconditioner) of the 3D workload: 65^3 jittered vertex grid
(seed 1), 6 Kuhn tetrahedra per cube, E=1, nu=0.3, clamped at x=0, body force
(0,0,-1); 811,200 DOFs. The hierarchy and the right-hand side are resident in
HBM before the timed region. The headline runs the FP32 V-cycle inside FP64
PCG; the all-FP64 V-ASMG-PCG and FP64 Jacobi-PCG are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_solves(solver, d_rhs, d_x, n, rtol=1e-6):
    import torch
    out = []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = solver.solve_device(d_rhs, d_x, rtol)
        torch.cuda.synchronize()
        out.append(((time.perf_counter() - t0) * 1e3, info))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "the solver has no multi-GPU path (see DESIGN.md)"}))
        sys.exit(2)

    import torch
    from paper_2505_09064_amd import vasmg as V
    from workloads import cfg2

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    mesh = cfg2()
    log(f"mesh {mesh.name}: {mesh.n_vertices} vertices, {mesh.elems.shape[0]} tets, "
        f"{mesh.n_dofs} DOFs ({time.perf_counter() - t0:.1f}s)")
    d_rhs = torch.from_numpy(mesh.rhs[0]).to("cuda")
    d_x = torch.zeros_like(d_rhs)

    t0 = time.perf_counter()
    mixed = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, verbose=1)
    t_setup = time.perf_counter() - t0
    log(f"setup (mixed) {t_setup:.1f}s")
    for i in range(args.warmup):
        info = mixed.solve_device(d_rhs, d_x, 1e-6)
        log(f"warmup {i}: {info['iterations']} its, {info['t_solve_ms']:.2f} ms")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = time_solves(mixed, d_rhs, d_x, args.steps)
    t_total = time.perf_counter() - t_start
    ms = np.array([r[0] for r in runs])
    its = [r[1]["iterations"] for r in runs]
    dev_ms = np.array([r[1]["t_solve_ms"] for r in runs])
    info = runs[-1][1]
    log(f"mixed: {np.mean(ms):.3f} ms/solve (device {np.mean(dev_ms):.3f}), its {its[0]}, "
        f"rel_res_true {info['rel_res_true']:.2e}")

    variants = {}
    if not args.no_variants:
        fp64 = V.Solver.from_mesh(mesh, precision=V.FP64)
        time_solves(fp64, d_rhs, d_x, 1)
        r64 = time_solves(fp64, d_rhs, d_x, max(3, args.steps // 4))
        variants["fp64_vasmg"] = dict(ms_per_solve=float(np.mean([r[0] for r in r64])),
                                      iterations=r64[-1][1]["iterations"])
        fp64.free()
        jac = V.Solver.from_mesh(mesh, precision=V.FP64, preconditioner=V.PRECOND_JACOBI)
        rj = time_solves(jac, d_rhs, d_x, 2)
        variants["fp64_jacobi_pcg"] = dict(ms_per_solve=float(np.mean([r[0] for r in rj])),
                                           iterations=rj[-1][1]["iterations"])
        jac.free()
        log(f"variants: {variants}")

    ms_per = float(np.mean(ms))
    line = {
        "metric": "V-ASMG-PCG time-to-rtol 1e-6 + HBM GB/s, FP32-precond vs FP64; p50/p99 lat",
        "value": 1e3 / ms_per,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle in f64 PCG",
        "data": "synthetic",
        "config": {"workload": "3D P1 elasticity, 65^3 jittered Kuhn mesh (seed 1), clamped x=0, "
                               "f=(0,0,-1), 811,200 DOFs, V(1,1) V-ASMG-PCG rtol 1e-6",
                   "n_dofs": mesh.n_dofs, "precision": "fp32_precond"},
        "iterations": its[0],
        "p50_ms": float(np.percentile(ms, 50)),
        "p99_ms": float(np.percentile(ms, 99)),
        "device_ms_mean": float(np.mean(dev_ms)),
        "rel_res_true": info["rel_res_true"],
        "setup_s": t_setup,
        "timed_region_s": t_total,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
