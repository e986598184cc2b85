"""Writes full-size reference values for the GPU parity tests, from the oracle only.

For a workload (default: the 3D 65^3 jittered Kuhn mesh clamped at x=0 with
f=(0,0,-1), 811,200 DOFs) this runs the oracle's FP64 V-ASMG-PCG in the
coloured Gauss-Seidel order (the GPU's order) and in FP32-V-cycle mode to
rtol 1e-6, and stores iteration counts, residuals, level sizes and the solution
at 256 seeded sample vertices plus its norms.

Run:  python tests/golden/make_oracle_golden.py [cfg2|cfg1|cfg3] > out.json
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
import workloads  # noqa: E402


def main(name: str):
    mesh = getattr(workloads, name)()
    t0 = time.perf_counter()
    o = Oracle(mesh.coords, mesh.elems, mesh.E, mesh.nu, mesh.fixed)
    t_setup = time.perf_counter() - t0
    x64, i64 = o.solve(mesh.rhs[0], 1e-6, precision="fp64")
    x32, i32 = o.solve(mesh.rhs[0], 1e-6, precision="fp32")
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(o.free, size=min(256, o.free.size), replace=False))
    out = dict(
        workload=mesh.name, n_dofs=int(o.A[0].shape[0]), rtol=1e-6,
        levels=o.level_stats(),
        fp64=dict(iterations=i64["iterations"], rel_res=i64["rel_res"],
                  rel_res_true=i64["rel_res_true"], solve_seconds=i64["solve_seconds"]),
        fp32=dict(iterations=i32["iterations"], rel_res_true=i32["rel_res_true"],
                  rel_err_vs_fp64=float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64))),
        x_norm2=float(np.linalg.norm(x64)), x_norminf=float(np.abs(x64).max()),
        sample_vertices=sample.tolist(), sample_x=x64[sample].tolist(),
        setup_seconds=t_setup,
    )
    json.dump(out, sys.stdout, indent=1)
    sys.stdout.write("\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cfg2")
