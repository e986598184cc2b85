"""Writes full-size reference values for the GPU parity tests, from the oracle only.

For a workload (default: the 3D 65^3 jittered Kuhn mesh clamped at x=0 with
f=(0,0,-1), 811,200 DOFs) this runs the oracle's FP64 V-ASMG-PCG in the
coloured Gauss-Seidel order (the GPU's order) and in FP32-V-cycle mode to
rtol 1e-6, and stores iteration counts, residuals, level sizes, the solution
at 256 seeded sample vertices, its norms, and a sketch of the whole solution
vector: its projections on 32 seeded random-sign vectors (sketch(); for an
error e, |R e| / sqrt(32) estimates |e|, so a GPU solution's sketch bounds its
whole-vector 2-norm distance from the oracle's).

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


SKETCH_ROWS = 32


def sketch(x: np.ndarray, rows: int = SKETCH_ROWS, seed: int = 7) -> np.ndarray:
    """Projections of the flattened x on `rows` seeded random-sign vectors."""
    v = np.asarray(x, dtype=np.float64).ravel()
    R = np.random.default_rng(seed).integers(0, 2, size=(rows, v.size), dtype=np.int8)
    return (R.astype(np.float64) * 2.0 - 1.0) @ v


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
        sketch_rows=SKETCH_ROWS, sketch_x=sketch(x64).tolist(),
        setup_seconds=t_setup,
    )
    json.dump(out, sys.stdout, indent=1)
    sys.stdout.write("\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cfg2")
