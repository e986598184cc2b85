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


HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak

# HBM traffic of one launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) of `bench.py --counters`, calibrated by a 256 MiB copy
# (profiles/k_gs_cell_bwd_level1_65cubed_mixed.md). Valid only for the kernel
# source it was measured on: reported as null once kernels.hpp has changed.
TRAFFIC_RECORD = {"kernels_sha256": "79cbcb57094d2792d54c70b9af206c644b2b447c0c898e276d1a2df2dccb2069",
                  "bytes_per_launch": 49692850}


def traffic_per_launch():
    import hashlib
    path = os.path.join(ROOT, "paper_2505_09064_amd", "csrc", "kernels.hpp")
    sha = hashlib.sha256(open(path, "rb").read()).hexdigest()
    if TRAFFIC_RECORD["kernels_sha256"] == sha:
        return TRAFFIC_RECORD["bytes_per_launch"]
    return None


def device_info(torch):
    """The GPU the benchmark ran on, as the runtime reports it (the roofline's
    peak assumes an MI355X: 256 compute units, 8 TB/s HBM3E)."""
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count, "memory_gib": round(p.total_memory / 2**30, 1)}


def host_cpu():
    """Core count and CPU model of the machine the benchmark runs on."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.strip().startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(mesh, its_gpu: int, max_reps: int = 3, budget_s: float = 60.0):
    """The oracle (plain NumPy/SciPy FP64 V-ASMG-PCG, coloured Gauss-Seidel in the
    GPU's order) on the benchmarked workload itself, on one core: its setup is
    timed apart, then the solve phase to rtol 1e-6 is timed up to max_reps times
    (fewer once budget_s of solves have run); the median is reported."""
    from threadpoolctl import threadpool_limits

    from oracle import Oracle
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = Oracle(mesh.coords, mesh.elems, mesh.E, mesh.nu, mesh.fixed)
        t_setup = time.perf_counter() - t0
        log(f"cpu baseline: oracle setup {t_setup:.1f}s")
        ts, its = [], 0
        for r in range(max_reps):
            _, info = o.solve(mesh.rhs[0], 1e-6)
            ts.append(info["solve_seconds"])
            its = info["iterations"]
            log(f"cpu baseline: oracle solve {r}: {ts[-1]:.2f}s, {its} its")
            if sum(ts) > budget_s:
                break
    return dict(n_dofs=int(o.A[0].shape[0]), iterations=its, solve_s=float(np.median(ts)),
                reps=len(ts), setup_s=t_setup)


def cpu_baseline_cfg1(reps: int = 10):
    """The 33^2 manufactured-solution workload (1,922 DOFs): the plain method's
    CPU seconds to rtol 1e-6 (oracle, FP64, one core), median of reps solves."""
    from threadpoolctl import threadpool_limits

    from oracle import Oracle
    from workloads import cfg1
    m = cfg1()
    with threadpool_limits(limits=1):
        o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
        out = {}
        for smoother in ("colored", "lex"):
            ts, its = [], 0
            for _ in range(reps):
                _, info = o.solve(m.rhs[0], 1e-6, smoother=smoother)
                ts.append(info["solve_seconds"])
                its = info["iterations"]
            out[smoother] = {"solve_s_median": float(np.median(ts)), "iterations": its,
                             "reps": reps}
    return out


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


def bench_block16(args, V, torch):
    """The 65^3 workload with 16 Fourier load cases: block solves only (K = 16,
    FP32 V-cycle), for profiling the block kernels."""
    from workloads import cfg2, load_fourier_tet
    mesh = cfg2()
    d_F = torch.from_numpy(np.stack(load_fourier_tet(mesh.coords, mesh.elems, 16))).to("cuda")
    d_X = torch.zeros_like(d_F)
    blk = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, block_rhs=16,
                             autotune=0 if args.no_autotune else 1)
    time_solves(blk, d_F, d_X, max(1, args.warmup))
    rb = time_solves(blk, d_F, d_X, max(1, min(args.steps, 5)))
    ms = float(np.mean([r[0] for r in rb]))
    ib = rb[-1][1]
    blk.free()
    print(json.dumps({
        "metric": "V-ASMG-PCG time-to-rtol 1e-6, 16 load cases", "value": 16.0 / (ms * 1e-3),
        "unit": "load cases/s", "n_gpus": 1, "steps": len(rb), "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (V-cycle) + f64 (PCG)", "data": "synthetic",
        "config": {"workload": "3D P1 elasticity, 65^3 jittered Kuhn mesh (seed 1), clamped x=0, "
                               "16 Fourier body-force load cases, 811,200 DOFs each, block solve K=16",
                   "n_dofs": mesh.n_dofs},
        "iterations": [int(i["iterations"]) for i in ib],
        "max_rel_res_true": float(max(i["rel_res_true"] for i in ib))}), flush=True)


def bench_setup(args, V, torch):
    """Device setup of the 65^3 workload (setup_device = 1, FP32 V-cycle, autotune
    off), three times in one process: the first loads the kernels, the later
    ones are what a serving process pays per request of this size."""
    from workloads import cfg2
    mesh = cfg2()
    times, phases = [], []
    for rep in range(3):
        t0 = time.perf_counter()
        s = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, setup_device=1, autotune=0)
        times.append(time.perf_counter() - t0)
        phases.append({n: round(ms, 2) for n, ms in s.setup_phases()})
        s.free()
        log(f"setup {rep}: {1e3 * times[-1]:.1f} ms {phases[-1]}")
    warm = float(np.median(times[1:]))
    print(json.dumps({
        "metric": "V-ASMG device setup time (fine assembly, tree, prolongations, Galerkin "
                  "products, colouring, layouts)", "value": warm, "unit": "s",
        "n_gpus": 1, "steps": 2, "warmup": 1, "ms_per_step": 1e3 * warm, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (setup)", "data": "synthetic",
        "config": {"workload": "3D P1 elasticity, 65^3 jittered Kuhn mesh (seed 1), clamped x=0, "
                               "811,200 DOFs, setup_device=1, autotune off",
                   "n_dofs": mesh.n_dofs},
        "first_setup_s": times[0], "setup_s": times, "phases_ms": phases}), flush=True)


def bench_cfg3(args, V, torch):
    """The 2D nearly incompressible graded workload: 1025^2 vertices with the map
    x -> x^2, y -> y^2, nu = 0.49, E in {1, 100} on a random 8x8 checkerboard
    (seed 2), 2,093,058 DOFs. FP32 V-cycle in FP64 PCG against all-FP64, both to
    rtol 1e-6; the error of each against the FP64 oracle's solution (sampled
    values stored by the oracle) is reported."""
    from workloads import cfg3
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "cfg3_oracle.json")))
    idx = np.array(gold["sample_vertices"])
    ref = np.array(gold["sample_x"])
    mesh = cfg3()
    d_rhs = torch.from_numpy(mesh.rhs[0]).to("cuda")
    d_x = torch.zeros_like(d_rhs)
    res = {}
    for name, prec in (("mixed", V.FP32_PRECOND), ("fp64", V.FP64)):
        t0 = time.perf_counter()
        s = V.Solver.from_mesh(mesh, precision=prec, setup_device=1, verbose=1,
                               autotune=0 if args.no_autotune else 1)
        t_setup = time.perf_counter() - t0
        time_solves(s, d_rhs, d_x, max(1, args.warmup))
        runs = time_solves(s, d_rhs, d_x, max(1, min(args.steps, 5)))
        x = d_x.cpu().numpy()
        info = runs[-1][1]
        res[name] = {"ms": float(np.mean([r[0] for r in runs])), "iterations": info["iterations"],
                     "rel_res_true": info["rel_res_true"], "setup_s": t_setup,
                     "error_vs_fp64_oracle": float(np.abs(x[idx] - ref).max() / gold["x_norminf"])}
        log(f"{name}: {res[name]}")
        s.free()
    ms = res["mixed"]["ms"]
    print(json.dumps({
        "metric": "V-ASMG-PCG time-to-rtol 1e-6, FP32-precond vs FP64", "value": 1e3 / ms,
        "unit": "solves/s", "n_gpus": 1, "steps": max(1, min(args.steps, 5)), "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (V-cycle) + f64 (PCG)", "data": "synthetic",
        "config": {"workload": "2D plane strain, 1025^2 graded mesh (x^2, y^2), nu=0.49, E in {1,100} "
                               "on a random 8x8 checkerboard (seed 2), V(1,1) V-ASMG-PCG rtol 1e-6",
                   "n_dofs": mesh.n_dofs},
        "iterations": res["mixed"]["iterations"], "rel_res_true": res["mixed"]["rel_res_true"],
        "error_vs_fp64_oracle": res["mixed"]["error_vs_fp64_oracle"],
        "oracle_iterations": {"fp64": gold["fp64"]["iterations"], "fp32_mode": gold["fp32"]["iterations"]},
        "fp64": res["fp64"]}), flush=True)


def bench_cfg4(args, V, torch):
    """129^3 jittered Kuhn mesh (seed 3), clamped at x=0, 16 Fourier load cases,
    6,390,144 DOFs per case: one block solve (K = 16, FP32 V-cycle) against the
    same 16 columns solved one after another by a single-column handle."""
    from workloads import load_fourier_tet, small3d
    t0 = time.perf_counter()
    mesh = small3d(129, seed=3, fix="x0")
    log(f"mesh 129^3: {mesh.n_dofs} DOFs ({time.perf_counter() - t0:.1f}s)")
    mesh.rhs = load_fourier_tet(mesh.coords, mesh.elems, 16)
    log(f"16 load cases ({time.perf_counter() - t0:.1f}s)")
    d_F = torch.from_numpy(np.stack(mesh.rhs)).to("cuda")
    d_X = torch.zeros_like(d_F)
    t0 = time.perf_counter()
    blk = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, block_rhs=16, verbose=1,
                             autotune=0 if args.no_autotune else 1)
    t_setup = time.perf_counter() - t0
    log(f"setup (block) {t_setup:.1f}s")
    time_solves(blk, d_F, d_X, args.warmup if args.warmup > 0 else 1)
    rb = time_solves(blk, d_F, d_X, max(1, min(args.steps, 3)))
    ms_blk = float(np.mean([r[0] for r in rb]))
    ib = rb[-1][1]
    log(f"block: {ms_blk:.1f} ms for 16 cases, its {[i['iterations'] for i in ib]}")
    blk.free()
    # the column-by-column handle is built with the device setup (Galerkin
    # products and level layouts on the device): same structure, values to rounding
    t0 = time.perf_counter()
    one = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, autotune=1, setup_device=1,
                             verbose=1)
    t_setup_dev = time.perf_counter() - t0
    log(f"setup (single column, device) {t_setup_dev:.1f}s")
    time_solves(one, d_F[:1], d_X[:1], 1)
    rs = time_solves(one, d_F, d_X, 1)
    ms_seq = rs[-1][0]
    iseq = rs[-1][1]
    log(f"column by column: {ms_seq:.1f} ms for 16 cases, its {[i['iterations'] for i in iseq]}")
    one.free()
    line = {
        "metric": "V-ASMG-PCG time-to-rtol 1e-6, 16 load cases",
        "value": 16.0 / (ms_blk * 1e-3), "unit": "load cases/s", "n_gpus": 1,
        "steps": len(rb), "warmup": args.warmup, "ms_per_step": ms_blk, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (V-cycle) + f64 (PCG)",
        "data": "synthetic",
        "config": {"workload": "3D P1 elasticity, 129^3 jittered Kuhn mesh (seed 3), clamped x=0, "
                               "16 Fourier body-force load cases, 6,390,144 DOFs each, V(1,1) "
                               "V-ASMG-PCG rtol 1e-6, block solve K=16", "n_dofs": mesh.n_dofs},
        "iterations": [int(i["iterations"]) for i in ib],
        "max_rel_res_true": float(max(i["rel_res_true"] for i in ib)),
        "setup_s": t_setup,
        "setup_device_s": t_setup_dev,
        "column_by_column_ms": ms_seq,
        "column_by_column_iterations": [int(i["iterations"]) for i in iseq],
        "speedup_vs_column_by_column": ms_seq / ms_blk,
    }
    print(json.dumps(line), flush=True)


PACK_MAX_DOFS = 20000      # serving: requests this small are packed in the packed phase


def pack_leg(V, meshes, reps: int = 3):
    """Small requests (at most PACK_MAX_DOFS DOFs) of the serving stream solved
    one after another on one stream, each alone, against the same requests
    packed (vasmg_pack: up to 16 per pack, same dimension, coarsest levels
    within 256 DOFs together), FP32 V-cycle, rtol 1e-6. Setups, uploads and
    packing happen before the timed region; the solves run with their inputs
    resident in HBM. Median of `reps` passes over all of them."""
    import torch
    small = [m for m in meshes if m.n_dofs <= PACK_MAX_DOFS]
    if len(small) < 2:
        return None
    alone, rhs = [], []
    for m in small:
        alone.append(V.Solver.from_mesh(m, precision=V.FP32_PRECOND, autotune=0))
        rhs.append(torch.from_numpy(np.ascontiguousarray(m.rhs[0])).to("cuda"))
    xs = [torch.zeros_like(r) for r in rhs]
    # packs: by dimension, in order, closed at 16 parts or 256 coarsest DOFs
    packs, cur, coarse = [], [], 0
    hosts = [V.Solver.from_mesh(m, precision=V.FP32_PRECOND, host_only=1) for m in small]
    order = sorted(range(len(small)), key=lambda i: small[i].dim)
    for i in order:
        h = hosts[i]
        nl = h.hierarchy_info()[0]
        c = h.level_info(nl - 1)["n_vertices"] * small[i].dim
        if cur and (small[cur[0]].dim != small[i].dim or len(cur) == 16 or coarse + c > 256):
            packs.append(cur)
            cur, coarse = [], 0
        cur.append(i)
        coarse += c
    packs.append(cur)
    pks = [V.PackedSolver([hosts[i] for i in p]) for p in packs]
    prhs = [torch.cat([rhs[i] for i in p]) for p in packs]
    px = [torch.zeros_like(r) for r in prhs]
    t_alone, t_packed, it_alone, it_packed = [], [], None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it_alone = [s.solve_device(r, x, 1e-6)["iterations"] for s, r, x in zip(alone, rhs, xs)]
        torch.cuda.synchronize()
        t_alone.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        infos = [pk.solve_packed_device(r, x, 1e-6) for pk, r, x in zip(pks, prhs, px)]
        torch.cuda.synchronize()
        t_packed.append(time.perf_counter() - t0)
        it_packed = {i: inf["iterations"] for p, inf_p in zip(packs, infos) for i, inf in zip(p, inf_p)}
    diff, dit = 0.0, 0
    for p, x in zip(packs, px):
        parts = torch.split(x, [small[i].n_vertices for i in p])
        for i, xp in zip(p, parts):
            a = xs[i].cpu().numpy()
            diff = max(diff, float(np.linalg.norm(xp.cpu().numpy() - a) / max(np.linalg.norm(a), 1e-300)))
            dit = max(dit, abs(it_packed[i] - it_alone[i]))
    for o in alone + pks + hosts:
        o.free()
    ta, tp = float(np.median(t_alone)), float(np.median(t_packed))
    n = len(small)
    return {
        "small_requests": n, "max_dofs": PACK_MAX_DOFS,
        "dofs_mean": float(np.mean([m.n_dofs for m in small])), "packs": len(packs),
        "mean_parts_per_pack": n / len(packs),
        "ms_per_request_alone": 1e3 * ta / n, "ms_per_request_packed": 1e3 * tp / n,
        "speedup": ta / tp, "mean_iterations_alone": float(np.mean(it_alone)),
        "max_iteration_difference": dit, "max_rel_diff_packed_vs_alone": diff,
    }


def serve_leg(V, N: int, host_setup: bool = False, saturated: bool = True):
    """The serving stream: requests i = 0..N-1 (2D or 3D jittered meshes, DOFs
    log-uniform in [1e3, 1e6], 1:100 materials), each a new mesh, so latency
    includes its setup (the device setup above the server's default size limits,
    the host setup below them and everywhere with host_setup). The
    single-stream rate is measured first by serving the first 8 requests one at a
    time (one slot, one setup worker); then all N arrive as a Poisson stream at
    0.7x that rate into a server with 4 slots and 4 setup workers. Latency =
    done - arrival. The first 8 results must be bitwise identical alone and in
    the mix. With saturated: all N submitted at once, first unpacked, then with
    requests of at most PACK_MAX_DOFS packed (vasmg_pack: one solve per pack);
    the packed results are compared with the unpacked ones. Returns a dict of
    the figures."""
    from workloads import request_mesh
    N = max(8, N)
    t0 = time.perf_counter()
    meshes = []
    for i in range(N):
        meshes.append(request_mesh(i))
        if i % 8 == 7:
            log(f"generated {i + 1}/{N} requests ({time.perf_counter() - t0:.1f}s)")
    dofs = np.array([m.n_dofs for m in meshes])
    opts = dict(precision=V.FP32_PRECOND, setup_device=0 if host_setup else 1)

    # single stream: one request at a time end to end
    srv = V.Server(slots=1, setup_workers=1, **opts)
    alone = []
    t0 = time.perf_counter()
    for i in range(8):
        rid = srv.submit(meshes[i], meshes[i].rhs[0], 1e-6)
        alone.append(srv.wait(rid))
    t_single = time.perf_counter() - t0
    srv.close()
    rate1 = 8.0 / t_single
    lam = 0.7 * rate1
    log(f"single stream: {rate1:.2f} requests/s (8 requests, {t_single:.1f}s); arrivals at {lam:.2f}/s")

    rng = np.random.default_rng(7)
    gaps = rng.exponential(1.0 / lam, size=N)
    srv = V.Server(slots=4, setup_workers=4, **opts)
    ids = []
    t0 = time.perf_counter()
    t_next = 0.0
    for i in range(N):
        t_next += gaps[i]
        dt = t_next - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(srv.submit(meshes[i], meshes[i].rhs[0], 1e-6))
        if i % 8 == 7:
            log(f"submitted {i + 1}/{N}, {srv.stats()}")
    got = [srv.wait(r) for r in ids]
    t_all = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    got2, t_sat, lat2 = None, None, None
    if saturated:
        # saturation: every request submitted at once (capacity of the batching)
        srv2 = V.Server(slots=4, setup_workers=4, **opts)
        t1 = time.perf_counter()
        ids2 = [srv2.submit(m, m.rhs[0], 1e-6) for m in meshes]
        got2 = [srv2.wait(r) for r in ids2]
        t_sat = time.perf_counter() - t1
        srv2.close()
        lat2 = np.array([g[1]["t_done_ms"] - g[1]["t_submit_ms"] for g in got2])
        log(f"saturated: {N / t_sat:.2f} requests/s")
        # the same, small requests packed (one upload and one solve per pack)
        srv3 = V.Server(slots=4, setup_workers=4, pack_max_dofs=PACK_MAX_DOFS, pack_max_parts=16,
                        **opts)
        t1 = time.perf_counter()
        ids3 = [srv3.submit(m, m.rhs[0], 1e-6) for m in meshes]
        got3 = [srv3.wait(r) for r in ids3]
        t_pack = time.perf_counter() - t1
        srv3.close()
        lat3 = np.array([g[1]["t_done_ms"] - g[1]["t_submit_ms"] for g in got3])
        small = [i for i in range(N) if dofs[i] <= PACK_MAX_DOFS]
        packed = [i for i in small if got3[i][1]["pack_size"] > 1]
        # device time of a small request's solve: alone, and its share of its pack
        solo_ms = [got2[i][1]["info"]["t_solve_ms"] for i in small]
        share_ms = [got3[i][1]["info"]["t_solve_ms"] / got3[i][1]["pack_size"] for i in small]
        diff = max((np.linalg.norm(got3[i][0] - got2[i][0]) / max(np.linalg.norm(got2[i][0]), 1e-300)
                    for i in range(N) if got3[i][0] is not None and got2[i][0] is not None),
                   default=0.0)
        pack_stats = {
            "packed_saturated_requests_per_s": N / t_pack,
            "packed_saturated_p50_ms": float(np.percentile(lat3, 50)),
            "packed_saturated_p99_ms": float(np.percentile(lat3, 99)),
            "pack_max_dofs": PACK_MAX_DOFS, "small_requests": len(small),
            "small_requests_packed": len(packed),
            "mean_pack_size": float(np.mean([got3[i][1]["pack_size"] for i in packed])) if packed else 1.0,
            "small_request_solve_ms_alone": float(np.mean(solo_ms)) if small else None,
            "small_request_solve_ms_packed_share": float(np.mean(share_ms)) if small else None,
            "packed_all_ok": all(g[1]["status"] == V.OK for g in got3),
            "packed_vs_unpacked_max_rel_diff": float(diff),
        }
        log(f"packed saturated: {N / t_pack:.2f} requests/s, {len(packed)}/{len(small)} small "
            f"requests packed, solve {pack_stats['small_request_solve_ms_alone']:.2f} ms alone -> "
            f"{pack_stats['small_request_solve_ms_packed_share']:.2f} ms share")
    res = [g[1] for g in got]
    ok = [r["status"] == V.OK for r in res] + [g[1]["status"] == V.OK for g in (got2 or [])]
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in res])
    setup = np.array([r["t_setup_end_ms"] - r["t_setup_start_ms"] for r in res])
    solve = np.array([r["info"]["t_solve_ms"] for r in res])
    queue = np.array([r["t_admit_ms"] - r["t_setup_end_ms"] for r in res])
    same = all(np.array_equal(got[i][0], alone[i][0]) and
               (got2 is None or np.array_equal(got2[i][0], alone[i][0])) for i in range(8))
    overlap = 0
    iv = sorted((r["t_admit_ms"], r["t_done_ms"]) for r in res)
    for a in range(len(iv)):
        for b in range(a + 1, len(iv)):
            if iv[b][0] < iv[a][1]:
                overlap += 1
    out = {
        "requests": N, "requests_per_s": N / t_all, "ms_per_request": 1e3 * t_all / N,
        "dofs_min": int(dofs.min()), "dofs_max": int(dofs.max()), "dofs_mean": float(dofs.mean()),
        "setup": ("host" if host_setup else
                  "device (fine assembly, tree, P, Galerkin products) above 131,072 DOFs in 2D "
                  "and 16,384 in 3D, host below"),
        "requests_set_up_on_device": int(sum(r["setup_device"] for r in res)),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "single_stream_requests_per_s": rate1, "arrival_rate": lam,
        "mean_setup_ms": float(setup.mean()), "mean_solve_ms": float(solve.mean()),
        "mean_admission_wait_ms": float(queue.mean()),
        "all_ok": bool(all(ok)), "same_alone_and_in_mix": bool(same),
        "overlapping_request_pairs_on_device": overlap,
        "peak_device_bytes": int(st["peak_bytes"]), "budget_bytes": int(st["budget_bytes"]),
    }
    if saturated:
        out.update({"saturated_requests_per_s": N / t_sat,
                    "saturated_p50_ms": float(np.percentile(lat2, 50)),
                    "saturated_p99_ms": float(np.percentile(lat2, 99))})
        out.update(pack_stats)
    pk = pack_leg(V, meshes)
    if pk is not None:
        out["packed_small_solves"] = pk
        log(f"packed small solves: {pk['small_requests']} requests in {pk['packs']} packs, "
            f"{pk['ms_per_request_alone']:.2f} ms alone -> {pk['ms_per_request_packed']:.2f} ms "
            f"per request ({pk['speedup']:.1f}x), max rel diff {pk['max_rel_diff_packed_vs_alone']:.1e}")
    return out


def bench_serve(args, V):
    """The serving stream as its own benchmark line (serve_leg)."""
    r = serve_leg(V, args.requests, args.host_setup)
    N = r["requests"]
    line = {
        "metric": "serving: requests/s and p50/p99 latency (setup + solve), rtol 1e-6",
        "value": r["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": N, "warmup": 0,
        "ms_per_step": r["ms_per_request"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (V-cycle) + f64 (PCG)", "data": "synthetic",
        "config": {"workload": f"{N} requests, 2D/3D jittered P1 elasticity meshes, DOFs "
                               "log-uniform in [1e3, 1e6] (seeded per request), Poisson arrivals "
                               "at 0.7x the single-stream rate, 4 slots, 4 setup workers",
                   "dofs_min": r["dofs_min"], "dofs_max": r["dofs_max"],
                   "dofs_mean": r["dofs_mean"], "setup": r["setup"]},
        **{k: v for k, v in r.items() if k not in ("requests", "requests_per_s", "ms_per_request",
                                                   "dofs_min", "dofs_max", "dofs_mean", "setup")},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--workload", choices=["cfg2", "cfg3", "block16", "cfg4", "serve", "setup"],
                    default="cfg2",
                    help="cfg2: the headline 65^3 workload (default); cfg3: the graded 2D "
                         "nu=0.49 workload, mixed vs FP64; cfg4: 129^3 with 16 load "
                         "cases, block solve against column-by-column solves; block16: the 65^3 mesh with "
                         "16 load cases, block solve only; serve: the request stream through the "
                         "continuous-batching server; setup: three device setups of the 65^3 workload")
    ap.add_argument("--requests", type=int, default=48, help="serve: number of requests")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving leg reported among the headline's variants")
    ap.add_argument("--no-serve", action="store_true",
                    help="leave the serving leg out of the headline's variants")
    ap.add_argument("--host-setup", action="store_true",
                    help="serve: setup workers build the whole hierarchy on the host (default: "
                         "their Galerkin products on the device)")
    ap.add_argument("--counters", action="store_true",
                    help="driver for rocprofv3 --pmc runs: a 256 MiB device copy (counter "
                         "calibration) followed by one replayed PCG iteration of the workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "the solver has no multi-GPU path"}))
        sys.exit(2)

    import torch
    from paper_2505_09064_amd import vasmg as V
    from workloads import cfg2

    torch.cuda.set_device(0)
    if args.workload == "cfg4":
        bench_cfg4(args, V, torch)
        return
    if args.workload == "block16":
        bench_block16(args, V, torch)
        return
    if args.workload == "cfg3":
        bench_cfg3(args, V, torch)
        return
    if args.workload == "setup":
        bench_setup(args, V, torch)
        return
    if args.workload == "serve":
        bench_serve(args, V)
        return
    if args.counters:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)                       # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        mesh = cfg2()
        s = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND,
                               autotune=0 if args.no_autotune else 1)
        for p in s.profile_iteration(1):
            log(f"{p['name']:13s} L{p['level']:2d} launches {p['launches']:3d} "
                f"bytes {p['bytes']:.0f} ms {p['ms']:.4f}")
        s.free()
        return
    t0 = time.perf_counter()
    mesh = cfg2()
    log(f"mesh {mesh.name}: {mesh.n_vertices} vertices, {mesh.elems.shape[0]} tets, "
        f"{mesh.n_dofs} DOFs ({time.perf_counter() - t0:.1f}s)")
    d_rhs = torch.from_numpy(mesh.rhs[0]).to("cuda")
    d_x = torch.zeros_like(d_rhs)

    t0 = time.perf_counter()
    mixed = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, verbose=1,
                               autotune=0 if args.no_autotune else 1)
    t_setup = time.perf_counter() - t0
    log(f"setup (mixed) {t_setup:.1f}s")
    # the same hierarchy with the Galerkin products and level layouts on the device
    t0 = time.perf_counter()
    dev_setup = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, setup_device=1,
                                   autotune=0 if args.no_autotune else 1)
    t_setup_dev = time.perf_counter() - t0
    dev_info = dev_setup.solve_device(d_rhs, d_x, 1e-6)
    dev_setup.free()
    # a second device setup (the kernels loaded by now, autotune off): the cost a
    # serving process pays per request of this size
    t0 = time.perf_counter()
    dev2 = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, setup_device=1, autotune=0)
    t_setup_dev2 = time.perf_counter() - t0
    dev_phases = {n: round(ms, 2) for n, ms in dev2.setup_phases()}
    dev2.free()
    log(f"setup (mixed, device, second, autotune off) {t_setup_dev2:.3f}s: {dev_phases}")
    log(f"setup (mixed, device Galerkin + layout) {t_setup_dev:.2f}s, "
        f"{dev_info['iterations']} its")
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
        fp64 = V.Solver.from_mesh(mesh, precision=V.FP64, autotune=0 if args.no_autotune else 1)
        time_solves(fp64, d_rhs, d_x, 1)
        r64 = time_solves(fp64, d_rhs, d_x, max(3, args.steps // 4))
        ms64 = float(np.mean([r[0] for r in r64]))
        ph64 = fp64.profile_iteration(3)
        b64 = sum(p["bytes"] for p in ph64) / 3          # byte model, one FP64 iteration
        spmv_b = sum(p["bytes"] for p in ph64 if p["name"] == "spmv_f64") / 3
        vec_b = sum(p["bytes"] for p in ph64 if p["name"] == "pcg_vectors") / 3
        variants["fp64_vasmg"] = dict(ms_per_solve=ms64, iterations=r64[-1][1]["iterations"],
                                      iteration_bytes=b64,
                                      solve_GBps=b64 * r64[-1][1]["iterations"] / (ms64 * 1e-3) / 1e9)
        fp64.free()
        # leaf capacity 27: the 3D analogue of the capacity under which the method
        # reduces to geometric multigrid on uniform grids (the paper's Theorem 2)
        c27 = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, leaf_capacity=27,
                                 autotune=0 if args.no_autotune else 1)
        time_solves(c27, d_rhs, d_x, 1)
        rc = time_solves(c27, d_rhs, d_x, max(3, args.steps // 4))
        variants["mixed_capacity27"] = dict(ms_per_solve=float(np.mean([r[0] for r in rc])),
                                            iterations=rc[-1][1]["iterations"],
                                            rel_res_true=rc[-1][1]["rel_res_true"])
        c27.free()
        # Gauss-Seidel by colour blocks on level 1 (8 colours of up to 8 cells
        # swept in sequence inside a block, instead of 27 colours of cells)
        cbk = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, color_blocks=1,
                                 autotune=0 if args.no_autotune else 1)
        time_solves(cbk, d_rhs, d_x, 1)
        rk = time_solves(cbk, d_rhs, d_x, max(3, args.steps // 4))
        variants["mixed_color_blocks"] = dict(ms_per_solve=float(np.mean([r[0] for r in rk])),
                                              iterations=rk[-1][1]["iterations"],
                                              rel_res_true=rk[-1][1]["rel_res_true"])
        cbk.free()
        # block right-hand sides: 16 smooth random load cases solved as 16 PCG
        # recurrences that share every matrix read
        from workloads import load_fourier_tet
        t0 = time.perf_counter()
        F16 = np.stack(load_fourier_tet(mesh.coords, mesh.elems, 16))
        log(f"16 load cases: {time.perf_counter() - t0:.1f}s")
        d_F16 = torch.from_numpy(F16).to("cuda")
        d_X16 = torch.zeros_like(d_F16)
        blk = V.Solver.from_mesh(mesh, precision=V.FP32_PRECOND, block_rhs=16,
                                 autotune=0 if args.no_autotune else 1)
        time_solves(blk, d_F16, d_X16, 1)
        rb = time_solves(blk, d_F16, d_X16, max(3, args.steps // 4))
        ib = rb[-1][1]
        variants["mixed_block16"] = dict(
            ms_per_block_solve=float(np.mean([r[0] for r in rb])),
            ms_per_rhs=float(np.mean([r[0] for r in rb])) / 16,
            iterations=[int(i["iterations"]) for i in ib],
            max_rel_res_true=float(max(i["rel_res_true"] for i in ib)),
            loads="16 Fourier body forces (8 modes per component, seed 3) on the same mesh")
        blk.free()
        jac = V.Solver.from_mesh(mesh, precision=V.FP64, preconditioner=V.PRECOND_JACOBI)
        rj = time_solves(jac, d_rhs, d_x, 2)
        msj = float(np.mean([r[0] for r in rj]))
        # byte model of one Jacobi-PCG iteration: the FP64 SpMV and PCG vector
        # phases (same fine matrix as above) plus z = D^-1 r (inverse diagonal
        # blocks once, r in, z out; padded vectors)
        n0 = mesh.n_dofs // 3
        bj = spmv_b + vec_b + n0 * 9 * 8 + 2 * n0 * 4 * 8
        variants["fp64_jacobi_pcg"] = dict(ms_per_solve=msj, iterations=rj[-1][1]["iterations"],
                                           iteration_bytes=bj,
                                           solve_GBps=bj * rj[-1][1]["iterations"] / (msj * 1e-3) / 1e9)
        jac.free()
        # the small 2D manufactured-solution workload on the GPU (latency-bound)
        from workloads import cfg1
        m1 = cfg1()
        d1 = torch.from_numpy(m1.rhs[0]).to("cuda")
        x1 = torch.zeros_like(d1)
        s1 = V.Solver.from_mesh(m1, precision=V.FP64)
        time_solves(s1, d1, x1, 3)
        r1 = time_solves(s1, d1, x1, 20)
        t1 = np.array([r[0] for r in r1])
        variants["cfg1_gpu_fp64"] = dict(
            workload="2D plane strain, 33^2 jittered (seed 0), manufactured solution, 1,922 DOFs",
            p50_ms=float(np.percentile(t1, 50)), p99_ms=float(np.percentile(t1, 99)),
            iterations=r1[-1][1]["iterations"])
        s1.free()
        # the graded nearly incompressible 2D workload (2,093,058 DOFs, 20 levels)
        from workloads import cfg3
        gold3 = json.load(open(os.path.join(ROOT, "tests", "golden", "cfg3_oracle.json")))
        m3 = cfg3()
        d3 = torch.from_numpy(m3.rhs[0]).to("cuda")
        x3 = torch.zeros_like(d3)
        t0 = time.perf_counter()
        s3 = V.Solver.from_mesh(m3, precision=V.FP32_PRECOND, setup_device=1,
                                autotune=0 if args.no_autotune else 1)
        t_setup3 = time.perf_counter() - t0
        time_solves(s3, d3, x3, 1)
        r3 = time_solves(s3, d3, x3, 5)
        t3 = np.array([r[0] for r in r3])
        i3 = np.array(gold3["sample_vertices"])
        err3 = float(np.abs(x3.cpu().numpy()[i3] - np.array(gold3["sample_x"])).max() / gold3["x_norminf"])
        variants["cfg3_mixed"] = dict(
            workload="2D plane strain, 1025^2 graded mesh (x^2, y^2), nu=0.49, E in {1,100} on a "
                     "random 8x8 checkerboard (seed 2), 2,093,058 DOFs, FP32 V-cycle in FP64 PCG",
            ms_per_solve=float(t3.mean()), p50_ms=float(np.percentile(t3, 50)),
            p99_ms=float(np.percentile(t3, 99)), iterations=r3[-1][1]["iterations"],
            oracle_fp32_mode_iterations=gold3["fp32"]["iterations"],
            rel_res_true=r3[-1][1]["rel_res_true"], error_vs_fp64_oracle=err3,
            setup_s_device_with_autotune=t_setup3)
        s3.free()
        del d3, x3
        log(f"variants: {variants}")
        if not args.no_serve:
            variants["serving"] = serve_leg(V, args.serve_requests)
            log(f"serving: {variants['serving']}")

    # per-phase device time and algorithmic bytes of one iteration (event-timed
    # launches on the solve's stream, same kernels and launch configuration)
    phases = mixed.profile_iteration(3)
    reps = 3
    it_ms = sum(p["ms"] for p in phases) / reps
    it_bytes = sum(p["bytes"] for p in phases) / reps
    dom = max(phases, key=lambda p: p["ms"])
    dom_launch_ms = dom["ms"] / dom["launches"]
    dom_launch_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_launch_bytes / dom_launch_ms / 1e6          # GB/s
    log(f"dominant phase: {dom['name']} level {dom['level']}: "
        f"{dom['launches'] / reps:.0f} launches/iteration, {dom_launch_ms * 1e3:.2f} us and "
        f"{dom_launch_bytes / 1e6:.2f} MB per launch -> {achieved:.0f} GB/s")
    log("phases of one iteration (event-timed launches):")
    for p in sorted(phases, key=lambda p: -p["ms"]):
        log(f"  {p['name']:13s} L{p['level']:2d} {p['launches'] / reps:4.0f} launches "
            f"{p['ms'] / reps:7.4f} ms/it {1e3 * p['ms'] / max(p['launches'], 1):7.2f} us/launch "
            f"{p['bytes'] / p['ms'] / 1e6:6.0f} GB/s {100 * p['ms'] / reps / it_ms:5.1f}%")
    mixed.free()

    cpu = None
    if not args.no_cpu_baseline:
        hc = host_cpu()
        cb = cpu_baseline(mesh, its[0])
        c1 = cpu_baseline_cfg1()
        cpu = {"value": 1.0 / cb["solve_s"], "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": (f"the whole benchmarked workload ({cb['n_dofs']} DOFs): oracle FP64 "
                          f"V-ASMG-PCG solve phase (coloured GS, rtol 1e-6, {cb['iterations']} its), "
                          f"median of {cb['reps']} solves of {cb['solve_s']:.2f} s on one core "
                          f"(threadpoolctl limit 1); oracle setup {cb['setup_s']:.1f} s not timed"),
               "solve_s": cb["solve_s"], "reps": cb["reps"], "iterations": cb["iterations"],
               "setup_s": cb["setup_s"],
               "host": hc,
               "cfg1_plain_method_cpu": dict(
                   workload="2D plane strain, 33^2 jittered (seed 0), manufactured solution, "
                            "1,922 DOFs, FP64 V(1,1) V-ASMG-PCG rtol 1e-6, oracle on one core",
                   **c1)}
        log(f"cpu baseline: {cpu}")

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
        "dtype": "f32 (V-cycle) + f64 (PCG)",
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
        "setup_device_s": t_setup_dev,
        "setup_device_warm_s": t_setup_dev2,
        "setup_device_warm_phases_ms": dev_phases,
        "setup_device_iterations": dev_info["iterations"],
        "timed_region_s": t_total,
        "iteration_ms_profiled": it_ms,
        "iteration_bytes": it_bytes,
        "solve_GBps": it_bytes * its[0] / (ms_per * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_per_launch(),
                     "kernel": f"{dom['name']} on level {dom['level']}",
                     "launch_us": dom_launch_ms * 1e3, "launch_bytes": dom_launch_bytes},
        "cpu_baseline": cpu,
        "device": device_info(torch),
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
