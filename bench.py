"""Throughput of the fused collide-and-stream step on one MI355X.

Workload (headline): D2Q9 modified MRT on the 4096^2 periodic cellular-flow
grid (rotated anisotropic D, 64 Gaussian hills), populations in FP32
shifted storage.  One step = one collide-and-stream pass over all nodes.
The line also carries the plain FP64 step on the same grid, the roofline of
the dominant kernel and the FP64 CPU oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_LU = {("d2q9", "fp64"): 144, ("d2q9", "fp32"): 72, ("d2q9", "fp16"): 44,
                ("d3q15", "fp64"): 240, ("d3q15", "fp32"): 120}


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    solver.step(steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def gpu_variant(wl, precision, steps, warmup):
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision)
    ev, wall = time_steps(s, steps, warmup)
    nonfinite = s.nonfinite()
    s.close()
    nodes = wl.nodes
    t_step = ev / steps
    bpl = BYTES_PER_LU[(wl.lattice, precision)]
    return {"precision": precision, "steps": steps, "ms_per_step": t_step * 1e3,
            "mlups": nodes / t_step / 1e6, "achieved_gbs": nodes * bpl / t_step / 1e9,
            "bytes_per_lu": bpl, "hbm_frac": nodes * bpl / t_step / 1e9 / HBM_PEAK_GBS,
            "wall_s": wall, "nonfinite": nonfinite}


def cpu_baseline(wl, steps=2):
    """The FP64 oracle as it stands, one BLAS thread, on the same grid."""
    import numpy as np
    from oracle import lbm as O
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:
        limiter = None
    prob = O.problem_for(wl)
    f = prob.equilibrium(wl.phi0())
    t0 = time.perf_counter()
    for _ in range(steps):
        f = prob.step(f)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {"value": wl.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps of the full {wl.shape[0]}x{wl.shape[1]} grid "
                      f"({dt:.1f} s), numpy with one BLAS thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1404_2363_amd import workloads as W
    from paper_1404_2363_amd import _lib
    _lib.load()
    torch.cuda.init()
    wl = W.cellular()
    print(f"bench: D2Q9 cellular {wl.shape} fp32, {args.steps} steps", file=sys.stderr, flush=True)
    main_v = gpu_variant(wl, "fp32", args.steps, args.warmup)
    print(f"bench: fp32 {main_v['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    fp64_v = gpu_variant(wl, "fp64", max(args.steps // 2, 1), max(args.warmup // 2, 1))
    print(f"bench: fp64 {fp64_v['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(wl)
    line = {
        "metric": "MLUPS (D2Q9 4096^2, FP32 shifted storage)",
        "value": main_v["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_v["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q9 modified MRT, 4096x4096 periodic, cellular u (U0=0.05), D eigenvalues "
                               "0.01/0.1 rotated 30 deg, 64 Gaussian hills sigma=32",
                   "storage": "fp32 shifted", "nodes": wl.nodes},
        "roofline": {"bound": "hbm", "achieved": main_v["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": main_v["hbm_frac"], "traffic": None,
                     "kernel": "k_step_d2q9<float>", "bytes_per_lu": 72},
        "variants": {"d2q9_4096_fp64": fp64_v, "d2q9_4096_fp32": main_v,
                     "speedup_fp32_over_fp64": main_v["mlups"] / fp64_v["mlups"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
