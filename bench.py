#!/usr/bin/env python3
"""Benchmark of the DVM/BGK iteration on one MI355X.

Workload: 2D synthetic digital rock, 512 x 512 voxels of seeded overlapping
discs (radii U(4, 20) px, porosity 0.40, pore space percolating along x1),
Kn = 1 (L = 512 voxels), 32 x 32 half-range Gauss-Hermite velocities, specular
lateral faces, pressure jump 1. A step is one full iteration of the hot path:
the upwind sweep of every discrete velocity, the moment / source / wall-density
kernel and the FP64 residual and permeability reduction.

Prints one JSON line: cell-velocity updates per second (fluid voxels x
velocities x iterations / wall time, inputs resident in HBM), the roofline of
the dominant kernel (the sweep) from HIP-event timings, the CPU oracle timed on
a bounded sample of the same workload, and time-to-residual 1e-6 for the FP64
form and the FP32 form.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(mask, nv, kn, target_s=15.0):
    """The CPU oracle (FP64, OpenMP over velocities) on the same workload,
    timed for a bounded number of iterations."""
    from oracle.oracle import OracleSolver
    threads = len(os.sched_getaffinity(0))
    o = OracleSolver(mask, nv, kn, threads=threads)
    t0 = time.perf_counter()
    o.iterate(1)
    t1 = time.perf_counter() - t0
    more = max(1, min(50, int(target_s / max(t1, 1e-3)) - 1))
    t0 = time.perf_counter()
    o.iterate(more)
    dt = time.perf_counter() - t0
    fluid = int((mask == 0).sum())
    K = nv[0] * nv[1]
    o.close()
    return {"value": fluid * K * more / dt, "unit": "cell-velocity updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d iterations of the same 512x512 workload after 1 untimed iteration "
                      "(%.1f s of CPU work)" % (more, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--kn", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttr", action="store_true")
    ap.add_argument("--tile", type=int, nargs="*", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1712_01132_amd import geometry, poredvm

    torch.cuda.set_device(0)
    nv = [32, 32]
    log("generating the 512x512 rock (seed 1)")
    mask = geometry.workload_rock2d(seed=1)
    fluid = int((mask == 0).sum())
    K = nv[0] * nv[1]
    log("porosity %.4f, fluid voxels %d, velocities %d" % (1 - mask.mean(), fluid, K))

    s = poredvm.Solver(mask, nv, args.kn, precision=args.precision, tile=args.tile)
    s.iterate(args.warmup)
    torch.cuda.synchronize()
    log("warmup done (%d iterations)" % args.warmup)
    t0 = time.perf_counter()
    r = s.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r["iters"] == args.steps, r
    ups = fluid * K * args.steps / dt
    log("timed %d iterations: %.3f ms/iter, %.3e updates/s" % (args.steps, 1e3 * dt / args.steps, ups))

    tm = s.time_kernels(10)
    es = 8 if args.precision == "fp64" else 4
    sweep_bytes = es * fluid * K  # h written once per fluid voxel and velocity
    per_launch_bytes = sweep_bytes / tm["sweep_launches_per_iter"]
    per_launch_s = tm["sweep_ms_per_launch"] * 1e-3
    achieved = per_launch_bytes / per_launch_s / 1e9
    log("kernel timing: %s" % json.dumps(tm))
    mom_gbs = sweep_bytes / (tm["moments_ms_per_launch"] * 1e-3) / 1e9
    s.close()

    out = {
        "metric": "cell-velocity updates/s (time-to-residual 1e-6 reported alongside)",
        "value": ups,
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "rock2d: 512x512 seeded overlapping discs r~U(4,20), porosity 0.40, "
                               "Kn=%g, 32x32 half-range Gauss-Hermite velocities, %s sweep" % (args.kn, args.precision),
                   "fluid_voxels": fluid, "velocities": K, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_kernel", "bytes_per_launch": per_launch_bytes,
                     "launch_ms": tm["sweep_ms_per_launch"],
                     "launches_per_iter": tm["sweep_launches_per_iter"],
                     "moments_kernel_gbs": mom_gbs},
    }
    if not args.no_ttr:
        ttr = {}
        for prec in ("fp64", "fp32"):
            s = poredvm.Solver(mask, nv, args.kn, precision=prec, tile=args.tile)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rr = s.iterate(20000, 1e-6)
            torch.cuda.synchronize()
            ttr[prec] = {"seconds": time.perf_counter() - t0, "iterations": rr["iters"], "k": rr["k"],
                         "converged": rr["converged"]}
            s.close()
            log("time to r<=1e-6 (%s): %s" % (prec, json.dumps(ttr[prec])))
        ttr["k_rel_diff_fp32_vs_fp64"] = abs(ttr["fp32"]["k"] - ttr["fp64"]["k"]) / abs(ttr["fp64"]["k"])
        out["time_to_residual_1e-6"] = ttr
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the same workload")
        out["cpu_baseline"] = cpu_baseline(mask, nv, args.kn)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
