#!/usr/bin/env python3
"""Benchmark of the DVM/BGK iteration on one MI355X.

Workload (the `value` line): 2D synthetic digital rock, 512 x 512 voxels of
seeded overlapping discs (radii U(4, 20) px, porosity 0.40, pore space
percolating along x1), Kn = 1 (L = 512 voxels), 32 x 32 half-range
Gauss-Hermite velocities, specular lateral faces, pressure jump 1, FP64.
A step is one full iteration of the hot path: the upwind sweep of every
discrete velocity, the moment / source / wall-density kernel and the FP64
residual and permeability reduction.

Prints one JSON line with cell-velocity updates per second (fluid voxels x
velocities x iterations / wall time, inputs resident in HBM), the roofline of
the dominant kernel (the sweep) from HIP-event timings on the solver's stream,
the CPU oracle timed on a bounded sample of the same workload, and extra
fields: the FP32 form, the 3D pack (96^3, 16^3 velocities, FP32), the
64-problem batch (24 x 24 velocities, FP32) and time-to-residual 1e-6.
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
            "sample": "%d iterations of the same 512x512 rock (Kn=1, 32x32 velocities) after one "
                      "untimed iteration, %.1f s of CPU work" % (more, dt)}


def timed_updates(solver, fluid, K, steps, warmup):
    import torch
    solver.iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = solver.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r["iters"] == steps, r
    return fluid * K * steps / dt, dt


# HBM bytes per sweep launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes
# (scaled by a 1 GiB copy; summaries in profiles/), valid only for the kernel
# source they were taken on. Key: (source hash, schedule, tile, bytes per value).
_H = "3e9c9fb2dde38e62"
TRAFFIC = {
    (_H, "rows-xcd", (4, 4), 8): 523.4e6 + 841.9e6,            # rock2d FP64
    (_H, "rows-xcd", (4, 4), 4): 264.1e6 + 421.4e6,            # rock2d FP32
    (_H, "queue", (4, 4, 4), 4): 12069.6e6 + 5104.0e6,         # pack3d FP32, 1 launch
    (_H, "columns", (4, 4, 4), 4): 13454.6e6 + 5096.5e6,       # pack3d FP32, 1 launch
    (_H, "queue", (8, 8), 4): 5960.5e6 + 4601.8e6,             # batch64 FP32, 1 launch
}
# the same for the moment kernel of that iteration (h read once, moments written)
MOM_TRAFFIC = {
    (_H, "rows-xcd", (4, 4), 8): 880.2e6 + 12.8e6,
    (_H, "rows-xcd", (4, 4), 4): 445.3e6 + 9.5e6,
    (_H, "queue", (4, 4, 4), 4): 5236.9e6 + 35.7e6,
    (_H, "columns", (4, 4, 4), 4): 5236.9e6 + 35.7e6,
    (_H, "queue", (8, 8), 4): 5821.9e6 + 184.4e6,
}


def kernel_source_hash():
    """sha256 prefix over the iteration's kernel sources (dvm_*.hip, dvm_*.h)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1712_01132_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "dvm_*.hip")) + glob.glob(os.path.join(csrc, "dvm_*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


SWEEP_KERNEL = {"diagonals": "sweep_kernel", "queue": "sweep_queue_kernel", "columns": "sweep_queue_kernel",
                "strips": "sweep_strips_kernel",
                "rows": "sweep_rows_kernel", "rows-xcd": "sweep_rows_kernel"}


def roofline(tm, elem, traffic_key=None, schedule="diagonals"):
    """Sweep kernel: algorithmic bytes = h written once per fluid voxel and
    velocity; per launch = that over the launches of one iteration."""
    per_iter = elem * tm["fluid_cells"] * tm["velocities"]
    per_launch = per_iter / tm["sweep_launches_per_iter"]
    achieved = per_launch / (tm["sweep_ms_per_launch"] * 1e-3) / 1e9
    traffic = TRAFFIC.get(traffic_key) if traffic_key else None
    mom_traffic = MOM_TRAFFIC.get(traffic_key) if traffic_key else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": SWEEP_KERNEL.get(schedule, schedule),
            "bytes_per_launch": per_launch, "launch_ms": tm["sweep_ms_per_launch"],
            "launches_per_iter": tm["sweep_launches_per_iter"],
            "moments_kernel": {"bytes_per_launch": per_iter, "launch_ms": tm["moments_ms_per_launch"],
                               "achieved_gbs": per_iter / (tm["moments_ms_per_launch"] * 1e-3) / 1e9,
                               "traffic": mom_traffic}}


# Workloads of --only: (what, precision, default tile)
ONLY = {"rock2d-fp64": ("rock2d", "fp64", (4, 4)), "rock2d-fp32": ("rock2d", "fp32", (4, 4)),
        "pack3d-fp32": ("pack3d", "fp32", (4, 4, 4)), "batch64-fp32": ("batch64", "fp32", (8, 8)),
        "unet-train": ("unet", "bf16", None)}


def only_workload(args):
    """One workload alone, for rocprofv3 runs: `--warmup` untimed and
    `--steps` timed iterations (training steps for the network)."""
    import torch
    from paper_1712_01132_amd import geometry, poredvm
    what, prec, tile = ONLY[args.only]
    tile = tuple(args.tile) if args.tile else tile
    torch.cuda.set_device(0)
    if what == "unet":
        import numpy as np
        from paper_1712_01132_amd import warmstart
        B = 8
        net = warmstart.Net(256, 256, batch_max=B, dataset_max=B)
        net.set_params(warmstart.init_params(0))
        for i in range(B):
            m, kn = geometry.workload_warmstart(20000 + i)
            net.set_sample(i, m, kn, np.zeros(m.shape), np.zeros((2,) + m.shape))
        net.time(list(range(B)), reps=max(1, args.warmup))
        t = net.time(list(range(B)), reps=max(1, args.steps))
        net.close()
        print(json.dumps({"workload": args.only, "timing": t}), flush=True)
        return
    if what == "batch64":
        probs = geometry.workload_batch(64)
        s = poredvm.Batch(probs, [24, 24], precision=prec, tile=list(tile), schedule=args.schedule)
        fluid, K = sum(int((m == 0).sum()) for m, _ in probs), 576
    else:
        m = geometry.workload_rock2d(seed=1) if what == "rock2d" else geometry.workload_pack3d(seed=7)
        nv, kn = ([32, 32], args.kn) if what == "rock2d" else ([16, 16, 16], 0.5)
        s = poredvm.Solver(m, nv, kn, precision=prec, tile=list(tile), schedule=args.schedule)
        fluid, K = int((m == 0).sum()), 1024 if what == "rock2d" else 4096
    if what == "batch64":
        s.iterate(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ups = fluid * K * args.steps / dt
    else:
        ups, dt = timed_updates(s, fluid, K, args.steps, args.warmup)
    sched = s.schedule
    s.close()
    print(json.dumps({"workload": args.only, "schedule": sched, "tile": list(tile), "steps": args.steps,
                      "ms_per_step": 1e3 * dt / args.steps, "updates_per_s": ups,
                      "kernel_source": kernel_source_hash()}), flush=True)


def copy_calibration(mib):
    """A plain device copy of known size: each launch reads and writes
    mib MiB, so FETCH_SIZE / WRITE_SIZE of this kernel give the counters'
    scale."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 3}), flush=True)


SWITCH_TOL = 2e-6      # FP32 phase ends here (its rounding floor on this workload is about 1e-6)
FP32_MAX_ITERS = 40000
TTR_MAX_ITERS = 60000


def _fields(s):
    """rho, u, tau and q of a solver (FP64 host arrays)."""
    rho, u, tau, q = s.moments(diagnostics=True)
    return {"rho": rho, "u": u, "tau": tau, "q": q}


def field_errors(f32, k32, f64, k64, mask):
    """Errors of one solution against another, relative to the other's range
    over the fluid voxels: max |a - b| / max |b| for rho and tau minus their
    fluid means and for u and q (all components); |k_a - k_b| / |k_b|."""
    import numpy as np
    fl = mask == 0

    def rel(a, b, centre):
        a = a[..., fl]
        b = b[..., fl]
        if centre:
            a = a - a.mean()
            b = b - b.mean()
        sc = float(np.abs(b).max())
        return float(np.abs(a - b).max()) / (sc if sc > 0 else 1.0)

    return {"rho_minus_mean": rel(f32["rho"], f64["rho"], True), "u": rel(f32["u"], f64["u"], False),
            "tau_minus_mean": rel(f32["tau"], f64["tau"], True), "q": rel(f32["q"], f64["q"], False),
            "k": abs(k32 - k64) / abs(k64)}


def _ttr_fp64(mask, nv, kn, tile, tol=1e-6, ramp=False, keep=None):
    from paper_1712_01132_amd import poredvm, warmstart
    s = poredvm.Solver(mask, nv, kn, precision="fp64", tile=tile)
    if ramp:
        s.set_initial(*warmstart.ramp_start(mask))
    t0 = time.perf_counter()
    r = s.iterate(TTR_MAX_ITERS, tol)
    dt = time.perf_counter() - t0
    if keep is not None:
        keep["fields"] = _fields(s)
    s.close()
    return {"seconds": dt, "iterations": r["total_iters"], "k": r["k"], "converged": r["converged"]}


def _ttr_fp32_alone(mask, nv, kn, tile32, net=None, trial=50, tol=1e-6, keep=None):
    """The FP32 iteration by itself to r <= tol (the offset form of h reaches
    it), from the pressure ramp or from a network's prediction judged against
    the ramp as in _ttr_fp32_then_fp64."""
    from paper_1712_01132_amd import poredvm, warmstart
    t0 = time.perf_counter()
    used = False
    if net is not None:
        start = net.predict(mask, kn)
        a, used, _, _ = warmstart.judged_start(mask, nv, kn, start, trial=trial, precision="fp32", tile=tile32)
    else:
        a = poredvm.Solver(mask, nv, kn, precision="fp32", tile=tile32)
        a.set_initial(*warmstart.ramp_start(mask))
    r = a.iterate(TTR_MAX_ITERS, tol)
    dt = time.perf_counter() - t0
    if keep is not None:
        keep["fields"] = _fields(a)
    a.close()
    return {"seconds": dt, "iterations": r["total_iters"], "k": r["k"], "converged": r["converged"],
            "warm_start_used": used}


def _ttr_fp32_then_fp64(mask, nv, kn, tile, tile32, net=None, trial=50, tol=1e-6, ramp=False):
    """FP32 iterations until r <= SWITCH_TOL, then the FP64 iteration from the
    exact FP32 state. From rest, from the pressure ramp (ramp=True), or with a
    network: its prediction and the ramp are each run `trial` iterations in
    FP32 and the start with the smaller residual goes on."""
    from paper_1712_01132_amd import poredvm, warmstart
    b = poredvm.Solver(mask, nv, kn, precision="fp64", tile=tile)
    t0 = time.perf_counter()
    used = False
    if net is not None:
        start = net.predict(mask, kn)
        a, used, _, _ = warmstart.judged_start(mask, nv, kn, start, trial=trial, precision="fp32", tile=tile32)
    else:
        a = poredvm.Solver(mask, nv, kn, precision="fp32", tile=tile32)
        if ramp:
            a.set_initial(*warmstart.ramp_start(mask))
    r32 = a.iterate(FP32_MAX_ITERS, SWITCH_TOL)
    b.set_state(a.get_state())
    r64 = b.iterate(TTR_MAX_ITERS, tol)
    dt = time.perf_counter() - t0
    a.close()
    b.close()
    return {"seconds": dt, "iterations": r64["total_iters"], "fp32_iterations": r32["total_iters"],
            "k": r64["k"], "converged": r64["converged"], "warm_start_used": used}


BF16_PEAK_TFLOPS = 2500.0


def unet_source_hash():
    """sha256 prefix over the network's kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for f in ("unet_kernels.hip", "unet_internal.h"):
        h.update(f.encode())
        with open(os.path.join(ROOT, "paper_1712_01132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# HBM bytes of one training step's MFMA kernels (FETCH_SIZE / WRITE_SIZE,
# scaled; profiles/unet_train_bf16.md), by network source hash
UNET_TRAFFIC = {"ddf9230b001a6b44": 5477.1e6 + 1223.3e6}


def unet_timing():
    """The network's bf16 matrix-core kernels at the training shape (8 samples
    of 256 x 256): forward pass and training step (forward, backward, Adam)."""
    import numpy as np
    from paper_1712_01132_amd import geometry, warmstart
    B = 8
    net = warmstart.Net(256, 256, batch_max=B, dataset_max=B)
    net.set_params(warmstart.init_params(0))
    for i in range(B):
        m, kn = geometry.workload_warmstart(20000 + i)
        net.set_sample(i, m, kn, np.zeros(m.shape), np.zeros((2,) + m.shape))
    net.time(list(range(B)), reps=2)
    t = net.time(list(range(B)), reps=10)
    net.close()
    fwd = t["forward_flop"] / (t["forward_ms"] * 1e-3) / 1e12
    step_mfma = t["step_flop"] / (t["mfma_ms_per_step"] * 1e-3) / 1e12
    res = {"batch": B, "size": [256, 256], "forward_ms": t["forward_ms"], "step_ms": t["step_ms"],
           "forward_tflops": fwd, "step_tflops": t["step_flop"] / (t["step_ms"] * 1e-3) / 1e12,
           "mfma_kernels_ms_per_step": t["mfma_ms_per_step"],
           "roofline": {"bound": "mfma", "achieved": step_mfma, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": step_mfma / BF16_PEAK_TFLOPS, "traffic": UNET_TRAFFIC.get(unet_source_hash()),
                        "note": "convolution FLOP of one training step / summed durations of its MFMA kernels; "
                                "traffic: HBM bytes of those kernels per step"}}
    log("warm-start network: %s" % json.dumps(res))
    return res


def warmstart_heldout(n=16, tol=1e-6, max_iters=30000):
    """Held-out geometries of the warm-start set (seeds 20000.., never
    trained on): the unchanged FP32 iteration to r <= tol from rest, from the
    pressure ramp and from the network's prediction (unjudged), each start as
    one batch of the n problems. Iterations per problem and the batch's wall
    time (it ends with its slowest problem)."""
    import numpy as np
    import torch
    from paper_1712_01132_amd import geometry, poredvm, warmstart
    probs = [geometry.workload_warmstart(20000 + i) for i in range(n)]
    try:
        params, _ = warmstart.load_weights()
    except (OSError, KeyError) as e:
        return {"skipped": "no trained weights (%s)" % e}
    net = warmstart.Net(256, 256, batch_max=1, dataset_max=0)
    net.set_params(params)
    t0 = time.perf_counter()
    pred = [net.predict(m, kn) for m, kn in probs]
    t_pred = time.perf_counter() - t0
    net.close()
    starts = {"cold": None, "ramp": [warmstart.ramp_start(m) for m, _ in probs], "warm": pred}
    out = {"problems": n, "seeds": [20000, 20000 + n - 1], "tol": tol, "precision": "fp32",
           "prediction_seconds": t_pred}
    for name in ("cold", "ramp", "warm"):
        b = poredvm.Batch(probs, [24, 24], precision="fp32", tile=[8, 8])
        if starts[name] is not None:
            for i, (rho, u) in enumerate(starts[name]):
                b.set_initial(i, rho, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = b.iterate(max_iters, tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        it = [int(x["total_iters"]) for x in st]
        out[name] = {"iterations": it, "sum": int(np.sum(it)), "median": float(np.median(it)),
                     "max": int(np.max(it)), "converged": int(sum(x["converged"] for x in st)), "seconds": dt}
        log("held-out %s: %s" % (name, json.dumps(out[name])))
    w, r, c = (np.array(out[k]["iterations"], dtype=float) for k in ("warm", "ramp", "cold"))
    out["warm_vs_ramp"] = {"sum_ratio": float(w.sum() / r.sum()), "median_ratio": float(np.median(w / r)),
                           "better": int((w < r).sum())}
    out["warm_vs_cold"] = {"sum_ratio": float(w.sum() / c.sum()), "median_ratio": float(np.median(w / c)),
                           "better": int((w < c).sum())}
    return out


def model_timing(mask, nv, kn, fluid, K, steps=40, warmup=5):
    """The same 512^2 rock in FP64 with the other models: updates/s count the
    distribution's velocities only (psi, where present, is extra work)."""
    from paper_1712_01132_amd import poredvm
    # all on the row pipeline with 4x4 tiles (the autotuner's choice for this rock)
    cases = {
        "bgk_tau_feedback_psi": dict(tau_feedback=True),
        "shakhov_pr_2_3": dict(tau_feedback=True, prandtl=2.0 / 3.0),
        "maxwell_walls_alpha_0.8": dict(accommodation=0.8),
        "shakhov_maxwell_walls": dict(tau_feedback=True, prandtl=2.0 / 3.0, accommodation=0.8),
    }
    res = {}
    for name, kw in cases.items():
        s = poredvm.Solver(mask, nv, kn, precision="fp64", tile=[4, 4], **kw)
        ups, dt = timed_updates(s, fluid, K, steps, warmup)
        res[name] = {"updates_per_s": ups, "ms_per_step": 1e3 * dt / steps, "schedule": s.schedule}
        s.close()
        log("model %s: %.3e updates/s (%s)" % (name, ups, res[name]["schedule"]))
    return res


def time_to_residual(mask, nv, kn, tile, tile32):
    out = {}
    f64 = {}
    log("time to r<=1e-6, FP64 from rest")
    out["fp64"] = _ttr_fp64(mask, nv, kn, tile, keep=f64)
    log("  %s" % json.dumps(out["fp64"]))
    log("time to r<=1e-6, FP32 alone from the pressure ramp")
    f32 = {}
    out["fp32_ramp_alone"] = _ttr_fp32_alone(mask, nv, kn, tile32, keep=f32)
    out["fp32_ramp_alone"]["errors_vs_fp64"] = field_errors(f32["fields"], out["fp32_ramp_alone"]["k"],
                                                            f64["fields"], out["fp64"]["k"], mask)
    log("  %s" % json.dumps(out["fp32_ramp_alone"]))
    log("time to r<=1e-6, FP32 from rest, finished in FP64")
    out["fp32_then_fp64"] = _ttr_fp32_then_fp64(mask, nv, kn, tile, tile32)
    log("  %s" % json.dumps(out["fp32_then_fp64"]))
    log("time to r<=1e-6, FP32 from the pressure ramp rho = 1/2 - x1, finished in FP64")
    out["fp32_ramp_then_fp64"] = _ttr_fp32_then_fp64(mask, nv, kn, tile, tile32, ramp=True)
    log("  %s" % json.dumps(out["fp32_ramp_then_fp64"]))
    try:
        from paper_1712_01132_amd import warmstart
        params, _ = warmstart.load_weights()
    except (OSError, KeyError) as e:
        params = None
        out["fp32_warm_then_fp64"] = {"skipped": "no trained weights (%s)" % e}
    if params is not None:
        net = warmstart.Net(mask.shape[1], mask.shape[0], batch_max=1, dataset_max=0)
        net.set_params(params)
        log("time to r<=1e-6, FP32 from the network's prediction (50-iteration trial against the ramp), "
            "finished in FP64")
        res = _ttr_fp32_then_fp64(mask, nv, kn, tile, tile32, net=net, trial=50)
        out["fp32_warm_then_fp64"] = res
        log("  %s" % json.dumps(res))
        log("time to r<=1e-6, FP32 alone from the network's prediction (judged against the ramp)")
        fw = {}
        res = _ttr_fp32_alone(mask, nv, kn, tile32, net=net, trial=50, keep=fw)
        res["errors_vs_fp64"] = field_errors(fw["fields"], res["k"], f64["fields"], out["fp64"]["k"], mask)
        out["fp32_warm_alone"] = res
        log("  %s" % json.dumps(res))
        net.close()
    k64 = out["fp64"]["k"]
    for key in ("fp32_then_fp64", "fp32_ramp_then_fp64", "fp32_warm_then_fp64", "fp32_ramp_alone",
                "fp32_warm_alone"):
        if "k" in out[key]:
            out[key]["k_rel_diff_vs_fp64"] = abs(out[key]["k"] - k64) / abs(k64)
            out[key]["speedup_vs_fp64"] = out["fp64"]["seconds"] / out[key]["seconds"]
    out["note"] = ("seconds from the first iteration launch: network inference, the FP32 solvers' "
                   "creation, the 50-iteration trial and the FP32->FP64 handover are included; the FP64 "
                   "solver's creation and weight loading are not. r is the field residual "
                   "max|du|/max|u| in FP64. errors_vs_fp64: the FP32 solution at r <= 1e-6 against the "
                   "FP64 one at r <= 1e-6 (from rest), relative to the FP64 field's range over the fluid")
    return out


def pack3d_precision_errors(m3, tile3, sched3, tol=1e-6):
    """The 96^3 pack, Kn = 0.5: FP32 and FP64 each from the pressure ramp to
    r <= tol, per-result errors as in field_errors."""
    from paper_1712_01132_amd import poredvm, warmstart
    res, fields = {}, {}
    for prec in ("fp64", "fp32"):
        log("pack3d %s from the ramp to r<=%g" % (prec, tol))
        s = poredvm.Solver(m3, [16, 16, 16], 0.5, precision=prec, tile=tile3, schedule=sched3)
        s.set_initial(*warmstart.ramp_start(m3))
        t0 = time.perf_counter()
        r = s.iterate(20000, tol)
        res[prec] = {"seconds": time.perf_counter() - t0, "iterations": r["total_iters"], "k": r["k"],
                     "converged": r["converged"], "schedule": s.schedule}
        fields[prec] = _fields(s)
        s.close()
        log("  %s" % json.dumps(res[prec]))
    res["errors_vs_fp64"] = field_errors(fields["fp32"], res["fp32"]["k"], fields["fp64"], res["fp64"]["k"], m3)
    return res


def precision_errors(mask, nv, tile, tile32, kns=(0.1, 10.0), tol=1e-6):
    """FP32 against FP64 on the rock at other Kn: each from the pressure ramp
    to r <= tol, per-result errors as in field_errors."""
    out = {}
    for kn in kns:
        log("FP32 vs FP64 at Kn=%g, both from the ramp to r<=%g" % (kn, tol))
        f64, f32 = {}, {}
        a = _ttr_fp64(mask, nv, kn, tile, tol=tol, ramp=True, keep=f64)
        b = _ttr_fp32_alone(mask, nv, kn, tile32, tol=tol, keep=f32)
        out["kn_%g" % kn] = {"fp64": a, "fp32": b,
                             "errors_vs_fp64": field_errors(f32["fields"], b["k"], f64["fields"], a["k"], mask)}
        log("  %s" % json.dumps(out["kn_%g" % kn]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kn", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="only the 512^2 FP64 line")
    ap.add_argument("--tile", type=int, nargs="*", default=None,
                    help="sweep tile (default: chosen by the autotuner before the timed region)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 3 times (scale for HBM byte counters)")
    ap.add_argument("--only", choices=sorted(ONLY), default=None,
                    help="only run --steps iterations (after --warmup) of one workload with a given schedule "
                         "and tile, for profilers; prints one JSON line with its timing")
    ap.add_argument("--schedule", default="auto", help="sweep schedule for --only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.only:
        only_workload(args)
        return

    import torch
    from paper_1712_01132_amd import geometry, poredvm

    torch.cuda.set_device(0)
    nv = [32, 32]
    log("generating the 512x512 rock (seed 1)")
    mask = geometry.workload_rock2d(seed=1)
    fluid = int((mask == 0).sum())
    K = nv[0] * nv[1]
    log("porosity %.4f, fluid voxels %d, velocities %d" % (1 - mask.mean(), fluid, K))

    from paper_1712_01132_amd import autotune
    tile64, tune64 = (args.tile, None) if args.tile else autotune.best_tile(mask, nv, "fp64", use_cache=False)
    log("FP64 tile %s (autotuner: %s)" % (tile64, tune64))
    s = poredvm.Solver(mask, nv, args.kn, precision="fp64", tile=list(tile64))
    ups, dt = timed_updates(s, fluid, K, args.steps, args.warmup)
    log("FP64: %d iterations in %.3f s: %.3f ms/iter, %.3e updates/s" % (args.steps, dt, 1e3 * dt / args.steps, ups))
    tm = s.time_kernels(10)
    sched64 = s.schedule
    log("FP64 kernel timing (%s schedule): %s" % (sched64, json.dumps(tm)))
    s.close()

    out = {
        "metric": "cell-velocity updates/s (time-to-residual 1e-6 alongside)",
        "value": ups,
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rock2d: 512x512 seeded overlapping discs r~U(4,20), porosity 0.40, Kn=%g, "
                               "32x32 half-range Gauss-Hermite velocities, FP64" % args.kn,
                   "fluid_voxels": fluid, "velocities": K, "parallelism": "1 GPU",
                   "tile": list(tile64), "autotune_ms_per_iteration": tune64},
        "roofline": roofline(tm, 8, (kernel_source_hash(), sched64, tuple(tile64), 8), sched64),
    }
    if not args.no_extra:
        extra = {}
        tile32, tune32 = (args.tile, None) if args.tile else autotune.best_tile(mask, nv, "fp32", use_cache=False)
        s = poredvm.Solver(mask, nv, args.kn, precision="fp32", tile=list(tile32))
        u32, d32 = timed_updates(s, fluid, K, args.steps, args.warmup)
        t32 = s.time_kernels(10)
        sched32 = s.schedule
        s.close()
        extra["rock2d_fp32"] = {"updates_per_s": u32, "ms_per_step": 1e3 * d32 / args.steps,
                                "tile": list(tile32), "autotune_ms_per_iteration": tune32,
                                "roofline": roofline(t32, 4, (kernel_source_hash(), sched32, tuple(tile32), 4), sched32)}
        log("FP32: %.3e updates/s" % u32)
        # time to residual 1e-6: FP64 from rest, and the FP32 forms finished in FP64
        extra["rock2d_time_to_residual_1e-6"] = time_to_residual(mask, nv, args.kn, list(tile64), list(tile32))
        extra["rock2d_fp32_vs_fp64"] = precision_errors(mask, nv, list(tile64), list(tile32))
        # 3D pack
        log("generating the 96^3 sphere pack (seed 7)")
        m3 = geometry.workload_pack3d(seed=7)
        f3 = int((m3 == 0).sum())
        (sched3, tile3), tune3 = autotune.best_config(m3, [16, 16, 16], "fp32", iters=2, use_cache=False)
        log("3D schedule %s, tile %s (autotuner: %s)" % (sched3, tile3, tune3))
        s = poredvm.Solver(m3, [16, 16, 16], 0.5, precision="fp32", tile=list(tile3), schedule=sched3)
        u3, d3 = timed_updates(s, f3, 4096, 20, 3)
        t3 = s.time_kernels(3)
        s.close()
        extra["pack3d_fp32"] = {"updates_per_s": u3, "ms_per_step": 1e3 * d3 / 20, "fluid_voxels": f3,
                                "tile": list(tile3), "schedule": sched3, "autotune_ms_per_iteration": tune3,
                                "velocities": 4096,
                                "roofline": roofline(t3, 4, (kernel_source_hash(), sched3, tuple(tile3), 4), sched3)}
        log("3D pack FP32: %.3e updates/s, %s" % (u3, json.dumps(t3)))
        extra["pack3d_fp32_vs_fp64"] = pack3d_precision_errors(m3, list(tile3), sched3)
        # 64-problem batch
        log("generating the 64-problem batch")
        probs = geometry.workload_batch(64)
        fb = sum(int((m == 0).sum()) for m, _ in probs)
        (schedb, tileb), tuneb = autotune.best_config(probs, [24, 24], "fp32", iters=3, use_cache=False)
        log("batch schedule %s, tile %s (autotuner: %s)" % (schedb, tileb, tuneb))
        b = poredvm.Batch(probs, [24, 24], precision="fp32", tile=list(tileb), schedule=schedb)
        b.iterate(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb = b.iterate(30)
        torch.cuda.synchronize()
        db = time.perf_counter() - t0
        tb = b.time_kernels(3)
        b.close()
        extra["batch64_fp32"] = {"updates_per_s": fb * 576 * 30 / db, "ms_per_step": 1e3 * db / 30,
                                 "tile": list(tileb), "schedule": schedb, "autotune_ms_per_iteration": tuneb,
                                 "fluid_voxels": fb, "velocities": 576, "problems": 64,
                                 "roofline": roofline(tb, 4, (kernel_source_hash(), schedb, tuple(tileb), 4), schedb)}
        log("batch64 FP32: %.3e updates/s" % (fb * 576 * 30 / db))
        extra["warmstart_unet"] = unet_timing()
        extra["warmstart_heldout"] = warmstart_heldout()
        extra["rock2d_models_fp64"] = model_timing(mask, nv, args.kn, fluid, K)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the same workload")
        out["cpu_baseline"] = cpu_baseline(mask, nv, args.kn)
        log("CPU oracle: %s" % json.dumps(out["cpu_baseline"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
