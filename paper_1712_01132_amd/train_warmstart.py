"""Train the warm-start network on fields the iteration itself converges.

    python -m paper_1712_01132_amd.train_warmstart --train 1024 --heldout 64 \\
        --out paper_1712_01132_amd/weights/warmstart_unet.npz

1. Draws the seeded 256 x 256 disc geometries (training seeds 10000.., held-out
   seeds 20000..; Kn log-uniform in [0.05, 20]).
2. Solves them with the batched FP32 iteration (24 x 24 half-range
   Gauss-Hermite velocities) until r <= --tol or --max-iters.
3. Stores the fields in the network's device-resident training set.
4. Trains with Adam (cosine learning-rate decay) in the library's bf16
   matrix-core kernels.
5. Saves the weights.
6. Compares the iterations from rest and from the network's prediction on the
   held-out problems.

Progress goes to stderr, one line per solved chunk and per epoch.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def log(msg):
    print("[train] " + msg, file=sys.stderr, flush=True)


def solve_chunk(probs, nv, tol, max_iters, precision="fp32", starts=None, step=1000):
    """Iterate a batch of (mask, kn) problems until each meets r <= tol (it then
    retires) or max_iters. Returns per-problem stats (taken when the problem
    first met the tolerance) and the final fields."""
    from . import poredvm
    b = poredvm.Batch(probs, nv, precision=precision, tile=[8, 8])
    if starts is not None:
        for i, (rho, u) in enumerate(starts):
            b.set_initial(i, rho, u)
    done = 0
    first = [None] * len(probs)
    st = None
    while done < max_iters:
        st = b.iterate(min(step, max_iters - done), tol)
        done += step
        for i, s in enumerate(st):
            if first[i] is None and s["converged"]:
                first[i] = s
        if all(f is not None for f in first):
            break
    fields = [b.moments(i) for i in range(len(probs))]
    b.close()
    return [f if f is not None else s for f, s in zip(first, st)], fields


def mirrored(mask, rho, u, jump=1.0, flip_x1=False, flip_x2=False):
    """The same problem reflected: mirroring the geometry across x2 mirrors
    the solution with u2 -> -u2. Mirroring across x1 reverses the driving, so
    the mirrored solution is negated to restore it: the density deviation from
    the ramp -J (x1 - 1/2) and u2 change sign, u1 does not. Both hold exactly
    for the discrete iteration up to its free density constant, because the
    octant sweeps, the images and the jump rule are mirror-symmetric."""
    n2, n1 = mask.shape
    x1 = (np.arange(n1) + 0.5) / n1
    ramp = -jump * (x1[None, :] - 0.5)
    dev = rho - ramp
    u1, u2 = u[0].copy(), u[1].copy()
    m = mask
    if flip_x2:
        m, dev, u1, u2 = m[::-1, :], dev[::-1, :], u1[::-1, :], -u2[::-1, :]
    if flip_x1:
        m, dev, u1, u2 = m[:, ::-1], -dev[:, ::-1], u1[:, ::-1], -u2[:, ::-1]
    rho2 = np.where(m != 0, 0.0, dev + ramp)
    return np.ascontiguousarray(m), np.ascontiguousarray(rho2), np.ascontiguousarray(np.stack([u1, u2]))


def _aug(m, rho, u, a):
    mm, rr, uu = mirrored(m, rho, u, flip_x1=bool(a & 1), flip_x2=bool(a & 2))
    return mm, rr, uu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=1024)
    ap.add_argument("--heldout", type=int, default=64)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--nv", type=int, default=24)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iters", type=int, default=4000)
    ap.add_argument("--chunk", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval", type=int, default=64, help="held-out problems for the warm/cold comparison")
    ap.add_argument("--eval-tol", type=float, default=1e-5)
    ap.add_argument("--eval-max-iters", type=int, default=8000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--augment", type=int, default=1, help="add the three mirror images of every training sample")
    args = ap.parse_args()

    import torch
    from . import geometry, warmstart
    torch.cuda.set_device(0)
    t0 = time.time()
    n = args.size
    nv = [args.nv, args.nv]
    seeds = list(range(10000, 10000 + args.train)) + list(range(20000, 20000 + args.heldout))
    probs = [geometry.workload_warmstart(s, n) for s in seeds]
    log("drew %d geometries in %.1f s" % (len(probs), time.time() - t0))

    naug = 4 if args.augment else 1
    ntrain = args.train * naug
    net = warmstart.Net(n, n, batch_max=args.batch, dataset_max=ntrain + args.heldout)
    gen = {"iters": [], "converged": 0, "r": []}
    held_fields = []
    for c0 in range(0, len(probs), args.chunk):
        chunk = probs[c0:c0 + args.chunk]
        tc = time.time()
        st, fields = solve_chunk(chunk, nv, args.tol, args.max_iters)
        for i, ((m, kn), (rho, u)) in enumerate(zip(chunk, fields)):
            j = c0 + i
            if j < args.train:
                net.set_sample(j * naug, m, kn, rho, u)
                for a in range(1, naug):
                    ma, ra, ua = _aug(m, rho, u, a)
                    net.set_sample(j * naug + a, ma, kn, ra, ua)
            else:
                net.set_sample(ntrain + j - args.train, m, kn, rho, u)
                held_fields.append((rho, u))
        gen["iters"] += [s["total_iters"] for s in st]
        gen["r"] += [s["r"] for s in st]
        gen["converged"] += sum(s["converged"] for s in st)
        log("solved %d/%d: %.1f s, median iterations %d, converged %d/%d" % (
            c0 + len(chunk), len(probs), time.time() - tc, int(np.median([s["total_iters"] for s in st])),
            sum(s["converged"] for s in st), len(chunk)))
    gen_s = time.time() - t0

    # training
    rng = np.random.default_rng(args.seed)
    net.set_params(warmstart.init_params(args.seed))
    train_slots = np.arange(ntrain)
    held_slots = np.arange(ntrain, ntrain + args.heldout)
    steps_per_epoch = ntrain // args.batch
    total = steps_per_epoch * args.epochs
    history = []
    best = (float("inf"), -1, None)
    tt = time.time()
    step = 0

    def held_loss():
        vals = []
        for i in range(0, len(held_slots) - args.batch + 1, args.batch):
            vals.append(net.train_step(held_slots[i:i + args.batch], update=False))
        return float(np.mean(vals)) if vals else float("nan")

    for ep in range(args.epochs):
        perm = rng.permutation(train_slots)
        losses = []
        for i in range(steps_per_epoch):
            lr = args.lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * step / total)))
            losses.append(net.train_step(perm[i * args.batch:(i + 1) * args.batch], lr=lr))
            step += 1
        hl = held_loss()
        history.append((float(np.mean(losses)), hl))
        if hl < best[0]:
            best = (hl, ep, net.params())
        log("epoch %d: train loss %.4e, held-out loss %.4e, %.1f s" % (ep, history[-1][0], hl, time.time() - tt))
    train_s = time.time() - tt
    timing = net.time(train_slots[:args.batch], reps=5)
    params = best[2]  # the epoch with the lowest held-out loss
    net.set_params(params)
    meta = {"train": args.train, "heldout": args.heldout, "size": n, "nv": args.nv, "tol": args.tol,
            "max_iters": args.max_iters, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "train_loss": [h[0] for h in history], "heldout_loss": [h[1] for h in history],
            "gen_seconds": gen_s, "train_seconds": train_s, "gen_median_iters": float(np.median(gen["iters"])),
            "gen_converged": gen["converged"], "timing": timing, "best_epoch": best[1],
            "augment": naug}
    if args.out:
        warmstart.save_weights(params, args.out, meta=json.dumps(meta))
        log("saved %s" % args.out)

    # warm versus cold on held-out problems
    ne = min(args.eval, args.heldout)
    if ne > 0:
        evp = probs[args.train:args.train + ne]
        starts = [net.predict(m, kn) for m, kn in evp]
        sc, _ = solve_chunk(evp, nv, args.eval_tol, args.eval_max_iters)
        sw, _ = solve_chunk(evp, nv, args.eval_tol, args.eval_max_iters, starts=starts)
        sr, _ = solve_chunk(evp, nv, args.eval_tol, args.eval_max_iters,
                            starts=[warmstart.ramp_start(m) for m, _ in evp])
        ic = np.array([s["total_iters"] for s in sc])
        iw = np.array([s["total_iters"] for s in sw])
        ir = np.array([s["total_iters"] for s in sr])
        kc = np.array([s["k"] for s in sc])
        kw = np.array([s["k"] for s in sw])
        meta["eval"] = {"problems": ne, "tol": args.eval_tol, "cold_iters": ic.tolist(), "warm_iters": iw.tolist(),
                        "cold_converged": int(sum(s["converged"] for s in sc)),
                        "warm_converged": int(sum(s["converged"] for s in sw)),
                        "median_ratio": float(np.median(iw / ic)), "k_rel_diff_max": float(np.max(np.abs(kw - kc) / np.abs(kc))),
                        "ramp_iters": ir.tolist(), "median_ratio_ramp": float(np.median(ir / ic)),
                        "median_ratio_warm_vs_ramp": float(np.median(iw / ir))}
        log("held-out warm/cold iterations to r <= %g: median ratio %.3f, cold median %d, warm median %d, "
            "warm better in %d/%d" % (args.eval_tol, meta["eval"]["median_ratio"], int(np.median(ic)),
                                      int(np.median(iw)), int(np.sum(iw < ic)), ne))
        if args.out:
            warmstart.save_weights(params, args.out, meta=json.dumps(meta))
    print(json.dumps({k: v for k, v in meta.items() if k not in ("eval",)} | (
        {"eval_summary": {k: v for k, v in meta["eval"].items() if not k.endswith("_iters")}} if "eval" in meta else {})),
        flush=True)
    net.close()


if __name__ == "__main__":
    main()
