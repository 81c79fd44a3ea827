"""Sweep schedule and tile autotuner.

The sweep kernel is compiled for square tile edges 4 and 8 in (x1, x2). A tile
may be narrower than its compiled edge along either axis and of any depth
along x3. The best shape depends on the problem size (tiles per tile diagonal
against diagonals per iteration), on the precision and on the number of
velocity groups; for batches and 3D problems the schedule (per-XCD queues of
tiles, or in 3D of tile columns, in one launch, or one launch per tile
diagonal) is tuned with it.
`best_config` times each candidate with the library's own per-kernel HIP-event
timing (pdvm_time_kernels) on the real problem, or on the real batch, and
keeps the fastest per size class. The choice is cached in a JSON file
(PDVM_AUTOTUNE_CACHE, default ~/.cache/poredvm/autotune.json).
"""
import json
import math
import os

import numpy as np

from . import poredvm

CANDIDATES_2D = [(8, 8), (4, 4), (8, 4), (4, 8)]
CANDIDATES_3D = [(4, 4, 4), (4, 4, 8), (4, 4, 16), (8, 8, 4), (8, 8, 8)]


def cache_path():
    return os.environ.get("PDVM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "poredvm", "autotune.json"))


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home only costs re-tuning


def size_class(shapes, nv, precision):
    """Key of a problem (or batch): dimension, precision, velocity count and
    the sides rounded up to powers of two (the largest over a batch)."""
    dim = len(shapes[0])
    side = [max(s[-1 - a] for s in shapes) for a in range(dim)]
    cls = [2 ** int(math.ceil(math.log2(max(x, 2)))) for x in side]
    K = int(np.prod(nv))
    return "d%d-%s-K%d-n%s-p%d" % (dim, precision, K, "x".join(map(str, cls)), len(shapes))


def _time(make, iters):
    s = make()
    try:
        s.iterate(2)
        t = s.time_kernels(iters)
        return t["iter_ms"]
    finally:
        s.close()


# Sweep schedules the tuner compares besides the automatic choice: the
# per-XCD tile queues (one launch per iteration) and the per-diagonal launches
# for 3D problems and batches, and in 3D also the queues of tile columns. (A
# single 2D problem keeps the row pipeline, measured 2-2.5x faster than both
# on the 512^2 rock.)
SCHEDULES_MULTI = ("queue", "diagonals")
SCHEDULES_3D = ("columns", "queue", "diagonals")


def best_config(problems, nv, precision="fp32", iters=5, candidates=None, schedules=None, use_cache=True,
                verbose=False):
    """Fastest (schedule, tile) for `problems`: one mask, or a list of
    (mask, kn) for a batch (timed as a batch). Returns ((schedule, tile),
    {"schedule:tile": ms per iteration})."""
    batch = isinstance(problems, list)
    shapes = [m.shape for m, _ in problems] if batch else [problems.shape]
    dim = len(shapes[0])
    cands = candidates or (CANDIDATES_2D if dim == 2 else CANDIDATES_3D)
    if schedules is None:
        schedules = SCHEDULES_3D if dim == 3 else (SCHEDULES_MULTI if batch else ("auto",))
    key = "+".join(schedules) + "-" + size_class(shapes, nv, precision)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return (cache[key]["schedule"], tuple(cache[key]["tile"])), cache[key]["ms"]
    res = {}
    for sched in schedules:
        for tile in cands:
            if batch:
                def make(tile=tile, sched=sched):
                    return poredvm.Batch(problems, nv, precision=precision, tile=list(tile), schedule=sched)
            else:
                def make(tile=tile, sched=sched):
                    return poredvm.Solver(problems, nv, 1.0, precision=precision, tile=list(tile), schedule=sched)
            try:
                res[(sched, tile)] = _time(make, iters)
            except poredvm.PdvmError as e:
                if e.code != poredvm.PDVM_E_UNSUPPORTED:
                    raise
                continue  # e.g. the queue without blocks on every XCD
            if verbose:
                print("[autotune] %s %s tile %s: %.3f ms/iteration" % (key, sched, tile, res[(sched, tile)]),
                      flush=True)
    best = min(res, key=res.get)
    ms = {"%s:%s" % (k[0], "x".join(map(str, k[1]))): v for k, v in res.items()}
    if use_cache:
        cache = _load_cache()
        cache[key] = {"schedule": best[0], "tile": list(best[1]), "ms": ms}
        _save_cache(cache)
    return best, ms


def best_tile(problems, nv, precision="fp32", iters=5, candidates=None, use_cache=True, verbose=False):
    """Fastest tile for `problems` under the automatic schedule. Returns
    (tile, {tile: ms per iteration})."""
    (_, tile), ms = best_config(problems, nv, precision, iters, candidates, schedules=("auto",),
                                use_cache=use_cache, verbose=verbose)
    return tile, {k.split(":", 1)[1]: v for k, v in ms.items()}
