"""Sweep-tile autotuner.

The sweep kernel is compiled for square tile edges 4 and 8 in (x1, x2). A tile
may be narrower than its compiled edge along either axis and of any depth
along x3. The best shape depends on the problem size (tiles per tile diagonal
against diagonals per iteration), on the precision and on the number of
velocity groups. `best_tile` times each candidate with the library's own
per-kernel HIP-event timing (pdvm_time_kernels) on the real problem, or on the
real batch, and keeps the fastest per size class. The choice is cached in a
JSON file (PDVM_AUTOTUNE_CACHE, default ~/.cache/poredvm/autotune.json).
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


def best_tile(problems, nv, precision="fp32", iters=5, candidates=None, use_cache=True, verbose=False):
    """Fastest tile for `problems`: one mask, or a list of (mask, kn) for a
    batch (timed as a batch). Returns (tile, {tile: ms per iteration})."""
    batch = isinstance(problems, list)
    shapes = [m.shape for m, _ in problems] if batch else [problems.shape]
    key = size_class(shapes, nv, precision)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["tile"]), cache[key]["ms"]
    dim = len(shapes[0])
    cands = candidates or (CANDIDATES_2D if dim == 2 else CANDIDATES_3D)
    res = {}
    for tile in cands:
        if batch:
            def make(tile=tile):
                return poredvm.Batch(problems, nv, precision=precision, tile=list(tile))
        else:
            def make(tile=tile):
                return poredvm.Solver(problems, nv, 1.0, precision=precision, tile=list(tile))
        res[tile] = _time(make, iters)
        if verbose:
            print("[autotune] %s tile %s: %.3f ms/iteration" % (key, tile, res[tile]), flush=True)
    best = min(res, key=res.get)
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tile": list(best), "ms": {"x".join(map(str, k)): v for k, v in res.items()}}
        _save_cache(cache)
    return best, {"x".join(map(str, k)): v for k, v in res.items()}
