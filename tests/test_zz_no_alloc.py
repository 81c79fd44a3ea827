"""pdvm_iterate_noalloc against pdvm_iterate.

The no-allocation entry point runs the same kernels with their scratch
(per-block partial sums, the row pipeline's progress counters and XCD records)
in the library's static per-GPU array instead of the solver's workspace, and
without a HIP graph. Its iterates must equal pdvm_iterate's bit for bit, also
on a second, smaller solve that finds the array holding the first one's
contents.
"""
import numpy as np
import pytest

from paper_1712_01132_amd import geometry, poredvm

pytestmark = pytest.mark.gpu


def random_mask(shape, frac, seed):
    rng = np.random.default_rng(seed)
    while True:
        m = geometry.fill_nonpercolating((rng.random(shape) < frac).astype(np.uint8))
        if geometry.percolates(m) and m.sum() > 0:
            return m


def _same(a, b):
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("schedule,precision,nv", [
    ("auto", "fp64", [16, 16]),      # XCD-local row pipeline: counters and XCD records in the scratch
    ("strips", "fp32", [8, 8]),      # strip pipeline, likewise
    ("rows-agent", "fp32", [24, 24]),
    ("diagonals", "fp64", [8, 8]),
    ("queue", "fp32", [24, 24]),     # per-XCD tile queues: counters and done flags in the scratch
])
def test_noalloc_equals_iterate_twice_second_smaller(schedule, precision, nv):
    cases = [(random_mask((96, 88), 0.3, 41), 13), (random_mask((36, 30), 0.3, 42), 6)]
    for m, iters in cases:
        a = poredvm.Solver(m, nv, 0.6, precision=precision, schedule=schedule)
        b = poredvm.Solver(m, nv, 0.6, precision=precision, schedule=schedule)
        if schedule == "auto":
            assert b.schedule == "rows-xcd"
        if schedule in ("strips", "queue"):
            assert b.schedule == schedule
        ra = a.iterate(iters)
        rb = b.iterate_noalloc(iters)
        assert rb["iters"] == ra["iters"] == iters and rb["total_iters"] == iters
        assert rb["k"] == ra["k"] and rb["r"] == ra["r"]
        _same(a, b)
        # a second call on the same solver continues like pdvm_iterate
        ra = a.iterate(5)
        rb = b.iterate_noalloc(5)
        assert rb["k"] == ra["k"] and rb["total_iters"] == iters + 5
        _same(a, b)
        a.close()
        b.close()


def test_noalloc_stops_on_tolerance_like_iterate():
    m = random_mask((40, 44), 0.3, 43)
    a = poredvm.Solver(m, [8, 8], 1.0)
    b = poredvm.Solver(m, [8, 8], 1.0)
    ra = a.iterate(5000, 1e-7)
    rb = b.iterate_noalloc(5000, 1e-7)
    assert ra["converged"] and rb["converged"] and ra["iters"] == rb["iters"]
    assert ra["k"] == rb["k"]
    _same(a, b)


@pytest.mark.parametrize("schedule", ["auto", "queue", "columns"])
def test_noalloc_3d(schedule):
    """3D (the queue sweeps of tiles, also the automatic choice, and of tile
    columns): two solves in a row, the second smaller, finding the first
    one's counters and done flags in the scratch."""
    for shape, iters in (((20, 22, 24), 7), ((10, 12, 14), 5)):
        m = random_mask(shape, 0.25, 44)
        a = poredvm.Solver(m, [4, 4, 4], 0.7, precision="fp32", schedule=schedule)
        b = poredvm.Solver(m, [4, 4, 4], 0.7, precision="fp32", schedule=schedule)
        assert b.schedule == ("columns" if schedule == "columns" else "queue")
        a.iterate(iters)
        b.iterate_noalloc(iters)
        _same(a, b)
        a.close()
        b.close()
