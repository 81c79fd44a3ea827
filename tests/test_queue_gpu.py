"""The queue sweep (one launch per iteration, tiles taken from per-XCD queues
in diagonal order, each waiting for its upstream tiles' done flags) against the
per-diagonal launches: the same tile arithmetic on the same values, so every
iterate must be bitwise identical, in 2D and 3D, for single problems and
batches, with every source variant; and its fault path, forced from the host.
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


def run(m, nv, kn, sched, iters, **kw):
    s = poredvm.Solver(m, nv, kn, schedule=sched, **kw)
    assert s.schedule == sched
    r = s.iterate(iters)
    out = (s.moments(), r["k"], r["r"])
    s.close()
    return out


def same(a, b):
    (ma, ka, ra), (mb, kb, rb) = a, b
    for x, y in zip(ma, mb):
        assert np.array_equal(x, y)
    assert ka == kb and ra == rb


@pytest.mark.parametrize("shape,nv,tile,precision,lateral,rule", [
    ((12, 14, 16), [4, 4, 4], (4, 4, 4), "fp32", "specular", 1),
    ((13, 11, 17), [6, 6, 6], (4, 4, 3), "fp64", "specular", 1),
    ((10, 9, 12), [10, 10, 10], (4, 4, 1), "fp32", "periodic", 1),   # one-plane tiles: waits two tiles back
    ((11, 13, 10), [4, 4, 4], (3, 4, 5), "fp64", "specular", 0),
    ((16, 12, 14), [6, 6, 6], (8, 8, 2), "fp32", "specular", 1),
    ((9, 17, 11), [4, 6, 4], (8, 3, 4), "fp64", "periodic", 0),
    ((24, 20, 22), [8, 8, 8], (4, 4, 8), "fp32", "specular", 1),
    ((10, 12, 9), [4, 4, 4], (1, 4, 3), "fp64", "specular", 1),     # tiles one voxel wide along x1
    ((12, 9, 10), [6, 6, 6], (4, 1, 1), "fp32", "periodic", 0),     # ... along x2 and x3
])
def test_queue_equals_diagonals_bitwise_3d(shape, nv, tile, precision, lateral, rule):
    """Ragged tiles, tiles one voxel thick along x3, both stencil rules, both
    lateral conditions, one or several (partly empty) 64-velocity groups; tile
    items and column items."""
    m = random_mask(shape, 0.3, sum(shape) + 11)
    kw = dict(precision=precision, lateral=lateral, tile=tile, stencil_rule=rule)
    ref = run(m, nv, 0.6, "diagonals", 9, **kw)
    same(run(m, nv, 0.6, "queue", 9, **kw), ref)
    same(run(m, nv, 0.6, "columns", 9, **kw), ref)


@pytest.mark.parametrize("tile,precision", [((4, 4, 2), "fp32"), ((4, 4, 3), "fp64"), ((8, 8, 2), "fp32")])
def test_columns_skip_solid_tiles_bitwise(tile, precision):
    """Columns interrupted by tiles without fluid (solid slabs across x3 and a
    solid block): after such a tile the column reloads the planes below from
    h instead of carrying them."""
    m = random_mask((21, 13, 14), 0.2, 41)   # (x3, x2, x1)
    m[6:9] = 1                               # a slab across x3: whole tiles without fluid in every column
    m[12:18, 0:8, 0:8] = 1                   # a solid block: such tiles in some columns only
    m = geometry.fill_nonpercolating(m)
    assert geometry.percolates(m)
    kw = dict(precision=precision, lateral="specular", tile=tile)
    same(run(m, [6, 6, 6], 0.5, "columns", 8, **kw), run(m, [6, 6, 6], 0.5, "diagonals", 8, **kw))


@pytest.mark.parametrize("kw", [
    dict(tau_feedback=True),
    dict(tau_feedback=True, prandtl=2.0 / 3.0),
    dict(accommodation=0.6),
    dict(accommodation=0.7, tau_feedback=True, prandtl=0.5, precision="fp32"),
])
def test_queue_source_variants_3d(kw):
    m = random_mask((9, 10, 12), 0.25, 5)
    ref = run(m, [4, 4, 4], 0.8, "diagonals", 8, tile=(4, 4, 3), **kw)
    same(run(m, [4, 4, 4], 0.8, "queue", 8, tile=(4, 4, 3), **kw), ref)
    same(run(m, [4, 4, 4], 0.8, "columns", 8, tile=(4, 4, 3), **kw), ref)


@pytest.mark.parametrize("shape,nv,tile,precision,kw", [
    ((37, 29), [8, 8], (4, 4), "fp64", {}),
    ((33, 26), [24, 24], (8, 8), "fp32", dict(lateral="periodic")),
    ((40, 33), [16, 32], (8, 5), "fp32", dict(stencil_rule=0)),
    ((29, 40), [6, 10], (4, 4), "fp64", dict(tau_feedback=True)),
    ((37, 29), [8, 8], (4, 4), "fp64", dict(tau_feedback=True, prandtl=2.0 / 3.0)),
    ((43, 37), [8, 8], (8, 8), "fp32", dict(accommodation=0.65)),
    ((21, 30), [8, 8], (1, 4), "fp64", {}),                          # tiles one voxel wide along x1
    ((26, 19), [6, 6], (4, 1), "fp32", dict(stencil_rule=0)),         # ... along x2
])
def test_queue_equals_diagonals_bitwise_2d(shape, nv, tile, precision, kw):
    m = random_mask(shape, 0.3, sum(shape) + 5)
    same(run(m, nv, 0.7, "queue", 10, precision=precision, tile=tile, **kw),
         run(m, nv, 0.7, "diagonals", 10, precision=precision, tile=tile, **kw))


def test_queue_batch_equals_diagonals_bitwise():
    """A batch of uneven 2D problems (sizes and Kn differ) in one queue launch."""
    probs = [(random_mask(sh, 0.3, 60 + i), kn) for i, (sh, kn) in
             enumerate([((48, 40), 0.3), ((24, 36), 2.0), ((64, 64), 0.8), ((20, 20), 5.0), ((40, 56), 0.1)])]
    out = []
    for sched in ("queue", "diagonals"):
        b = poredvm.Batch(probs, [12, 12], precision="fp32", tile=(4, 4), schedule=sched)
        assert b.schedule == sched
        res = b.iterate(11)
        out.append(([b.moments(i) for i in range(len(probs))], [r["k"] for r in res]))
        b.close()
    (ma, ka), (mb, kb) = out
    assert ka == kb
    for a, b in zip(ma, mb):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_queue_batch_retires_converged_problems():
    probs = [(random_mask(sh, 0.3, 70 + i), kn) for i, (sh, kn) in
             enumerate([((30, 26), 0.5), ((26, 34), 3.0), ((22, 22), 1.0)])]
    b = poredvm.Batch(probs, [6, 6], precision="fp64", tile=(8, 8), schedule="queue")
    res = b.iterate(20000, 1e-9)
    assert all(r["converged"] for r in res)
    for i, (m, kn) in enumerate(probs):
        s = poredvm.Solver(m, [6, 6], kn, precision="fp64", tile=(8, 8), schedule="diagonals")
        r = s.iterate(20000, 1e-9)
        assert r["iters"] == res[i]["iters"] and r["k"] == res[i]["k"]
        s.close()


def test_queue_abandoned_sweep_keeps_state_and_poisons_the_solver():
    """A wait limit of 0 makes the queue's bounded waits give up (every block
    still ends): the iterate is discarded, the state stays the last completed
    iteration, and the solver refuses to iterate until a state is restored."""
    m = random_mask((40, 36, 44), 0.3, 81)
    s = poredvm.Solver(m, [8, 8, 8], 0.7, precision="fp32", tile=(4, 4, 4), schedule="queue")
    s.iterate(2)
    blob = s.get_state()
    before = s.moments(diagnostics=False)
    s.set_wait_limit(0.0)
    with pytest.raises(poredvm.PdvmError) as e:
        s.iterate(3)
    assert e.value.code == poredvm.PDVM_E_HIP and "discarded" in str(e.value)
    for x, y in zip(before, s.moments(diagnostics=False)):
        assert np.array_equal(x, y)
    s.set_wait_limit(2.0)
    with pytest.raises(poredvm.PdvmError) as e:
        s.iterate(1)
    assert e.value.code == poredvm.PDVM_E_STATE
    s.set_state(blob)
    s.iterate(3)
    ref = poredvm.Solver(m, [8, 8, 8], 0.7, precision="fp32", tile=(4, 4, 4), schedule="diagonals")
    ref.iterate(5)
    for x, y in zip(ref.moments(diagnostics=False), s.moments(diagnostics=False)):
        assert np.array_equal(x, y)


def test_autotuner_compares_the_3d_schedules(tmp_path, monkeypatch):
    """In 3D the tuner times tile queues, column queues and per-diagonal
    launches for every tile; its choice runs the same iterates as any other."""
    from paper_1712_01132_amd import autotune
    monkeypatch.setenv("PDVM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    m = random_mask((14, 12, 16), 0.3, 91)
    (sched, tile), ms = autotune.best_config(m, [4, 4, 4], "fp32", iters=2)
    assert sched in autotune.SCHEDULES_3D and tile in autotune.CANDIDATES_3D
    assert len(ms) == len(autotune.SCHEDULES_3D) * len(autotune.CANDIDATES_3D)
    assert all(v > 0 for v in ms.values())
    same(run(m, [4, 4, 4], 0.9, sched, 6, precision="fp32", tile=tile),
         run(m, [4, 4, 4], 0.9, "diagonals", 6, precision="fp32", tile=(4, 4, 4)))
