"""Batched problems: each problem of a batch evolves exactly as it does alone
(same kernels, same arithmetic per problem), and problems that converge
retire while the others continue."""
import numpy as np
import pytest

from paper_1712_01132_amd import geometry, poredvm

pytestmark = pytest.mark.gpu


def masks():
    out = []
    for seed, (n1, n2), kn in [(1, (40, 32), 0.2), (2, (24, 56), 2.0), (3, (64, 64), 0.7), (4, (17, 13), 5.0)]:
        rng = np.random.default_rng(seed)
        while True:
            m = geometry.fill_nonpercolating((rng.random((n2, n1)) < 0.3).astype(np.uint8))
            if geometry.percolates(m):
                break
        out.append((m, kn))
    return out


@pytest.mark.parametrize("precision,tile", [("fp64", (8, 8)), ("fp32", (4, 4))])
def test_batch_matches_single_problems_bitwise(precision, tile):
    probs = masks()
    b = poredvm.Batch(probs, [8, 8], precision=precision, tile=tile)
    rb = b.iterate(12)
    assert all(r["iters"] == 12 for r in rb)
    for i, (m, kn) in enumerate(probs):
        s = poredvm.Solver(m, [8, 8], kn, precision=precision, tile=tile)
        rs = s.iterate(12)
        rho_s, u_s = s.moments(diagnostics=False)
        rho_b, u_b = b.moments(i)
        assert np.array_equal(rho_s, rho_b) and np.array_equal(u_s, u_b)
        assert rs["k"] == rb[i]["k"]
        assert b.flux(i)[1] == s.flux()[1]
        s.close()


def test_batch_retires_converged_problems():
    probs = masks()
    b = poredvm.Batch(probs, [6, 6], precision="fp64", tile=(8, 8))
    res = b.iterate(20000, 1e-9)
    assert all(r["converged"] for r in res)
    iters = [r["iters"] for r in res]
    assert len(set(iters)) > 1  # the problems converge at different iterations
    snap = [b.moments(i) for i in range(len(probs))]
    res2 = b.iterate(50, 1e-9)  # everything already met the tolerance: one more iteration each at most
    for i in range(len(probs)):
        s = poredvm.Solver(probs[i][0], [6, 6], probs[i][1], precision="fp64", tile=(8, 8))
        r = s.iterate(20000, 1e-9)
        assert r["iters"] == iters[i]
        s.close()
    assert all(r["converged"] for r in res2)


def test_batch_rejects_mixed_velocity_grids():
    probs = masks()[:2]
    g1 = [poredvm.velocity_grid(8)] * 2
    cfg0, k0 = poredvm.make_config(probs[0][0], [8, 8], 1.0, grid=g1)
    cfg1, k1 = poredvm.make_config(probs[1][0], [6, 6], 1.0)
    arr = (poredvm.PdvmConfig * 2)(cfg0, cfg1)
    import ctypes
    h = ctypes.c_void_p()
    rc = poredvm.load().pdvm_batch_create(2, arr, None, ctypes.byref(h))
    assert rc == poredvm.PDVM_E_INVAL
    assert "velocity grid" in poredvm._err()


def test_autotuner_times_candidates_and_caches(tmp_path, monkeypatch):
    from paper_1712_01132_amd import autotune
    monkeypatch.setenv("PDVM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    m = geometry.random_discs(64, 48, 0.5, 3.0, 6.0, seed=3)
    tile, ms = autotune.best_tile(m, [8, 8], "fp32", iters=2)
    assert tile in autotune.CANDIDATES_2D and len(ms) == len(autotune.CANDIDATES_2D)
    assert all(v > 0 for v in ms.values())
    again, _ = autotune.best_tile(m, [8, 8], "fp32", iters=2)  # from the cache
    assert again == tile
    # the chosen tile runs the same iteration as any other tile (bitwise)
    res = []
    for t in (tile, (4, 4)):
        s = poredvm.Solver(m, [8, 8], 0.5, precision="fp32", tile=list(t))
        s.iterate(5)
        res.append(s.moments(diagnostics=False))
        s.close()
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("nv,precision", [([6, 6], "fp64"), ([24, 24], "fp32"), ([32, 32], "fp64")])
def test_batch_strips_equal_tile_diagonals_bitwise(nv, precision):
    """All problems of a batch in one strip-pipeline launch against the
    per-diagonal launches."""
    probs = masks()
    res = []
    for sched in ("strips", "diagonals"):
        b = poredvm.Batch(probs, nv, precision=precision, schedule=sched)
        assert b.schedule == sched
        b.iterate(9)
        res.append([b.moments(i) for i in range(len(probs))])
        b.close()
    for (ra, ua), (rb, ub) in zip(res[0], res[1]):
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub)


@pytest.mark.parametrize("nv,precision", [([6, 6], "fp64"), ([24, 24], "fp32")])
def test_batch_row_pipeline_equals_tile_diagonals_bitwise(nv, precision):
    """All problems of a batch in one row-pipeline launch (each problem's
    blocks padded to multiples of 8) against the per-diagonal launches."""
    probs = masks()
    res = []
    for sched in ("rows", "diagonals"):
        b = poredvm.Batch(probs, nv, precision=precision, tile=[8, 8], schedule=sched)
        assert b.schedule.startswith(sched[:4])
        b.iterate(9)
        res.append([b.moments(i) for i in range(len(probs))])
        b.close()
    for (ra, ua), (rb, ub) in zip(res[0], res[1]):
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub)


def test_autotuner_tunes_schedule_and_tile_for_a_batch(tmp_path, monkeypatch):
    """For a batch the tuner times both one-launch queues and per-diagonal
    launches for every tile; its choice runs the same iterates as any other."""
    from paper_1712_01132_amd import autotune
    monkeypatch.setenv("PDVM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    probs = masks()
    (sched, tile), ms = autotune.best_config(probs, [8, 8], "fp32", iters=2)
    assert sched in autotune.SCHEDULES_MULTI and tile in autotune.CANDIDATES_2D
    assert len(ms) == len(autotune.SCHEDULES_MULTI) * len(autotune.CANDIDATES_2D)
    assert autotune.best_config(probs, [8, 8], "fp32", iters=2)[0] == (sched, tile)  # cached
    out = []
    for sc, t in ((sched, tile), ("diagonals", (4, 4))):
        b = poredvm.Batch(probs, [8, 8], precision="fp32", tile=list(t), schedule=sc)
        b.iterate(6)
        out.append([b.moments(i) for i in range(len(probs))])
        b.close()
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
