"""Fault path of the row-pipeline sweep, forced from the host.

A wait limit of 0 makes the sweep's bounded waits give up during the pipeline
fill (every kernel still runs to its end, on stale halo values): the iterate of
that sweep must be discarded, the state must stay the last completed iteration,
and the solver must refuse to iterate until a state is restored.
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


# 64 tile rows of 4x4 tiles (eight bands): the top band's first tile waits
# for dozens of tile steps, far longer than 128 polls
SHAPE = (256, 64)


def _solver(m):
    s = poredvm.Solver(m, [8, 8], 0.7, tile=(4, 4), schedule="rows")
    assert s.schedule.startswith("rows")
    return s


def test_abandoned_sweep_keeps_state_and_poisons_the_solver():
    m = random_mask(SHAPE, 0.3, 31)
    s = _solver(m)
    s.iterate(3)
    blob = s.get_state()
    before = s.moments()
    s.set_wait_limit(0.0)
    with pytest.raises(poredvm.PdvmError) as e:
        s.iterate(5)
    assert e.value.code == poredvm.PDVM_E_HIP
    assert "discarded" in str(e.value)
    # the state is the last completed iteration, bit for bit
    for x, y in zip(before, s.moments()):
        assert np.array_equal(x, y)
    # poisoned: no further iteration (nor timing) until a state is restored
    s.set_wait_limit(2.0)
    for call in (lambda: s.iterate(2), lambda: s.time_kernels(1)):
        with pytest.raises(poredvm.PdvmError) as e:
            call()
        assert e.value.code == poredvm.PDVM_E_STATE
    for x, y in zip(before, s.moments()):
        assert np.array_equal(x, y)
    # restoring the checkpoint clears it; the run continues as an undisturbed one
    s.set_state(blob)
    r = s.iterate(5)
    assert r["total_iters"] == 8
    ref = _solver(m)
    ref.iterate(8)
    for x, y in zip(ref.moments(), s.moments()):
        assert np.array_equal(x, y)


def test_set_initial_clears_the_poison():
    m = random_mask(SHAPE, 0.3, 32)
    s = _solver(m)
    s.set_wait_limit(0.0)
    with pytest.raises(poredvm.PdvmError) as e:
        s.iterate(4)
    assert e.value.code == poredvm.PDVM_E_HIP
    rho, u = s.moments(diagnostics=False)
    assert np.abs(u).max() == 0.0  # nothing was accepted: still the rest state
    s.set_wait_limit(2.0)
    s.set_initial()
    s.iterate(4)
    ref = _solver(m)
    ref.iterate(4)
    for x, y in zip(ref.moments(), s.moments()):
        assert np.array_equal(x, y)


def test_wait_limit_range_is_checked():
    m = random_mask((16, 16), 0.3, 33)
    s = poredvm.Solver(m, [4, 4], 0.5)
    for bad in (-1.0, float("nan"), 1e9):
        with pytest.raises(poredvm.PdvmError) as e:
            s.set_wait_limit(bad)
        assert e.value.code == poredvm.PDVM_E_INVAL
