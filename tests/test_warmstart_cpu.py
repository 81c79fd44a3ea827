"""Host-side parts of the warm-start training: the mirror images used to
augment the training set are solutions of the mirrored problems. This is pinned
against the CPU oracle's iteration on the mirrored geometries."""
import numpy as np
import pytest

from oracle.oracle import OracleSolver
from paper_1712_01132_amd import geometry
from paper_1712_01132_amd.train_warmstart import mirrored


def _solve(mask):
    o = OracleSolver(mask, [6, 6], 0.5, threads=4)
    st = o.iterate(20000, 1e-13)
    assert st["converged"]
    rho, u = o.moments()[:2]
    o.close()
    return rho, u


@pytest.mark.parametrize("fx1,fx2", [(True, False), (False, True), (True, True)])
def test_mirrored_solution_solves_the_mirrored_problem(fx1, fx2):
    rng = np.random.default_rng(11)
    while True:
        m = geometry.fill_nonpercolating((rng.random((12, 16)) < 0.3).astype(np.uint8))
        if geometry.percolates(m):
            break
    rho, u = _solve(m)
    mm, rr, uu = mirrored(m, rho, u, flip_x1=fx1, flip_x2=fx2)
    rho2, u2 = _solve(mm)
    fl = mm == 0
    scale = np.abs(u2).max()
    assert np.max(np.abs(uu - u2)) <= 1e-9 * scale
    d = (rr - rho2)[fl]
    assert np.max(np.abs(d - d.mean())) <= 1e-9 * np.abs(rho2[fl]).max()
