"""The temperature term fed back in 2D (oracle, CPU).

In 2D the distribution is integrated over v3. The isothermal equation only
needs the reduced function phi = int h exp(-v3^2)/sqrt(pi) dv3; with the
temperature fed back the source tau (|v|^2 - 3/2) also needs the second one,
psi = int (v3^2 - 1/2) h exp(-v3^2)/sqrt(pi) dv3 (Sec. 2, Eq.
linearised_Boltzmann_equation, reduced over v3). The pin: a 2D geometry
extruded to two identical layers along x3, with specular x3 faces and a
six-node v3 grid, is the same physical problem, so at convergence it has the
same rho, u, tau and q as the native (phi, psi) solve. The 3D oracle has no
reduction, so a dropped psi term, a wrong psi source or the 3D factor
|v|^2 - 3/2 in place of v1^2 + v2^2 - 1 in 2D all break the agreement.

The geometries are symmetric about the mid-plane across x1: the lagged
boundary values then leave no drift along the density null space, which the
two iterations (they differ in their x3 lag) would otherwise take
differently.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSolver
from paper_1712_01132_amd import geometry


def _disc_in_rectangle(n1, n2, r):
    c1 = np.arange(n1) + 0.5 - n1 / 2.0
    c2 = np.arange(n2) + 0.5 - n2 / 2.0
    return (c1[None, :] ** 2 + c2[:, None] ** 2 <= r * r).astype(np.uint8)


CASES = [
    (geometry.centred_disc(12, 3.0), 0.5),
    (_disc_in_rectangle(14, 10, 3.2), 0.15),
]


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("tau,pr,alpha", [(False, None, 1.0), (True, None, 1.0), (True, 2.0 / 3.0, 1.0),
                                          (False, None, 0.6), (True, None, 0.6)])
def test_2d_psi_equals_two_layer_extrusion(case, tau, pr, alpha):
    """pr: the Shakhov model, whose heat-flux source reduces to
    (4/5)(1 - Pr) q.v (v1^2 + v2^2 - 2) for phi and (2/5)(1 - Pr) q.v for psi.
    alpha < 1: Maxwell walls, whose specular part reflects psi as well (the
    extruded solid has no walls normal to x3)."""
    m, kn = CASES[case]
    nv = [8, 8]
    a = OracleSolver(m, nv, kn, tau_feedback=tau, threads=4, prandtl=pr, accommodation=alpha)
    b = OracleSolver(np.stack([m, m]), nv + [6], kn, tau_feedback=tau, threads=8, prandtl=pr,
                     accommodation=alpha)
    ra = a.iterate(40000, 1e-13)
    rb = b.iterate(40000, 1e-13)
    assert ra["converged"] and rb["converged"]
    rho, u, t, q = a.moments()
    rho3, u3, t3, q3 = b.moments()
    scale = np.abs(u).max()
    tol = 1e-10 * scale
    # the two layers agree and carry no flow along x3
    assert np.abs(u3[:, 0] - u3[:, 1]).max() <= tol
    assert np.abs(u3[2]).max() <= tol
    assert np.abs(rho - rho3[0]).max() <= tol
    assert np.abs(u - u3[:2, 0]).max() <= tol
    assert np.abs(t - t3[0]).max() <= tol
    assert np.abs(q - q3[:2, 0]).max() <= tol
    if tau:
        # the feedback (and the Shakhov term) matters at this tolerance
        ref = OracleSolver(m, nv, kn, tau_feedback=pr is not None, threads=4, accommodation=alpha)
        ref.iterate(40000, 1e-13)
        _, _, ti, qi = ref.moments()
        assert np.abs(t - ti).max() > 1e3 * tol
        assert np.abs(q - qi).max() > 1e3 * tol
