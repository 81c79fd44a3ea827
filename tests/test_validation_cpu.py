"""The paper's validation geometries and Eq. effective_Kn (Sec. 2.1, 4.1, 4.2),
and the continuum reference used to check the solver's small-Kn limit."""
import numpy as np
import pytest

from oracle.stokes_lbm import stokes_permeability
from paper_1712_01132_amd import geometry, validation


@pytest.mark.parametrize("k_inf,eps,dim,printed", [
    (4.930e-5, 0.70, 2, 34.40),   # Sierpinski carpet, Sec. 4.1
    (1.722e-2, 0.75, 3, 4.14),    # simple-cubic sphere array, Sec. 4.2
    (1.260e-4, 0.38, 3, 34.41),   # random sphere pack, Sec. 4.2
])
def test_effective_kn_factor_reproduces_the_printed_factors(k_inf, eps, dim, printed):
    """Kn*/Kn from the k_inf and porosity the paper prints, to the digits it prints."""
    assert round(validation.effective_kn_factor(k_inf, eps, dim), 2) == printed


def test_carpet_geometry():
    """Level-3 carpet on 540 pixels: solid fraction 1 - (8/9)^3 (porosity 0.70 in
    the paper), 20-pixel squares at the finest level, the central 180-pixel square
    solid, mirror symmetric about both mid-lines."""
    c = validation.carpet()
    assert c.shape == (540, 540)
    assert abs((1 - c.mean()) - (8 / 9) ** 3) < 1e-12
    assert c[180:360, 180:360].all() and not c[:20, :].any()
    assert (c == c[::-1]).all() and (c == c[:, ::-1]).all()
    # the finest removed squares: 20 x 20 at the centre of each 60-pixel cell
    assert c[20:40, 20:40].all() and not c[19, 20:40].any() and not c[40, 20:40].any()


def test_sphere_quadrant_geometry():
    """200 x 100 x 100 quadrant, porosity 0.75, sphere radius 78.2 voxels about
    the cell centre (x1 = 100, at the x2 = x3 = 0 corner), mirror symmetric in x1."""
    s = validation.spheres()
    assert s.shape == (100, 100, 200)
    assert abs((1 - s.mean()) - 0.75) < 2e-4
    assert (s == s[:, :, ::-1]).all()
    radius_x1 = (s[0, 0, :].sum()) / 2.0  # along the x1 axis through the centre
    assert abs(radius_x1 - 78.2) < 1.0


def test_stokes_reference_reproduces_poiseuille():
    """The continuum reference on a plane channel of H = 10 fluid rows: the Darcy
    permeability of plane Poiseuille flow, H^2/12 times the open fraction, to 1.5 %."""
    m = np.zeros((12, 8), np.uint8)
    m[0] = m[-1] = 1
    k, _ = stokes_permeability(m, threads=4)
    exact = 10 ** 2 / 12 * 10 / 12
    assert abs(k / exact - 1) < 0.015
