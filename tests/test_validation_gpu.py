"""The paper's validation cases on the GPU (Sec. 4.1, Table 1; Sec. 4.2,
Table 3), with the paper's velocity grids and stop test (Err(l) < 1e-8).

* Simple-cubic sphere array (Table 3): the solver reproduces the printed
  permeabilities within 5 % (measured: +2.1 % at Kn = 0.1, +3.6 % at Kn = 1).
  The authors' code differs in details the paper does not fix (stencil order
  next to walls, corner points), so closer agreement is not expected.
* Sierpinski carpet (Table 1): the printed permeabilities are NOT reproduced.
  At the smallest Kn the solver is instead checked against the continuum
  permeability of the carpet as described, computed by an independent
  lattice-Boltzmann Stokes solve (tests/golden/carpet_stokes.json, written by
  tests/golden/make_carpet_stokes.py): the apparent permeability must exceed it
  by a slip excess of at most 20 %. The printed k_inf is 3.3 times below that
  continuum value.
"""
import json
import os

import pytest

from paper_1712_01132_amd import poredvm, validation

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "carpet_stokes.json")


def _k(mask, kn, nv, precision):
    s = poredvm.Solver(mask, nv, kn, precision=precision)
    try:
        st = s.iterate(20000, 1e-8, stop_mode="paper")
    finally:
        s.close()
    assert st["converged"]
    return st["k"]


@pytest.mark.parametrize("kn,precision", [(0.1, "fp64"), (1.0, "fp32")])
def test_sphere_array_matches_table3(kn, precision):
    k = _k(validation.spheres(), kn, validation.SPHERES_NV[kn], precision)
    assert abs(k / validation.SPHERES_TABLE3[kn] - 1) < 0.05, k


def test_carpet_small_kn_approaches_the_continuum_permeability():
    with open(GOLD) as f:
        k_inf = json.load(f)["carpet_540"]["k_over_L2"]
    k = _k(validation.carpet(), 0.001, validation.CARPET_NV[0.001], "fp64")
    assert 1.0 < k / k_inf < 1.2, (k, k_inf)


def test_carpet_kn_sweep_is_monotone():
    """Rarefaction raises the apparent permeability: k(0.01) < k(0.1) < k(1)."""
    c = validation.carpet()
    ks = [_k(c, kn, validation.CARPET_NV[kn], "fp64") for kn in (0.01, 0.1, 1.0)]
    assert ks[0] < ks[1] < ks[2], ks
