"""Host-side checks of libporedvm that need no GPU: the shared library loads
and exports every entry point include/poredvm.h declares, the library's own
quadrature matches the oracle's and the Gauss exactness conditions, and
invalid configurations are rejected before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import quadrature
from paper_1712_01132_amd import geometry, poredvm, warmstart

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdvm_[a-z_]+)\s*\(", text)))


@pytest.mark.parametrize("header,exported", [("poredvm.h", poredvm.EXPORTED),
                                             ("poredvm_unet.h", warmstart.EXPORTED)])
def test_library_exports_every_declared_symbol(header, exported):
    lib = poredvm.load()
    declared = _declared_symbols(header)
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(declared) == sorted(exported)


def test_network_parameter_count_matches_layer_table():
    n = sum(c * t * i + c for _, c, t, i in warmstart.LAYERS)
    assert warmstart.num_params() == n
    p = warmstart.init_params(0)
    assert p.shape == (n,) and p.dtype == np.float32
    assert all(w.shape == (c, t, i) for (w, b), (_, c, t, i) in zip(warmstart.split_params(p), warmstart.LAYERS))


def test_network_rejects_bad_shapes_without_a_device():
    lib = warmstart._lib()
    h = ctypes.c_void_p()
    assert lib.pdvm_unet_create(30, 32, 4, 0, None, ctypes.byref(h)) == poredvm.PDVM_E_INVAL
    assert lib.pdvm_unet_create(32, 32, 64, 0, None, ctypes.byref(h)) == poredvm.PDVM_E_INVAL
    assert b"multiples of 8" in lib.pdvm_unet_last_error(None)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 24, 32, 48, 64])
def test_library_quadrature_matches_oracle_and_is_gauss(n):
    x, w = poredvm.velocity_grid(n)
    xo, wo = quadrature.full_line_grid(n)
    assert np.max(np.abs(x - xo)) <= 2e-16 * np.abs(xo).max()
    assert np.max(np.abs(w - wo) / wo) <= 1e-14
    pos = x > 0
    for m in range(n):  # half-range rule with n/2 nodes: exact to degree n - 1
        exact = math.gamma((m + 1) / 2) / 2 / math.sqrt(math.pi)
        assert abs(np.sum(w[pos] * x[pos] ** m) - exact) <= 1e-13 * exact


def test_library_quadrature_rejects_bad_sizes():
    for n in (0, 1, 3, 66):
        with pytest.raises(poredvm.PdvmError):
            poredvm.velocity_grid(n)


def _bytes(cfg):
    return poredvm.load().pdvm_workspace_bytes(ctypes.byref(cfg))


def test_workspace_bytes_for_valid_config():
    cfg, keep = poredvm.make_config(geometry.centred_disc(64), [16, 16], 1.0)
    assert _bytes(cfg) > 64 * 64 * 256 * 8 * 2


@pytest.mark.parametrize("case,needle", [
    ("no_fluid", "no fluid"),
    ("no_path", "winds"),
    ("odd_nv", "even"),
    ("asym", "symmetric"),
    ("kn0", "kn"),
    ("wsum", "sum"),
    ("tau2d_wide", "psi"),
    ("shakhov_no_tau", "tau_feedback"),
    ("prandtl_neg", "prandtl"),
    ("maxwell_rule0", "stencil_rule 1"),
    ("maxwell_alpha0", "specular_fraction"),
    ("zero_node", "ascending"),
    ("columns_2d", "3D only"),
])
def test_invalid_configs_rejected(case, needle):
    m = geometry.centred_disc(16)
    nv = [4, 4]
    kw = {}
    grid = None
    if case == "no_fluid":
        m = np.ones((8, 8), np.uint8)
    elif case == "no_path":
        m = np.zeros((8, 8), np.uint8)
        m[:, 3] = 1  # a solid wall across the flow axis
    elif case == "odd_nv":
        x, w = quadrature.full_line_grid(4)
        grid = [(np.array([-1.0, 0.5, 1.0]), np.array([0.3, 0.4, 0.3]))] * 2
    elif case == "asym":
        x, w = quadrature.full_line_grid(4)
        x = x.copy()
        x[0] *= 1.1
        grid = [(x, w)] * 2
    elif case == "kn0":
        kw["kn"] = 0.0
    elif case == "wsum":
        x, w = quadrature.full_line_grid(4)
        grid = [(x, w * 1.001)] * 2
    elif case == "shakhov_no_tau":
        kw["prandtl"] = 2.0 / 3.0
    elif case == "prandtl_neg":
        kw.update(prandtl=-0.5, tau_feedback=True)
    elif case == "maxwell_rule0":
        kw.update(accommodation=0.5, stencil_rule=0)
    elif case == "maxwell_alpha0":
        kw.update(accommodation=0.0)
    elif case == "tau2d_wide":
        kw["tau_feedback"] = True  # psi doubles the 576 velocities of an octant: over 1024
        nv = [48, 48]
    elif case == "columns_2d":
        kw["schedule"] = "columns"
    elif case == "zero_node":
        grid = [(np.array([-1.0, -0.0, 0.0, 1.0]), np.array([0.25, 0.25, 0.25, 0.25]))] * 2
    kn = kw.pop("kn", 1.0)
    cfg, keep = poredvm.make_config(m, nv, kn, grid=grid, **kw)
    assert _bytes(cfg) == 0
    assert needle in poredvm._err()
