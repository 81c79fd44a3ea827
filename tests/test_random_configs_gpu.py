"""Seeded random configurations against the CPU oracle.

Each case draws a geometry (2D or 3D, random size and solid fraction), a
velocity grid (including octant sizes that leave the last 64-velocity group
partial), tile shape, schedule, precision, stencil rule, lateral faces and
the optional models (temperature feedback, Shakhov, Maxwell walls), within
what the library accepts, then compares a few iterations with the oracle at
the tolerances of the parity tests (1e-10 FP64, 1e-5 FP32). The draws are
fixed by the case index, so a failure names a reproducible configuration.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSolver
from paper_1712_01132_amd import geometry, poredvm

pytestmark = pytest.mark.gpu

RTOL = {"fp64": 1e-10, "fp32": 1e-5}


def draw(case):
    rng = np.random.default_rng(1000 + case)
    dim = 2 if case % 3 else 3
    if dim == 2:
        shape = tuple(int(x) for x in rng.integers(9, 48, size=2))
        nv = [int(2 * rng.integers(2, 13)) for _ in range(2)]
        tile = [int(rng.choice([1, 2, 3, 4, 5, 8])) for _ in range(2)]
    else:
        shape = tuple(int(x) for x in rng.integers(5, 13, size=3))
        nv = [int(2 * rng.integers(1, 5)) for _ in range(3)]
        tile = [int(rng.choice([2, 4, 8])) for _ in range(2)] + [int(rng.integers(1, 6))]
    rule = int(rng.integers(0, 2))
    tau = bool(rng.random() < 0.4)
    prandtl = float(rng.choice([0.5, 2.0 / 3.0])) if (tau and rng.random() < 0.5) else None
    alpha = float(rng.choice([0.4, 0.75])) if (rule == 1 and rng.random() < 0.35) else 1.0
    schedule = str(rng.choice(["auto", "rows", "diagonals"])) if dim == 2 else "auto"
    return {
        "shape": shape, "nv": nv, "tile": tile, "rule": rule, "tau": tau, "prandtl": prandtl, "alpha": alpha,
        "schedule": schedule,
        "precision": "fp32" if rng.random() < 0.35 else "fp64",
        "lateral": "periodic" if rng.random() < 0.3 else "specular",
        "kn": float(np.exp(rng.uniform(np.log(0.05), np.log(5.0)))),
        "frac": float(rng.uniform(0.1, 0.35)),
        "jump": float(rng.choice([1.0, -0.5, 2.0])),
        "seed": int(rng.integers(0, 1 << 30)),
    }


def mask_of(c):
    rng = np.random.default_rng(c["seed"])
    while True:
        m = geometry.fill_nonpercolating((rng.random(c["shape"]) < c["frac"]).astype(np.uint8))
        if geometry.percolates(m) and 0 < m.sum() < m.size - 4:
            return m


@pytest.mark.parametrize("case", range(64))
def test_random_configuration_matches_oracle(case):
    c = draw(case)
    print("case", case, c, flush=True)
    m = mask_of(c)
    o = OracleSolver(m, c["nv"], c["kn"], jump=c["jump"], lateral_periodic=c["lateral"] == "periodic",
                     tau_feedback=c["tau"], threads=16, stencil_rule=c["rule"], prandtl=c["prandtl"],
                     accommodation=c["alpha"])
    s = poredvm.Solver(m, c["nv"], c["kn"], jump=c["jump"], precision=c["precision"], lateral=c["lateral"],
                       tau_feedback=c["tau"], tile=c["tile"], grid=o.grid, stencil_rule=c["rule"],
                       schedule=c["schedule"], prandtl=c["prandtl"], accommodation=c["alpha"])
    try:
        o.iterate(6)
        s.iterate(6)
        ro, uo, to, qo = o.moments()
        rg, ug, tg, qg = s.moments()
        rtol = RTOL[c["precision"]]
        su = np.abs(uo).max()
        scale = max(su, np.abs(ro).max())
        assert np.abs(ug - uo).max() <= rtol * su, (case, np.abs(ug - uo).max() / su)
        assert np.abs(rg - ro).max() <= rtol * scale
        assert np.abs(tg - to).max() <= rtol * max(np.abs(to).max(), scale)
        assert np.abs(qg - qo).max() <= rtol * max(np.abs(qo).max(), scale)
        _, ko, _ = o.flux()
        _, kg, _ = s.flux()
        assert abs(kg - ko) <= rtol * abs(ko)
    finally:
        s.close()
