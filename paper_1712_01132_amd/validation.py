"""The effective Knudsen number and the Kn-sweep workflow (Sec. 2.1,
Eq. effective_Kn), and the paper's validation cases (Sec. 4.1, Table 1;
Sec. 4.2, Table 3).

The average pore size L* follows from the intrinsic permeability k_inf
(normalised by L^2) and the porosity eps: L*/L = sqrt(12 k_inf / eps) in 2D,
sqrt(8 k_inf / (pi eps)) in 3D, and Kn* = Kn / (L*/L). The paper takes as k_inf
the permeability at the smallest Knudsen number of a sweep, where the flow is
in the continuum regime; `kn_sweep` does the same with the GPU solver.
"""
import math

import numpy as np

from . import geometry, poredvm

# Permeabilities the paper prints (k normalised by L^2), keyed by Kn, with the
# velocity grids it used.
CARPET_TABLE1 = {0.001: 4.930e-5, 0.01: 1.355e-4, 0.1: 1.143e-3, 1.0: 1.490e-2}
CARPET_NV = {0.001: [8, 8], 0.01: [8, 8], 0.1: [8, 8], 1.0: [24, 24]}
SPHERES_TABLE3 = {0.01: 1.722e-2, 0.1: 3.862e-2, 1.0: 2.836e-1, 10.0: 3.375}
SPHERES_NV = {0.01: [8, 8, 8], 0.1: [8, 8, 8], 1.0: [16, 16, 16], 10.0: [16, 16, 16]}


def pore_size(k_inf, porosity, dim):
    """L*/L of Eq. effective_Kn."""
    if dim == 2:
        return math.sqrt(12.0 * k_inf / porosity)
    return math.sqrt(8.0 * k_inf / (math.pi * porosity))


def effective_kn_factor(k_inf, porosity, dim):
    """Kn* / Kn = 1 / (L*/L)."""
    return 1.0 / pore_size(k_inf, porosity, dim)


def kn_sweep(mask, kns, nv_of, precision="fp64", tol=1e-8, max_iters=400000, **solver_args):
    """Run the GPU solver at each Kn (paper stop mode: Err(l) < tol), take the
    smallest Kn's k as k_inf, and return the rows
    {kn, kn_star, k, k_over_kinf, iters, converged} and k_inf."""
    mask = np.asarray(mask)
    porosity = float(1.0 - mask.mean())
    rows = []
    for kn in sorted(kns):
        s = poredvm.Solver(mask, nv_of(kn), kn, precision=precision, **solver_args)
        try:
            st = s.iterate(max_iters, tol, stop_mode="paper")
        finally:
            s.close()
        rows.append({"kn": kn, "k": st["k"], "iters": st["total_iters"], "converged": st["converged"]})
    k_inf = rows[0]["k"]
    f = effective_kn_factor(k_inf, porosity, mask.ndim)
    for r in rows:
        r["kn_star"] = r["kn"] * f
        r["k_over_kinf"] = r["k"] / k_inf
    return rows, k_inf


def carpet(n=540):
    """The level-3 Sierpinski carpet of Sec. 4.1."""
    return geometry.sierpinski_carpet(3, n)


def spheres(n1=200):
    """The quadrant of the simple-cubic sphere array of Sec. 4.2."""
    return geometry.cubic_sphere_quadrant(n1, n1 // 2, n1 // 2, 0.75)
