"""Continuum (Stokes) permeability of a 2D voxel geometry by the lattice
Boltzmann method.

TEST INFRASTRUCTURE ONLY, and independent of both the kinetic oracle and the
GPU path: a different method for a different equation. It checks the small-Kn
end of the kinetic solver, where the apparent permeability k of the linearised
BGK solution tends to the intrinsic (Darcy) permeability k_inf of the
geometry. The paper uses that limit in Eq. effective_Kn (Sec. 2.1) and prints
k_inf for its Sierpinski carpet (Sec. 4.1, Table 1).

Method: D2Q9 lattice, BGK collision with relaxation time tau (lattice
viscosity (tau - 1/2) / 3), a uniform body force g along x1 entered with Guo's
forcing term, periodic in both directions, full-way bounce-back at solid
nodes (the wall lies half-way between a solid and a fluid node, i.e. on the
voxel face). At steady state Darcy's law gives k = nu <u1> / g, with <u1> the
mean over all nodes (solid nodes count as 0), in pixel^2. Divide by L^2
(L = N1 pixels) for the paper's normalisation. The force is small, so the
flow is in the Stokes regime.

Lateral faces: the kinetic solver mirrors them. A geometry that is symmetric
about its mid-plane in x2 gives the same flow with mirrored or periodic faces,
so the periodic box used here serves for such geometries (the carpet is one).

Plain PyTorch CPU tensor operations.
"""
import numpy as np
import torch

_E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
_W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
_OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def stokes_permeability(solid, tau=1.0, g=1e-6, check=1000, rtol=1e-7, max_steps=1_000_000, threads=None):
    """Darcy permeability (pixel^2) of a 2D mask (1 = solid, shape (N2, N1),
    x1 fastest) for flow along x1, and the number of steps taken. Stops when
    the mean velocity changes by less than rtol (relative) over `check` steps."""
    if threads:
        torch.set_num_threads(int(threads))
    solid = np.asarray(solid)
    ny, nx = solid.shape
    sol = torch.from_numpy(solid.astype(bool))
    fl = (~sol).to(torch.float64)
    ex = torch.tensor([e[0] for e in _E], dtype=torch.float64)[:, None, None]
    ey = torch.tensor([e[1] for e in _E], dtype=torch.float64)[:, None, None]
    w = torch.tensor(_W, dtype=torch.float64)[:, None, None]
    f = w.expand(9, ny, nx).clone()
    nu = (tau - 0.5) / 3.0
    prev = None
    q = 0.0
    for step in range(1, max_steps + 1):
        rho = f.sum(0)
        ux = ((f * ex).sum(0) + 0.5 * g) / rho
        uy = (f * ey).sum(0) / rho
        eu = ex * ux + ey * uy
        feq = w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
        force = (1.0 - 0.5 / tau) * w * (3.0 * (ex - ux) + 9.0 * eu * ex) * g
        post = f - (f - feq) / tau + force
        post = torch.where(sol[None], f[_OPP], post)  # solid nodes send back what reached them
        for i, (cx, cy) in enumerate(_E):
            f[i] = torch.roll(post[i], shifts=(cy, cx), dims=(0, 1))
        if step % check == 0:
            rho = f.sum(0)
            ux = ((f * ex).sum(0) + 0.5 * g) / rho
            q = float((ux * fl).sum()) / (nx * ny)
            if prev is not None and abs(q - prev) <= rtol * abs(q):
                return nu * q / g, step
            prev = q
    return nu * q / g, max_steps
